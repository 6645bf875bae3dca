// amgs_batched.hip -- placeholder until the batched persistent solver lands.
#include <hip/hip_runtime.h>
#include "../../include/amgs.h"
#include "amgs_batched.h"

extern "C" {
amgs_status_t amgs_batch_plan_create(amgs_handle_t, int32_t, const int64_t *, const int64_t *,
                                     amgs_variant_t, amgs_precision_t, const amgs_opts_t *,
                                     int32_t, amgs_batch_plan_t *plan)
{
    if (plan) *plan = nullptr;
    return AMGS_ERR_UNSUPPORTED;
}
amgs_status_t amgs_batch_plan_destroy(amgs_batch_plan_t) { return AMGS_ERR_UNSUPPORTED; }
size_t amgs_batch_workspace_bytes(amgs_batch_plan_t) { return 0; }
amgs_status_t amgs_qr_batched(amgs_batch_plan_t, const amgs_batch_desc_t *, void *, size_t,
                              int32_t *, void *)
{
    return AMGS_ERR_UNSUPPORTED;
}
int32_t amgs_batch_plan_tiles(amgs_batch_plan_t, int32_t *, int32_t) { return 0; }
}
