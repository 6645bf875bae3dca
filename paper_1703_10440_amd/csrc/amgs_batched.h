// amgs_batched.h -- batched persistent solver (internal interface).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/amgs.h"

namespace amgs {

constexpr int BT_NT = 512;          // threads per instance workgroup
constexpr int BT_RPT = 8;           // rows per thread: m <= BT_NT * BT_RPT
constexpr int BT_MAX_M = BT_NT * BT_RPT;
constexpr int BT_MAX_N = 256;       // largest n of an instance
constexpr int BT_RED = 8;           // values per workgroup reduction
constexpr int BT_NCLASS = 8;        // size classes: 4 ranges of m x (n <= 16, n > 16)
constexpr int BT_TILE_HA = 8;       // widest column block (registers): naive / HA
constexpr int BT_TILE_HP = 4;       // HP keeps z and x blocks
constexpr int BT_TUNE_MAX = 1024;   // instances in the autotuner's sample of the batch
constexpr int BT_TUNE_REPS = 5;     // timed passes per candidate (best taken)
constexpr float BT_TUNE_GAIN = 0.02f; // a width is taken only if the pass gets this much faster

// One entry of the device work list, in largest-first order.
struct BatchItem {
    int32_t k;       // index into the descriptor / info arrays
    int32_t B;       // columns per block (tile) for this instance
    int64_t ws;      // element offset of the instance's P (and X) in the workspace
};

inline int size_class(int64_t m, int64_t n)
{
    const int mc = m <= 512 ? 0 : m <= 1024 ? 1 : m <= 2048 ? 2 : 3;
    return mc * 2 + (n > 16 ? 1 : 0);
}

// Enqueue one pass over the work list (queue reset + persistent kernel).
void launch_batched(int precision, int variant, int bmax, int reorth, int grid,
                    const amgs_batch_desc_t *desc, const BatchItem *items, int32_t count,
                    void *work, int32_t *info, uint32_t *counter, hipStream_t s);
// Workgroups of the persistent kernel that fit on the device at once.
int batched_resident_wgs(int device, int precision, int variant, int bmax);

} // namespace amgs
