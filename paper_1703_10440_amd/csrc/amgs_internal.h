// amgs_internal.h -- launch contexts and kernel argument blocks (host and
// device side of the library; not part of the public ABI).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace amgs {

enum { VAR_NAIVE = 0, VAR_HA = 1, VAR_HP = 2 };
enum { SRC_UPD = 0, SRC_VEC = 1, SRC_DIV = 2 };
constexpr int MAX_CPW = 256;   // trailing columns per sweep workgroup (max)
constexpr int SWEEP_TARGET_WG = 1024; // sweep workgroups aimed for
constexpr int SWEEP_CB = 4;    // later columns streamed together by one sweep thread
constexpr double SWEEP_NT_BYTES = 192.0 * (1 << 20); // trailing block streamed non-temporally above this
constexpr int HP_XB = 8;       // HP recurrence terms applied per blocked update
constexpr int RE_GROUP = 8;    // second-pass coefficients per workgroup row
constexpr int DENSE_CB = 16;   // outputs per dense-MV workgroup pass
constexpr int SPMM_C = 8;      // columns per CSR block-product thread
constexpr int MAX_G_MV = 512;  // partials of an MV column kernel
constexpr int STREAM_CAP = 4096; // CSR entries staged per 512-row tile

// Partials of the projection sweep: part[c * g + w] holds workgroup w's part
// of r_{j,c} (element type of the storage precision).
struct SweepPart {
    void *part;
    int64_t g;
};

struct Geo {
    int U;          // rows per thread of the sweep (1,2,4,8)
    int64_t g_rows; // sweep row chunks of 256*U rows
    int U2;         // rows per thread of the column / second-pass kernels (<= 4)
    int64_t g_rows2;// their row chunks of 256*U2 rows
    int64_t g_rows1;// 256-row chunks (one row per thread)
    int lanes;      // lanes per CSR row in the MV kernel (0: 512-row tiles staged in LDS)
    int64_t g_csr;  // workgroups of the CSR MV kernel
    int64_t g_dense;// workgroups of the dense MV kernel
};

struct CsrMvArgs {
    int64_t m, n, j;
    const int32_t *row_ptr, *col_idx;
    const void *vals;
    const void *src, *qprev;
    void *y, *zt;
    double *R;
    int64_t ldr;
    const int32_t *info;
    SweepPart sp;
    const double *rr_part;
    int64_t n_rr;
    double *rr_out;
};

struct DenseMvArgs {
    int64_t m, n, j;
    const void *A;
    int64_t lda;
    const void *src, *qprev;
    void *y, *zt;
    double *R;
    int64_t ldr;
    const int32_t *info;
    SweepPart sp;
    const double *rr_part;
    int64_t n_rr;
    double *rr_out;
};

struct RowArgs {
    int64_t m, n, j;
    void *Q;
    int64_t ldq;
    void *P;
    int64_t ldp;
    void *X;
    int64_t ldx;
    void *zt;
    double *R;
    int64_t ldr;
    const int32_t *info;
    SweepPart sp;
    double *rr_out;
    double *s_part;
    const double *S;
};

struct SweepArgs {
    int64_t m, n, j;
    void *Q;
    int64_t ldq;
    void *P;
    int64_t ldp;
    const void *X;
    int64_t ldx;
    const void *zt, *xv;
    double *R;
    int64_t ldr;
    int32_t *info;
    SweepPart sp;
    const double *rr_part;
    int64_t n_rr;
    int64_t cpw;
};

// Everything one amgs_qr_* call needs on the host side.
struct Ctx {
    int64_t m, n;
    int is_dense;
    // A
    const void *A;
    int64_t lda;
    const int32_t *row_ptr, *col_idx;
    const void *vals;
    int64_t nnz;
    // matrices
    const void *Z;
    int64_t ldz;
    void *Q;
    int64_t ldq;
    double *R;
    int64_t ldr;
    void *P;
    int64_t ldp;
    void *X;      // HP block, ld = m
    void *zt, *xv;
    // reductions
    SweepPart sp;
    double *rr_part;
    int64_t n_rr_mv;  // partial count of the MV column kernel
    double *s_part;
    double *S;
    int32_t *info;
    Geo geo;
    hipStream_t stream;
    // when set, the sweep is launched with these events bound to its own
    // dispatch (exact kernel start and end, no extra stream markers)
    hipEvent_t ev_start, ev_stop;
};

Geo make_geo(int64_t m, int64_t nnz, int is_dense);

template <typename T> void launch_init(const Ctx &c, int copy);
template <typename T> void launch_mv(const Ctx &c, int64_t j, int src_mode);
template <typename T> void launch_col_hp(const Ctx &c, int64_t j, bool reorth_a);
template <typename T> void launch_reorth_a(const Ctx &c, int64_t j);
void launch_reorth_fin(const Ctx &c, int64_t j);
template <typename T> void launch_reorth_b(const Ctx &c, int64_t j, bool hp);
template <typename T> void launch_sweep(const Ctx &c, int64_t j, int variant, int64_t n_rr);
template <typename T> bool launch_hp_xblock(const Ctx &c, int64_t s);
template <typename T> void launch_csr_spmm(const Ctx &c);
template <typename T> void launch_dense_gemm(const Ctx &c);
void launch_csr_check(int64_t m, int64_t nnz, const int32_t *row_ptr, const int32_t *col_idx,
                      int32_t *flag, hipStream_t s);

} // namespace amgs
