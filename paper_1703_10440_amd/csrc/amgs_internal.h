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
constexpr int SPMM_C = 4;      // columns per CSR block-product load group
constexpr int SPMM_LC = 8;     // columns per pass of the multi-lane CSR block product
constexpr int MAX_G_MV = 512;  // partials of an MV column kernel
constexpr int MV_TILE = 512;   // rows (= threads) per padded-copy MV workgroup
constexpr int ELL_K = 8;       // most entries per row held in the padded copy of A
constexpr int16_t ELL_PAD = -32768;   // 16-bit column offset of a padding entry
constexpr int PANEL_B = 4;     // columns per panel of the panel schedule (inner panels of the two-level one)
constexpr int PANEL_B1 = 8;    // columns per outer panel of the two-level panel schedule
constexpr int PANEL_B2 = 16;   // columns per outermost panel of the three-level schedule
#ifndef AMGS_BS_ST
#define AMGS_BS_ST 4
#endif
constexpr int BS_ST = AMGS_BS_ST; // 16-row tiles per wave of the outer block sweep
constexpr int RB_GROUPS = 2;   // 16-column groups whose blocked-pass products a wave holds at once
constexpr int BS_MAXC = 256;   // later columns per outer-block-sweep workgroup (max, a multiple of 16)
constexpr int PS_CB = 2;       // later columns streamed together by a panel-sweep thread
constexpr int PS_MAXC = 64;    // later columns per panel-sweep workgroup (max)

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
    int lanes;      // lanes per CSR row in the MV kernel (0: a row per thread, through the padded copy)
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
    // padded copy of A: entry k of row r at k*m + r (column -1 past the end)
    const int32_t *ell_col;
    const void *ell_val;
    const int32_t *tile_long;  // per MV_TILE rows: some row has more than ell_k entries
    int32_t ell_k;
    // the same columns as 16-bit offsets from the row (ELL_PAD past the end),
    // used when *ell_wide is 0: every offset fits
    const int16_t *ell_d16;
    const int32_t *ell_wide;
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
    int64_t x_from;   // HP column kernel: first recurrence term (-1: column schedule)
    int32_t pend;     // k_reorth_a: apply the pending update r_{j-1,j} q_{j-1} and publish R
    int32_t z_in_zt;  // k_reorth_a: z_j is read from zt instead of Q
    int64_t re_lo;    // second pass: against the earlier columns [re_lo, j)
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
    int64_t c_lo;     // first later column (j + 1, or the first new column)
    int32_t norm;     // 0: column j is already final (successive orthogonalisation)
};

// One step of the panel schedule (see k_psweep): normalise column j, apply
// the pending columns [k0, k1) (coefficients already in R) to the later
// columns [c0, c1), and form their dots with p_d, d in [d0, j].
struct PSweepArgs {
    int64_t m, n, j;
    void *Q;
    int64_t ldq;
    void *P;
    int64_t ldp;
    void *X;
    int64_t ldx;
    const void *zt, *xv;
    double *R;
    int64_t ldr;
    int32_t *info;
    const double *rr_part;
    int64_t n_rr;
    int64_t k0, k1;   // pending update columns
    int64_t d0;       // first dot column (j - d0 + 1 dots)
    int64_t l0;       // panel start: partials of p_j^T q_k, k in [l0, j)
    int64_t c0, c1, cpw;
    void *part;       // dot partials: part[(c * pstride + d - d0) * g + w]
    int64_t pstride;
    int64_t g;
    void *lpart;      // lpart[((j - l0) * lstride + k - l0) * g + w]
    int64_t lstride;  // PANEL_B
};

// Outer block sweep of the two-level panel schedule (see k_bsweep): apply the
// pending block [k0, k1) (coefficients final in R) to the later columns
// [c0, c1) and form their dots with p_d, d in [d0, d0 + nd).
struct BSweepArgs {
    int64_t m;
    void *Q;
    int64_t ldq;
    const void *Zs;   // where the later columns are read (Q, or Z before their first write)
    int64_t ldzs;
    const void *P;
    int64_t ldp;
    const double *R;
    int64_t ldr;
    const int32_t *info;
    int64_t k0, k1;   // pending block, k1 - k0 <= the kernel's block width
    int64_t d0, nd;   // dot columns, nd <= the kernel's block width
    int64_t c0, c1, cpw;
    void *part;       // part[(c * PANEL_B1 + d - d0) * g + w]
    void *lpart;      // partials of P_I^T Q_I: lpart[(i * PANEL_B1 + k) * g + w]
    int64_t g;
};

// Blocked second pass of an outer panel [s, s + nz) (see k_rb_dots).
struct RbArgs {
    int64_t m;
    const void *Q;    // q_i for i < s; the panel's z columns (updated in place)
    int64_t ldq;
    const void *P;
    int64_t ldp;
    void *X;          // HP: the panel's x columns (updated in place)
    int64_t ldx;
    int64_t s, nz;
    void *part;       // binary64 partials part[(i * PANEL_B1 + c) * g + w]
    int64_t g;
    const double *S;  // the coefficients s_ic at [i * PANEL_B1 + c]
    const int32_t *info;
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
    // panel schedule (panel = 0: column schedule; 4: one level; 8: two levels)
    int panel;
    int Up;           // rows per thread of the panel sweeps
    int64_t g_p;      // their row chunks
    void *wpart;      // panel-sweep dot partials [n][PANEL_B or PANEL_B1][g_p]
    void *lpart;      // partials of strict_lower(P_I^T Q_I) [PANEL_B][PANEL_B][g_p] (inner panels)
    // two-level schedule: the outer block sweep's row chunks, its partials of
    // P_I^T Q_I [PANEL_B1][PANEL_B1][g_b], and the reduced L [PANEL_B1][PANEL_B1]
    int64_t g_b;
    void *lpart8;
    void *wred;   // first-stage sums of the block-dot and L partials (8 per row)
    int64_t x_from;   // HP column kernel: first recurrence term it applies (-1: column schedule)
    int64_t n_pub;    // column kernels publish r_{j-1,c} for c < n_pub
    int cgs;          // classical Gram-Schmidt (no pending MGS update in k_reorth_a)
    int64_t first;    // columns [0, first) are already final (successive orthogonalisation)
    int z_in_zt;      // k_reorth_a reads z_j from zt
    int no_pend;      // k_reorth_a: column j has no single pending update (first column of a panel)
    // blocked second pass (two-level schedule): the per-column pass covers
    // [re_lo, j); the outer panel's block pass keeps its coefficient
    // partials [n][PANEL_B1][g_b] and the reduced coefficients [n][PANEL_B1]
    int reorth_blk;
    int64_t re_lo;
    void *rb_part;
    double *rb_s;
    // padded copy of a CSR A for the column MV (ell_k = 0: not used)
    int32_t *ell_col;
    void *ell_val;
    int32_t *tile_long;
    int16_t *ell_d16;
    int32_t *ell_wide;
    int32_t ell_k;
    hipStream_t stream;
    // when set, the sweep is launched with these events bound to its own
    // dispatch (exact kernel start and end, no extra stream markers)
    hipEvent_t ev_start, ev_stop;
};

Geo make_geo(int64_t m, int64_t nnz, int is_dense);

template <typename T> void launch_init(const Ctx &c, int64_t ncopy);
template <typename T> void launch_csr_to_ell(const Ctx &c);
template <typename T> void launch_mv(const Ctx &c, int64_t j, int src_mode);
template <typename T> void launch_col_hp(const Ctx &c, int64_t j, bool reorth_a);
template <typename T> void launch_reorth_a(const Ctx &c, int64_t j);
void launch_reorth_fin(const Ctx &c, int64_t j);
template <typename T> void launch_rb(const Ctx &c, int64_t s, int64_t e, int variant);
template <typename T> void launch_reorth_b(const Ctx &c, int64_t j, bool hp);
template <typename T> void launch_sweep(const Ctx &c, int64_t j, int variant, int64_t n_rr);
template <typename T> bool launch_hp_xblock(const Ctx &c, int64_t s, int64_t c_from);
template <typename T> void launch_publish(const Ctx &c, int64_t jrow);
template <typename T> void launch_csr_spmm(const Ctx &c);
template <typename T> void launch_dense_gemm(const Ctx &c);
template <typename T> void launch_psweep(const Ctx &c, int variant, int64_t j, int64_t k0, int64_t k1,
                                         int64_t d0, int64_t l0, int64_t c0, int64_t c1, int64_t n_rr);
template <typename T> void launch_pfin(const Ctx &c, int64_t s, int64_t e, int64_t c1);
template <typename T> void launch_bsweep(const Ctx &c, int64_t k0, int64_t k1, int64_t d0,
                                         int64_t d1, int64_t c0, int64_t c1, bool from_z = false,
                                         int bb = PANEL_B1);
template <typename T> void launch_pfin2(const Ctx &c, int64_t s, int64_t e, int64_t c0, int64_t c1,
                                        int bb = PANEL_B1);
int64_t bsweep_chunks(int64_t m, size_t w);
template <typename T> void launch_pcol_blk(const Ctx &c, int variant, int64_t j, int64_t k0, int64_t k1,
                                            int64_t xk0);
int64_t pcol_blk_partials(const Ctx &c);
int panel_rows_for(int fp64);
void launch_csr_check(int64_t m, int64_t nnz, const int32_t *row_ptr, const int32_t *col_idx,
                      int32_t *flag, hipStream_t s);

} // namespace amgs
