// amgs_single.hip -- kernels of the single-problem A-orthonormalising MGS.
//
// Schedule.  Column j of the column-oriented algorithms (Alg. 3 naive,
// Alg. 5 HA, Alg. 6 HP) needs, in order: the projections r_ij = p_i^T z_j,
// z_j -= r_ij q_i for i < j; its vector x_j (one MV for naive/HA, the
// recurrence of eq. (5) for HP); r_jj = sqrt(z_j^T x_j); q_j = z_j / r_jj
// and p_j (x_j / r_jj by eq. (4), or A q_j for naive).  The library runs
// the same per-column operations right-looking (the order of Alg. 4/7/8):
// at step j one "sweep" kernel normalises column j and then passes once over
// every later column c, applying the pending update by q_{j-1}
// (z_c -= r_{j-1,c} q_{j-1}) and forming the partial dots p_j^T z_c.  A
// "column" kernel in between applies the last update to column j+1 and
// builds its x vector and its squared A-norm partials.  Two launches per
// column (three for naive, whose second MV p_j = A q_j has its own kernel).
//
// Reductions never use atomics or grid-wide barriers: a kernel writes one
// partial per workgroup, and the next kernel re-reduces those partials in a
// fixed order (every workgroup that needs a scalar reduces it itself, with
// identical bits).  The column kernel also publishes the finished r_{j-1,c}
// of the previous sweep into R, spread over its workgroups.
#include <hip/hip_ext.h>

#include "amgs_device.h"
#include "amgs_internal.h"

namespace amgs {

// ----------------------------------------------------------------- init
// Q <- Z (unless aliased), R <- 0, info <- 0.
template <typename T>
__global__ __launch_bounds__(256) void k_init(int64_t m, int64_t n, int64_t first,
                                              const T *__restrict__ Z, int64_t ldz,
                                              T *__restrict__ Q, int64_t ldq,
                                              double *__restrict__ R, int64_t ldr, int32_t *info,
                                              int64_t ncopy, int32_t *zero_word)
{
    // columns [0, first) are final already and left untouched; columns
    // [first, first + ncopy) are copied (element e = row k of column j, the
    // position advanced by the grid stride without a division per element)
    const int64_t nn = n - first;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t t0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (ncopy > 0) {
        const int64_t sj = stride / m, sk = stride - sj * m;
        int64_t j = first + t0 / m, k = t0 % m;
        for (int64_t e = t0; e < m * ncopy; e += stride) {
            Q[k + j * ldq] = Z[k + j * ldz];
            j += sj;
            k += sk;
            if (k >= m) {
                k -= m;
                ++j;
            }
        }
    }
    for (int64_t e = t0; e < n * nn; e += stride) {
        int64_t j = first + e / n, i = e % n;
        R[i + j * ldr] = 0.0;
    }
    if (t0 == 0) {
        *info = 0;
        if (zero_word) *zero_word = 0;   // the padded copy's flag, set later in the call
    }
}

// R[jrow, c] for c in [c0, n) from the sweep partials, when no column kernel
// runs between two sweeps (the final columns of successive
// orthogonalisation).
template <typename T>
__global__ __launch_bounds__(256) void k_publish(SweepPart sp, int64_t jrow, int64_t c0, int64_t n,
                                                 double *__restrict__ R, int64_t ldr,
                                                 const int32_t *info);

// ------------------------------------------------- publish finished r_{j-1,c}
// Spread over all waves of the launching grid: wave w of the grid finalises
// columns c = c0 + w, c0 + w + nwaves, ... from the previous sweep's partials.
template <typename T>
__device__ __forceinline__ void publish_row(const SweepPart &sp, int64_t jrow, int64_t c0,
                                            int64_t n, double *__restrict__ R, int64_t ldr)
{
    const T *part = (const T *)sp.part;
    const int64_t nw = (int64_t)gridDim.x * (blockDim.x / WAVE);
    const int64_t w = (int64_t)blockIdx.x * (blockDim.x / WAVE) + threadIdx.x / WAVE;
    for (int64_t c = c0 + w; c < n; c += nw) {
        T s = coef_reduce_wave(part + c * sp.g, sp.g);
        if ((threadIdx.x & (WAVE - 1)) == 0) R[jrow + c * ldr] = (double)s;
    }
}

template <typename T>
__global__ __launch_bounds__(256) void k_publish(SweepPart sp, int64_t jrow, int64_t c0, int64_t n,
                                                 double *__restrict__ R, int64_t ldr,
                                                 const int32_t *info)
{
    if (*info) return;
    publish_row<T>(sp, jrow, c0, n, R, ldr);
}

// ------------------------------------------------------- CSR MV (column kernel)
// y = A s where s is, per SRC:
//   SRC_UPD  s = z_j - r q_{j-1} computed on the fly (r = r_{j-1,j} re-reduced
//            from the previous sweep); the own-row value is also stored in zt;
//   SRC_VEC  s = src;
//   SRC_DIV  s = src / r_jj rounded to storage (r_jj re-reduced from rr
//            partials): the naive second MV p_j = A q_j.
// With RR, also writes this workgroup's partial of s^T y (binary64).
template <typename T, int L, int SRC, bool RR>
__global__ __launch_bounds__(512) void k_csr_mv(CsrMvArgs a)
{
    __shared__ double lds[512 / WAVE];
    __shared__ T s_r;
    __shared__ double s_rr;
    if (*a.info) return;
    const T *__restrict__ vals = (const T *)a.vals;
    const T *__restrict__ src = (const T *)a.src;
    const T *__restrict__ qprev = (const T *)a.qprev;
    T *__restrict__ y = (T *)a.y;
    T *__restrict__ zt = (T *)a.zt;

    T r = 0;
    double rjj = 1.0;
    if (SRC == SRC_UPD && qprev) r = coef_reduce_bcast((const T *)a.sp.part + a.j * a.sp.g, a.sp.g, &s_r);
    if (SRC == SRC_DIV) {
        double rr = block_reduce_bcast(a.rr_part, a.n_rr, &s_rr);
        if (!norm_ok(rr)) return;
        rjj = sqrt(rr);
    }
    auto load = [&](int64_t l) -> T {
        T v = src[l];
        if (SRC == SRC_UPD && qprev) v = upd(v, r, qprev[l]);
        if (SRC == SRC_DIV) v = scale_div(v, rjj);
        return v;
    };
    const int gpw = 512 / L;                   // rows per workgroup pass
    const int g = threadIdx.x / L, lig = threadIdx.x % L;
    double acc = 0.0;
    for (int64_t row = (int64_t)blockIdx.x * gpw + g; row < a.m; row += (int64_t)gridDim.x * gpw) {
        const int32_t e0 = a.row_ptr[row], e1 = a.row_ptr[row + 1];
        T s = 0;
        // each lane takes every L-th entry, eight at a time with all gathers
        // in flight; entries past the row's end are skipped
        for (int32_t eb = e0 + lig; eb < e1; eb += 8 * L) {
            int64_t col[8];
            T av[8], xv[8];
#pragma unroll
            for (int t = 0; t < 8; ++t) {
                const bool in = eb + t * L < e1;
                col[t] = in ? a.col_idx[eb + t * L] : row;
                av[t] = in ? vals[eb + t * L] : (T)0;
            }
#pragma unroll
            for (int t = 0; t < 8; ++t) xv[t] = load(col[t]);
#pragma unroll
            for (int t = 0; t < 8; ++t)
                if (eb + t * L < e1) s += av[t] * xv[t];
        }
#pragma unroll
        for (int off = L / 2; off >= 1; off >>= 1) s += __shfl_xor(s, off, L);
        if (lig == 0) {
            y[row] = s;
            if (SRC == SRC_UPD || RR) {
                T zs = load(row);
                if (SRC == SRC_UPD) zt[row] = zs;
                if (RR) acc += (double)zs * (double)s;
            }
        }
    }
    if (RR) {
        double t = block_sum<double, 512>(acc, lds);
        if (threadIdx.x == 0) a.rr_out[blockIdx.x] = t;
    }
    // R[j-1, c] for c >= j (read by later kernels only) is published last
    if (SRC == SRC_UPD && qprev) publish_row<T>(a.sp, a.j - 1, a.j, a.n, a.R, a.ldr);
}

// CSR MV for short rows, through a padded copy of A.  Once per call the
// first K entries of every row are copied into a column-major array (entry k
// of row r at k*m + r, column -1 past the row's end), so a thread finds its
// row's entries without reading the row bounds first: the entries and the
// row's own z are requested together, then every gather.  Entries past K
// (rows longer than K, flagged per tile of MV_TILE rows) are read from the
// CSR arrays.  Same contract as k_csr_mv; the sum runs in stored order.
// The columns are also stored as 16-bit offsets from the row (ELL_PAD past
// the row's end); when every offset fits (no workgroup sets *ell_wide,
// which the call's k_init has cleared) the MV reads those, 2 bytes per
// entry instead of 4.
template <typename T>
__global__ __launch_bounds__(MV_TILE) void k_csr_to_ell(int64_t m, int32_t K,
                                                        const int32_t *__restrict__ row_ptr,
                                                        const int32_t *__restrict__ col_idx,
                                                        const T *__restrict__ vals,
                                                        int32_t *__restrict__ ell_col,
                                                        T *__restrict__ ell_val,
                                                        int32_t *__restrict__ tile_long,
                                                        int16_t *__restrict__ ell_d16,
                                                        int32_t *__restrict__ ell_wide)
{
    const int64_t row = (int64_t)blockIdx.x * MV_TILE + threadIdx.x;
    int lng = 0, wide = 0;
    if (row < m) {
        const int32_t e0 = row_ptr[row], e1 = row_ptr[row + 1];
        for (int k = 0; k < K; ++k) {
            const int32_t e = e0 + k;
            int32_t cv = -1;
            T v = 0;
            int16_t d = ELL_PAD;
            if (e < e1) {
                cv = col_idx[e];
                v = vals[e];
                const int64_t off = (int64_t)cv - row;
                if (off > ELL_PAD && off <= 32767) d = (int16_t)off;
                else wide = 1;
            }
            ell_col[(int64_t)k * m + row] = cv;
            ell_val[(int64_t)k * m + row] = v;
            ell_d16[(int64_t)k * m + row] = d;
        }
        lng = e1 - e0 > K;
    }
    lng = __syncthreads_or(lng);
    wide = __syncthreads_or(wide);
    if (threadIdx.x == 0) {
        tile_long[blockIdx.x] = lng;
        if (wide) atomicOr(ell_wide, 1);
    }
}

// RPT rows per thread: the thread's rows in RPT consecutive grid-stride
// tiles are requested together (more loads in flight per wave).  D16: the
// columns come from the 16-bit offsets.
template <typename T, int SRC, bool RR, int RPT, bool D16, int EK>
__device__ __forceinline__ void csr_mv_ell_body(const CsrMvArgs &a)
{
    static_assert(MV_TILE / WAVE >= 8, "eight waves reduce the coefficient's segments");
    __shared__ double lds[MV_TILE / WAVE];
    __shared__ T s_seg[8];
    __shared__ double s_rr;
    const T *__restrict__ vals = (const T *)a.vals;
    const int32_t *__restrict__ ecol = a.ell_col;
    const int16_t *__restrict__ ed16 = a.ell_d16;
    const T *__restrict__ eval = (const T *)a.ell_val;
    const T *__restrict__ src = (const T *)a.src;
    const T *__restrict__ qprev = (const T *)a.qprev;
    T *__restrict__ y = (T *)a.y;
    T *__restrict__ zt = (T *)a.zt;
    const bool with_upd = SRC == SRC_UPD && qprev;
    const int tid = threadIdx.x;
    const int K = a.ell_k;
    const int64_t m = a.m;
    const int64_t stride = (int64_t)gridDim.x * MV_TILE;
    // Every load is unconditional and pinned (see ld_fix) before its value
    // is tested, so that all entries, and then all gathers, are in flight
    // together.  A row past the end reads row m - 1 (its results are not
    // stored), a slot from K on repeats slot K - 1 and a padding entry
    // gathers the row's own element; both are then skipped.  Without a
    // pending term q_{j-1} is read from src and not used.
    const T *__restrict__ qsrc = with_upd ? qprev : src;
    T r = 0;
    double rjj = 1.0;
    double acc = 0.0;
    bool first = true;
    for (int64_t row0 = (int64_t)blockIdx.x * MV_TILE; row0 < m; row0 += RPT * stride) {
        // everything that does not depend on the coefficient is requested
        // first: the rows' entries and their own z (and q_{j-1})
        int32_t col[RPT][EK];
        T av[RPT][EK];
        T own_s[RPT], own_q[RPT];
        int lng[RPT];
        int64_t rowc[RPT];
#pragma unroll
        for (int u = 0; u < RPT; ++u) {
            const int64_t t0 = row0 + u * stride;
            const int64_t row = t0 + tid;
            rowc[u] = row < m ? row : m - 1;
            lng[u] = a.tile_long[(t0 < m ? t0 : m - 1) / MV_TILE] & -(int)(t0 < m);
#pragma unroll
            for (int k = 0; k < EK; ++k) {
                const int64_t kc = k < K ? k : K - 1;
                // (a 16-bit offset is decoded after pin() below)
                col[u][k] = D16 ? (int32_t)ed16[kc * m + rowc[u]] : ecol[kc * m + rowc[u]];
                av[u][k] = eval[kc * m + rowc[u]];
            }
            own_s[u] = 0;
            own_q[u] = 0;
            if (SRC == SRC_UPD || RR) {
                own_s[u] = src[rowc[u]];
                if (SRC == SRC_UPD) own_q[u] = qsrc[rowc[u]];
            }
        }
        pin();
#pragma unroll
        for (int u = 0; u < RPT; ++u)
#pragma unroll
            for (int k = 0; k < EK; ++k) {
                int32_t cv = col[u][k];
                if (D16) cv = cv == ELL_PAD ? -1 : (int32_t)rowc[u] + cv;
                col[u][k] = cv | -(int32_t)(k >= K);
            }
        // the coefficient r_{j-1,j} is re-reduced by the workgroup's eight
        // waves, one segment of the partials each (the same bits as the
        // other kernels' coef_reduce_wave), or r_jj for the naive second MV
        // by wave 0 (sixteen partials in flight per lane, the same bits as
        // wave_reduce_seq), while those loads are in flight
        if (first && (with_upd || SRC == SRC_DIV)) {
            if (with_upd) {
                coef_reduce_segments((const T *)a.sp.part + a.j * a.sp.g, a.sp.g, s_seg);
            } else if (tid < WAVE) {
                const double v = wave_reduce_seq_deep<16>(a.rr_part, a.n_rr);
                if (tid == 0) s_rr = v;
            }
            __syncthreads();
            if (with_upd) {
                r = s_seg[0];
#pragma unroll
                for (int k = 1; k < 8; ++k) r += s_seg[k];
            }
            if (SRC == SRC_DIV) {
                const double rr = s_rr;
                if (!norm_ok(rr)) return; // uniform over the workgroup
                rjj = sqrt(rr);
            }
        }
        first = false;
        auto load = [&](int64_t l) -> T {
            T v = src[l];
            if (with_upd) v = upd(v, r, qprev[l]);
            if (SRC == SRC_DIV) v = scale_div(v, rjj);
            return v;
        };
        // every gather (with q_{j-1} at the same rows) is issued before any
        // is used
        T xv[RPT][EK], xq[SRC == SRC_UPD ? RPT : 1][EK];
#pragma unroll
        for (int u = 0; u < RPT; ++u)
#pragma unroll
            for (int k = 0; k < EK; ++k) {
                const int32_t c = col[u][k];
                const int64_t l = c >= 0 ? (int64_t)c : rowc[u];
                xv[u][k] = src[l];
                if (SRC == SRC_UPD) xq[SRC == SRC_UPD ? u : 0][k] = qsrc[l];
            }
        pin();
#pragma unroll
        for (int u = 0; u < RPT; ++u)
#pragma unroll
            for (int k = 0; k < EK; ++k) {
                if (SRC == SRC_UPD)
                    xv[u][k] = with_upd ? upd(xv[u][k], r, xq[SRC == SRC_UPD ? u : 0][k]) : xv[u][k];
                if (SRC == SRC_DIV) xv[u][k] = scale_div(xv[u][k], rjj);
            }
#pragma unroll
        for (int u = 0; u < RPT; ++u) {
            const int64_t row = row0 + u * stride + tid;
            if (row >= m) continue;
            // padding only follows a row's last entry: it is skipped, not
            // multiplied by zero
            T s = 0;
#pragma unroll
            for (int k = 0; k < EK; ++k) {
                const T t = s + av[u][k] * xv[u][k];
                s = col[u][k] >= 0 ? t : s;
            }
            if (lng[u]) {
                // the row's entries past the first K, eight at a time
                const int32_t e1 = a.row_ptr[row + 1];
                for (int32_t eb = a.row_ptr[row] + K; eb < e1; eb += 8) {
                    int64_t cl[8];
                    T cv[8], gv[8];
#pragma unroll
                    for (int t = 0; t < 8; ++t) {
                        const bool in = eb + t < e1;
                        cl[t] = in ? a.col_idx[eb + t] : row;
                        cv[t] = in ? vals[eb + t] : (T)0;
                    }
#pragma unroll
                    for (int t = 0; t < 8; ++t) gv[t] = load(cl[t]);
#pragma unroll
                    for (int t = 0; t < 8; ++t)
                        if (eb + t < e1) s += cv[t] * gv[t];
                }
            }
            y[row] = s;
            if (SRC == SRC_UPD || RR) {
                T zs = own_s[u];
                if (SRC == SRC_UPD) zs = with_upd ? upd(zs, r, own_q[u]) : zs;
                if (SRC == SRC_DIV) zs = scale_div(zs, rjj);
                if (SRC == SRC_UPD) zt[row] = zs;
                if (RR) acc += (double)zs * (double)s;
            }
        }
    }
    if (RR) {
        double t = block_sum<double, MV_TILE>(acc, lds);
        if (tid == 0) a.rr_out[blockIdx.x] = t;
    }
    // R[j-1, c] for c >= j, read by the next sweep, is published last so
    // that it does not delay this kernel's own loads
    if (with_upd) publish_row<T>(a.sp, a.j - 1, a.j, a.n, a.R, a.ldr);
}

// The padded-copy MV with the column format of this call's copy: the
// 16-bit offsets unless some offset did not fit (a wave-uniform test, once).
// EK: the slots a thread holds per row, ELL_K, or 7 when the copy has
// exactly seven (7-point stencils), so no slot is loaded twice.
template <typename T, int SRC, bool RR, int RPT, int EK>
__global__ __launch_bounds__(MV_TILE) void k_csr_mv_ell(CsrMvArgs a)
{
    if (*a.info) return;
    if (*a.ell_wide) csr_mv_ell_body<T, SRC, RR, RPT, false, EK>(a);
    else csr_mv_ell_body<T, SRC, RR, RPT, true, EK>(a);
}

// ----------------------------------------------------- dense MV (column kernel)
// Same contract as k_csr_mv for a dense symmetric column-major A: output
// entry k is the dot of column k of A with s.  A workgroup owns CB outputs at
// a time; its 256 threads stride down the columns (coalesced), each thread
// keeps CB accumulators, then a fixed-order workgroup reduction.
template <typename T, int CB, int SRC, bool RR>
__global__ __launch_bounds__(256) void k_dense_mv(DenseMvArgs a)
{
    __shared__ T red[256 / WAVE][CB];
    __shared__ double lds[256 / WAVE];
    __shared__ T s_r;
    __shared__ double s_rr;
    if (*a.info) return;
    const T *__restrict__ A = (const T *)a.A;
    const T *__restrict__ src = (const T *)a.src;
    const T *__restrict__ qprev = (const T *)a.qprev;
    T *__restrict__ y = (T *)a.y;
    T *__restrict__ zt = (T *)a.zt;
    T r = 0;
    double rjj = 1.0;
    if (SRC == SRC_UPD && qprev) r = coef_reduce_bcast((const T *)a.sp.part + a.j * a.sp.g, a.sp.g, &s_r);
    if (SRC == SRC_DIV) {
        double rr = block_reduce_bcast(a.rr_part, a.n_rr, &s_rr);
        if (!norm_ok(rr)) return;
        rjj = sqrt(rr);
    }
    auto load = [&](int64_t l) -> T {
        T v = src[l];
        if (SRC == SRC_UPD && qprev) v = upd(v, r, qprev[l]);
        if (SRC == SRC_DIV) v = scale_div(v, rjj);
        return v;
    };
    const int tid = threadIdx.x, wave = tid / WAVE;
    double acc_rr = 0.0;
    for (int64_t k0 = (int64_t)blockIdx.x * CB; k0 < a.m; k0 += (int64_t)gridDim.x * CB) {
        const int nc = (int)(a.m - k0 < CB ? a.m - k0 : CB);
        T acc[CB];
#pragma unroll
        for (int c = 0; c < CB; ++c) acc[c] = 0;
        const T *__restrict__ Ak = A + k0 * a.lda;
        // all CB column entries and the vector entry are requested before
        // the first multiply-add, so every load of a trip is in flight
        // together
        if (nc == CB) {
            for (int64_t l = tid; l < a.m; l += 256) {
                T av[CB];
#pragma unroll
                for (int c = 0; c < CB; ++c) av[c] = Ak[l + c * a.lda];
                const T s = load(l);
#pragma unroll
                for (int c = 0; c < CB; ++c) acc[c] += av[c] * s;
            }
        } else {
            for (int64_t l = tid; l < a.m; l += 256) {
                T av[CB];
#pragma unroll
                for (int c = 0; c < CB; ++c) av[c] = c < nc ? Ak[l + c * a.lda] : (T)0;
                const T s = load(l);
#pragma unroll
                for (int c = 0; c < CB; ++c)
                    if (c < nc) acc[c] += av[c] * s;
            }
        }
#pragma unroll
        for (int c = 0; c < CB; ++c) {
            T v = wave_sum(acc[c]);
            if ((tid & (WAVE - 1)) == 0) red[wave][c] = v;
        }
        __syncthreads();
        if (tid < nc) {
            T s = red[0][tid];
#pragma unroll
            for (int w = 1; w < 256 / WAVE; ++w) s += red[w][tid];
            y[k0 + tid] = s;
            if (SRC == SRC_UPD || RR) {
                T zs = load(k0 + tid);
                if (SRC == SRC_UPD) zt[k0 + tid] = zs;
                if (RR) acc_rr += (double)zs * (double)s;
            }
        }
        __syncthreads();
    }
    if (RR) {
        double t = block_sum<double, 256>(acc_rr, lds);
        if (tid == 0) a.rr_out[blockIdx.x] = t;
    }
    // R[j-1, c] for c >= j (read by later kernels only) is published last
    if (SRC == SRC_UPD && qprev) publish_row<T>(a.sp, a.j - 1, a.j, a.n, a.R, a.ldr);
}

// The p_i of one workgroup's group of second-pass coefficients,
// i in [i_lo, min(i_lo + RE_GROUP, j)), at its rows (zero elsewhere).
template <typename T, int U>
__device__ __forceinline__ void reorth_load(const T *__restrict__ P, int64_t ldp, int64_t j,
                                            int64_t i_lo, int64_t row0, int64_t m,
                                            T (&pv)[RE_GROUP][U])
{
    const int tid = threadIdx.x;
#pragma unroll
    for (int t = 0; t < RE_GROUP; ++t)
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t k = row0 + u * 256 + tid;
            const int64_t kc = k < m ? k : m - 1;
            pv[t][u] = ld_fix(P, k + (i_lo + t) * ldp, kc, i_lo + t < j && k < m);
        }
}

// Partials of the second-pass coefficients s_i = p_i^T z_j of that group
// over the workgroup's rows (binary64 accumulation): each wave reduces its
// part, and the four wave sums are combined in wave order.
template <typename T, int U>
__device__ __forceinline__ void reorth_partials(const T (&pv)[RE_GROUP][U], const T (&zr)[U],
                                                int64_t j, int64_t i_lo,
                                                double *__restrict__ s_part,
                                                double (*red)[RE_GROUP])
{
    const int tid = threadIdx.x, wave = tid / WAVE;
    const int64_t nb = j - i_lo < RE_GROUP ? j - i_lo : RE_GROUP;
#pragma unroll
    for (int t = 0; t < RE_GROUP; ++t) {
        double sacc = 0.0;
#pragma unroll
        for (int u = 0; u < U; ++u) sacc += (double)pv[t][u] * (double)zr[u];
        const double v = wave_sum(sacc);
        if ((tid & (WAVE - 1)) == 0) red[wave][t] = v;
    }
    __syncthreads();
    if (tid < nb) {
        double v = red[0][tid];
#pragma unroll
        for (int w = 1; w < 256 / WAVE; ++w) v += red[w][tid];
        s_part[(i_lo + tid) * gridDim.x + blockIdx.x] = v;
    }
}

// ------------------------------------------------------ HP column kernel
// Row-local: z_j -= r_{j-1,j} q_{j-1} in place, then the recurrence of
// eq. (5), x_j = x_j^{(0)} - sum_{i<j} r_ij p_i with i ascending, in
// place in X, and the partial of z_j^T x_j.  With REORTH_A it instead stops
// after the recurrence and writes partials of s_i = p_i^T z_j (binary64)
// for the second pass (no A-norm yet).
template <typename T, int U, bool REORTH_A>
__global__ __launch_bounds__(256) void k_col_hp(RowArgs a)
{
    __shared__ double lds[256 / WAVE];
    __shared__ double red[256 / WAVE][RE_GROUP];
    __shared__ T s_r;
    if (*a.info) return;
    const int64_t j = a.j;
    T *__restrict__ Q = (T *)a.Q;
    T *__restrict__ X = (T *)a.X;
    const T *__restrict__ P = (const T *)a.P;
    const int tid = threadIdx.x;
    const int64_t row0 = (int64_t)blockIdx.x * 256 * U;
    // issue the row loads before waiting for r_{j-1,j}
    T zr[U], qp[U], x[U], pv[HP_XB][U];
    // first recurrence term applied here: in the column schedule the terms
    // below XB floor((j-1)/XB) were applied by k_hp_xblock; in the panel
    // schedule the sweeps have applied all terms but the last
    const int64_t i0 = a.x_from >= 0 ? a.x_from : (j > 0 ? HP_XB * ((j - 1) / HP_XB) : 0);
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const int64_t k = row0 + u * 256 + tid;
        const bool in = k < a.m;
        const int64_t kc = in ? k : a.m - 1;
        const bool xin = in && blockIdx.y == 0;   // only grid row 0 needs x_j
        zr[u] = ld_fix(Q, k + j * a.ldq, kc, in);
        qp[u] = ld_fix(Q, k + (j - 1) * a.ldq, kc, in && j > 0);
        x[u] = ld_fix(X, k + j * a.ldx, kc, xin);
#pragma unroll
        for (int t = 0; t < HP_XB; ++t)
            pv[t][u] = ld_fix(P, k + (i0 + t) * a.ldp, kc, xin && i0 + t < j);
    }
    // the published r_ij of the recurrence (i < j - 1), requested with them
    double rv[HP_XB];
#pragma unroll
    for (int t = 0; t < HP_XB; ++t) rv[t] = ld_fix(a.R, (i0 + t) + j * a.ldr, 0, i0 + t < j - 1);
    pin();
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const int64_t k = row0 + u * 256 + tid;
        const bool in = k < a.m, xin = in && blockIdx.y == 0;
        zr[u] = pick(zr[u], in);
        qp[u] = pick(qp[u], in && j > 0);
        x[u] = pick(x[u], xin);
#pragma unroll
        for (int t = 0; t < HP_XB; ++t) pv[t][u] = pick(pv[t][u], xin && i0 + t < j);
    }
    // with REORTH_A the grid has one row per group of second-pass
    // coefficients; grid row 0 alone writes z_j (to zt, so that the other
    // grid rows still read the old z_j from Q), x_j, and publishes R
    const bool own = blockIdx.y == 0;
    T *__restrict__ zdst = REORTH_A ? (T *)a.zt : Q + j * a.ldq;
    T r = 0;
    if (j > 0) r = coef_reduce_bcast((const T *)a.sp.part + j * a.sp.g, a.sp.g, &s_r);
    T xr[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const int64_t k = row0 + u * 256 + tid;
        if (k < a.m && j > 0) zr[u] = upd(zr[u], r, qp[u]);
        if (k < a.m && own && (j > 0 || REORTH_A)) zdst[k] = zr[u];
    }
    // x recurrence, i ascending, terms i >= XB floor((j-1)/XB) (the earlier
    // ones were applied by k_hp_xblock); r_ij (i < j-1) were published by
    // earlier column kernels, r_{j-1,j} is the value re-reduced above.
    {
#pragma unroll
        for (int t = 0; t < HP_XB; ++t) {
            const int64_t i = i0 + t;
            if (i < j) {
                const T ri = (i == j - 1) ? r : (T)rv[t];
#pragma unroll
                for (int u = 0; u < U; ++u) x[u] = upd(x[u], ri, pv[t][u]);
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t k = row0 + u * 256 + tid;
            if (k < a.m && own) X[k + j * a.ldx] = x[u];
            xr[u] = x[u];
        }
    }
    if (!REORTH_A) {
        double acc = 0.0;
#pragma unroll
        for (int u = 0; u < U; ++u) acc += (double)zr[u] * (double)xr[u];
        double t = block_sum<double, 256>(acc, lds);
        if (tid == 0) a.rr_out[blockIdx.x] = t;
    } else {
        const int64_t i_lo = a.re_lo + (int64_t)blockIdx.y * RE_GROUP;
        T pr[RE_GROUP][U];
        reorth_load<T, U>(P, a.ldp, j, i_lo, row0, a.m, pr);
        reorth_partials<T, U>(pr, zr, j, i_lo, a.s_part, red);
    }
    // R[j-1, c] for c >= j (read by later kernels only) is published last
    if (j > 0 && own) publish_row<T>(a.sp, j - 1, j, a.n, a.R, a.ldr);
}

// ------------------------------------- second pass, step A for naive / HA
// zt = z_j - r_{j-1,j} q_{j-1} (row local) and partials of s_i = p_i^T zt.
// Also the first step of a classical Gram-Schmidt column (pend = 0): the
// partials of r_ij = p_i^T z_j^{(0)}, i < j, with z_j unmodified.
template <typename T, int U>
__global__ __launch_bounds__(256) void k_reorth_a(RowArgs a)
{
    __shared__ double red[256 / WAVE][RE_GROUP];
    __shared__ T s_r;
    if (*a.info) return;
    const int64_t j = a.j;
    const T *__restrict__ Q = (const T *)a.Q;
    const T *__restrict__ P = (const T *)a.P;
    T *__restrict__ zt = (T *)a.zt;
    const int tid = threadIdx.x;
    const int64_t row0 = (int64_t)blockIdx.x * 256 * U;
    // z_j from Q (or, for a second classical pass of naive / HA, from zt);
    // with pend, the pending update r_{j-1,j} q_{j-1} of the column
    // schedule is applied first (classical Gram-Schmidt has none).  All row
    // loads, this grid row's p_i included, are issued before the wait for
    // r_{j-1,j}.
    const bool pend = a.pend && j > 0;
    const T *__restrict__ zsrc = a.z_in_zt ? (const T *)zt : Q + j * a.ldq;
    const int64_t i_lo = a.re_lo + (int64_t)blockIdx.y * RE_GROUP;
    T zr[U], qp[U], pv[RE_GROUP][U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const int64_t k = row0 + u * 256 + tid;
        const int64_t kc = k < a.m ? k : a.m - 1;
        zr[u] = ld_fix(zsrc, k, kc, k < a.m);
        qp[u] = ld_fix(Q, k + (j - 1) * a.ldq, kc, k < a.m && pend);
    }
    reorth_load<T, U>(P, a.ldp, j, i_lo, row0, a.m, pv);
    pin();
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const int64_t k = row0 + u * 256 + tid;
        zr[u] = pick(zr[u], k < a.m);
        qp[u] = pick(qp[u], k < a.m && pend);
#pragma unroll
        for (int t = 0; t < RE_GROUP; ++t) pv[t][u] = pick(pv[t][u], i_lo + t < j && k < a.m);
    }
    T r = 0;
    if (pend) r = coef_reduce_bcast((const T *)a.sp.part + j * a.sp.g, a.sp.g, &s_r);
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const int64_t k = row0 + u * 256 + tid;
        if (k < a.m) {
            if (pend) zr[u] = upd(zr[u], r, qp[u]);
            if (blockIdx.y == 0 && !a.z_in_zt) zt[k] = zr[u];
        }
    }
    reorth_partials<T, U>(pv, zr, j, i_lo, a.s_part, red);
    // R[j-1, c] for c >= j (read by later kernels only) is published last
    if (pend && blockIdx.y == 0) publish_row<T>(a.sp, j - 1, j, a.n, a.R, a.ldr);
}

// ----------------------------------------------- second pass: finish s_i
// Wave w of the grid handles coefficient i = w: S[i] = sum of its partials,
// and r_ij += S[i].
__global__ __launch_bounds__(256) void k_reorth_fin(const double *__restrict__ s_part,
                                                    int64_t g, int64_t i0, int64_t j,
                                                    double *__restrict__ S,
                                                    double *__restrict__ R, int64_t ldr,
                                                    const int32_t *info)
{
    if (*info) return;
    const int64_t i = i0 + (int64_t)blockIdx.x * (blockDim.x / WAVE) + threadIdx.x / WAVE;
    if (i >= j) return;
    double s = wave_reduce_seq(s_part + i * g, g);
    if ((threadIdx.x & (WAVE - 1)) == 0) {
        S[i] = s;
        R[i + j * ldr] = R[i + j * ldr] + s;
    }
}

// ------------------------------------- second pass, step B (all variants)
// z_j <- z_j - sum_i S_i q_i and (HP) x_j <- x_j - sum_i S_i p_i, binary64
// accumulation, rounded once; HP also forms the A-norm partials.
template <typename T, int U, bool HP>
__global__ __launch_bounds__(256) void k_reorth_b(RowArgs a)
{
    __shared__ double lds[256 / WAVE];
    if (*a.info) return;
    const int64_t j = a.j;
    const T *__restrict__ Q = (const T *)a.Q;
    const T *__restrict__ P = (const T *)a.P;
    // z_j after the first pass is in zt (all variants); the corrected
    // column goes back to zt (naive, HA: their MV reads it) or to Q (HP)
    const T *__restrict__ zv = (const T *)a.zt;
    T *__restrict__ zout = HP ? (T *)a.Q + j * a.ldq : (T *)a.zt;
    T *__restrict__ xv = HP ? (T *)a.X + j * a.ldx : nullptr;
    const int tid = threadIdx.x;
    const int64_t row0 = (int64_t)blockIdx.x * 256 * U;
    double zd[U], xd[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const int64_t k = row0 + u * 256 + tid;
        const int64_t kc = k < a.m ? k : a.m - 1;
        zd[u] = (double)ld_fix(zv, k, kc, k < a.m);
        xd[u] = HP ? (double)ld_fix(xv, k, kc, k < a.m) : 0.0;
    }
    // the earlier columns eight at a time (one group for the columns of a
    // panel of eight), all of a group's loads in flight together
    for (int64_t ib = a.re_lo; ib < j; ib += 8) {
        T qv[8][U], pv[HP ? 8 : 1][U];
#pragma unroll
        for (int t = 0; t < 8; ++t)
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int64_t k = row0 + u * 256 + tid;
                const int64_t kc = k < a.m ? k : a.m - 1;
                const bool in = ib + t < j && k < a.m;
                qv[t][u] = ld_fix(Q, k + (ib + t) * a.ldq, kc, in);
                if (HP) pv[HP ? t : 0][u] = ld_fix(P, k + (ib + t) * a.ldp, kc, in);
            }
        double sv[8];
#pragma unroll
        for (int t = 0; t < 8; ++t) sv[t] = ld_fix(a.S, ib + t, ib, ib + t < j);
        pin();
#pragma unroll
        for (int t = 0; t < 8; ++t) {
            if (ib + t < j) {
                const double s = sv[t];
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    zd[u] -= s * (double)qv[t][u];
                    if (HP) xd[u] -= s * (double)pv[HP ? t : 0][u];
                }
            }
        }
    }
    double acc = 0.0;
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const int64_t k = row0 + u * 256 + tid;
        if (k < a.m) {
            const T z = (T)zd[u];
            zout[k] = z;
            if (HP) {
                const T x = (T)xd[u];
                xv[k] = x;
                acc += (double)z * (double)x;
            }
        }
    }
    if (HP) {
        double t = block_sum<double, 256>(acc, lds);
        if (tid == 0) a.rr_out[blockIdx.x] = t;
    }
}

// ------------------------------------------------------------ sweep
// Step j: r_jj from the A-norm partials (breakdown -> info = j+1); column j
// normalised: q_j = z_j / r_jj, p_j = x_j / r_jj (HA, HP; eq. (4)) or
// p_j = A q_j already formed (naive).  Then for every later column c owned
// by this workgroup (columns c0 .. c0+cpw-1 of grid row y):
//     z_c <- z_c - r_{j-1,c} q_{j-1}     (update of step j-1)
//     partial of r_{j,c} = p_j^T z_c     (dot of step j)
// with z_c read and written once.  One wave re-reduces the A-norm partials
// and broadcasts r_jj through LDS.

template <typename T, int U, int VAR, bool NTS>
__global__ __launch_bounds__(256) void k_sweep(SweepArgs a)
{
    __shared__ T red[256 / WAVE][MAX_CPW];
    __shared__ double s_rr;
    if (*a.info) return;
    const int64_t j = a.j, m = a.m;
    const int tid = threadIdx.x, wave = tid / WAVE;
    T *__restrict__ Q = (T *)a.Q;
    T *__restrict__ P = (T *)a.P;
    const int64_t row0 = (int64_t)blockIdx.x * 256 * U;
    const bool own = blockIdx.y == 0;
    const T *__restrict__ zsrc = VAR == VAR_HP ? Q + j * a.ldq : (const T *)a.zt;
    const T *__restrict__ xsrc = VAR == VAR_HP ? (const T *)a.X + j * a.ldx : (const T *)a.xv;
    // issue the vector loads before waiting for r_jj; a column that is
    // already final (norm = 0) only supplies its stored p_j
    T xs[U], zs[U], qp[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const int64_t k = row0 + u * 256 + tid;
        const bool in = k < m;
        xs[u] = in ? ((VAR == VAR_NAIVE || !a.norm) ? P[k + j * a.ldp] : xsrc[k]) : (T)0;
        zs[u] = (in && own && a.norm) ? zsrc[k] : (T)0;
        qp[u] = (in && j > 0) ? Q[k + (j - 1) * a.ldq] : (T)0;
    }
    const int64_t c0 = a.c_lo + (int64_t)blockIdx.y * a.cpw;
    const int64_t c1 = (c0 + a.cpw < a.n) ? c0 + a.cpw : a.n;
    const bool full_rows = row0 + 256 * U <= m;
    // start streaming the first group of later columns before waiting for
    // the A-norm reduction
    T zv[SWEEP_CB][U];
#pragma unroll
    for (int t = 0; t < SWEEP_CB; ++t) {
        const T *__restrict__ Zc = Q + (c0 + t) * a.ldq;
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t k = row0 + u * 256 + tid;
            zv[t][u] = (c0 + t < c1 && (full_rows || k < m)) ? ld_stream<NTS>(Zc + k) : (T)0;
        }
    }
    T p[U];
    if (a.norm) {
        if (wave == 0) {
            const double rr = wave_reduce_seq(a.rr_part, a.n_rr);
            if (tid == 0) s_rr = rr;
        }
        __syncthreads();
        const double rr = s_rr;
        if (!norm_ok(rr)) {
            if (blockIdx.x == 0 && blockIdx.y == 0 && tid == 0) *a.info = (int32_t)(j + 1);
            return;
        }
        const double rjj = sqrt(rr);
        if (blockIdx.x == 0 && blockIdx.y == 0 && tid == 0) a.R[j + j * a.ldr] = rjj;
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t k = row0 + u * 256 + tid;
            p[u] = VAR == VAR_NAIVE ? xs[u] : scale_div(xs[u], rjj);
            if (own && k < m) {
                // only the owning workgroup reads z_j: for HP it is
                // overwritten in place by q_j
                Q[k + j * a.ldq] = scale_div(zs[u], rjj);
                if (VAR != VAR_NAIVE) P[k + j * a.ldp] = p[u];
            }
        }
    } else {
#pragma unroll
        for (int u = 0; u < U; ++u) p[u] = xs[u];
    }
    if (c0 >= c1) return;
    for (int64_t cb = c0; cb < c1; cb += SWEEP_CB) {
        T r[SWEEP_CB], acc[SWEEP_CB];
#pragma unroll
        for (int t = 0; t < SWEEP_CB; ++t) {
            acc[t] = 0;
            r[t] = (j > 0 && cb + t < c1) ? (T)a.R[(j - 1) + (cb + t) * a.ldr] : (T)0;
        }
        if (cb > c0) {
#pragma unroll
            for (int t = 0; t < SWEEP_CB; ++t) {
                const T *__restrict__ Zc = Q + (cb + t) * a.ldq;
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const int64_t k = row0 + u * 256 + tid;
                    zv[t][u] = (cb + t < c1 && (full_rows || k < m)) ? ld_stream<NTS>(Zc + k) : (T)0;
                }
            }
        }
#pragma unroll
        for (int t = 0; t < SWEEP_CB; ++t) {
            T *__restrict__ Zc = Q + (cb + t) * a.ldq;
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int64_t k = row0 + u * 256 + tid;
                if (cb + t < c1 && (full_rows || k < m)) {
                    T z = zv[t][u];
                    if (j > 0) {
                        z = upd(z, r[t], qp[u]);
                        st_stream<NTS>(Zc + k, z);
                    }
                    acc[t] += p[u] * z;
                }
            }
        }
#pragma unroll
        for (int t = 0; t < SWEEP_CB; ++t) {
            T v = wave_sum(acc[t]);
            if ((tid & (WAVE - 1)) == 0 && cb + t < c1) red[wave][cb - c0 + t] = v;
        }
    }
    __syncthreads();
    for (int64_t c = tid; c < c1 - c0; c += 256) {
        T s = red[0][c];
#pragma unroll
        for (int w = 1; w < 256 / WAVE; ++w) s += red[w][c];
        ((T *)a.sp.part)[(c0 + c) * a.sp.g + blockIdx.x] = s;
    }
}

// ------------------------------------------- HP recurrence, blocked terms
// At steps s = XB, 2 XB, ... the terms i = s-XB .. s-1 of eq. (5) are
// applied to every later column: x_c <- x_c - r_ic p_i, i ascending.  The
// column kernel of column j then only adds the terms i >= XB floor((j-1)/XB),
// so every x_c receives its terms in ascending i, as in the sequential
// recurrence, while each p_i is streamed once per block instead of once per
// column.
template <typename T>
__global__ __launch_bounds__(256) void k_hp_xblock(int64_t m, int64_t n, int64_t s, int64_t c_lo,
                                                   int64_t cpw,
                                                   const T *__restrict__ P, int64_t ldp,
                                                   T *__restrict__ X, int64_t ldx,
                                                   const double *__restrict__ R, int64_t ldr,
                                                   const int32_t *info)
{
    if (*info) return;
    const int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t c0 = c_lo + (int64_t)blockIdx.y * cpw;
    const int64_t c1 = (c0 + cpw < n) ? c0 + cpw : n;
    if (k >= m || c0 >= c1) return;
    T pv[HP_XB];
#pragma unroll
    for (int i = 0; i < HP_XB; ++i) pv[i] = P[k + (s - HP_XB + i) * ldp];
    int64_t c = c0;
    for (; c + 4 <= c1; c += 4) {
        T x[4];
#pragma unroll
        for (int t = 0; t < 4; ++t) x[t] = X[k + (c + t) * ldx];
#pragma unroll
        for (int i = 0; i < HP_XB; ++i)
#pragma unroll
            for (int t = 0; t < 4; ++t) x[t] = upd(x[t], (T)R[(s - HP_XB + i) + (c + t) * ldr], pv[i]);
#pragma unroll
        for (int t = 0; t < 4; ++t) X[k + (c + t) * ldx] = x[t];
    }
    for (; c < c1; ++c) {
        T x = X[k + c * ldx];
#pragma unroll
        for (int i = 0; i < HP_XB; ++i) x = upd(x, (T)R[(s - HP_XB + i) + c * ldr], pv[i]);
        X[k + c * ldx] = x;
    }
}

// ------------------------------------------------- HP block product, CSR
// X = A Z for all n columns (the block product of Alg. 6).  Thread per row.
// Every load of a column group is issued without a branch, so that all of
// them are in flight together: an entry slot past the row's end reads a
// valid entry (the row's last one, or entry 0 for an empty row) and its
// product is then dropped by a select, not multiplied by zero.  Rows of at
// most eight entries keep their indices and values in registers for every
// column group; longer rows are taken eight entries at a time per group
// (those re-reads stay in the caches).  Columns go in groups of SPMM_C.
template <typename T>
__device__ __forceinline__ void spmm_group(const T *__restrict__ Zc, int64_t ldz, int nc,
                                          const int64_t (&l)[8], const T (&v)[8],
                                          const bool (&in)[8], T (&acc)[SPMM_C])
{
    constexpr int C = SPMM_C;
    T zz[C][8];
#pragma unroll
    for (int c = 0; c < C; ++c)
#pragma unroll
        for (int t = 0; t < 8; ++t) zz[c][t] = Zc[l[t] + (int64_t)(c < nc ? c : 0) * ldz];
#pragma unroll
    for (int c = 0; c < C; ++c)
#pragma unroll
        for (int t = 0; t < 8; ++t) {
            const T p = acc[c] + v[t] * zz[c][t];
            acc[c] = in[t] ? p : acc[c];
        }
}

template <typename T>
__global__ __launch_bounds__(256) void k_csr_spmm(int64_t m, int64_t n, int64_t nnz,
                                                  const int32_t *__restrict__ row_ptr,
                                                  const int32_t *__restrict__ col_idx,
                                                  const T *__restrict__ vals, const T *__restrict__ Z,
                                                  int64_t ldz, T *__restrict__ X, int64_t ldx)
{
    constexpr int C = SPMM_C;
    const int64_t row = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (row >= m) return;
    if (nnz == 0) {
        for (int64_t c = 0; c < n; ++c) X[row + c * ldx] = (T)0;
        return;
    }
    const int32_t e0 = row_ptr[row], e1 = row_ptr[row + 1];
    const int32_t safe = e1 > 0 ? e1 - 1 : 0;   // a valid entry for the unused slots
    int64_t l[8];
    T v[8];
    bool in[8];
    auto load_entries = [&](int32_t eb) {
#pragma unroll
        for (int t = 0; t < 8; ++t) {
            in[t] = eb + t < e1;
            const int32_t ei = in[t] ? eb + t : safe;
            l[t] = col_idx[ei];
            v[t] = vals[ei];
        }
    };
    const bool short_row = e1 - e0 <= 8;
    if (short_row) load_entries(e0);
    for (int64_t c0 = 0; c0 < n; c0 += C) {
        const int nc = (int)(n - c0 < C ? n - c0 : C);
        const T *__restrict__ Zc = Z + c0 * ldz;
        T acc[C];
#pragma unroll
        for (int c = 0; c < C; ++c) acc[c] = 0;
        if (short_row) {
            spmm_group<T>(Zc, ldz, nc, l, v, in, acc);
        } else {
            for (int32_t eb = e0; eb < e1; eb += 8) {
                load_entries(eb);
                spmm_group<T>(Zc, ldz, nc, l, v, in, acc);
            }
        }
        // X is not read again by this kernel: streamed past the caches, which
        // keep the gathered rows of Z
#pragma unroll
        for (int c = 0; c < C; ++c)
            if (c < nc) __builtin_nontemporal_store(acc[c], X + row + (c0 + c) * ldx);
    }
}

// HP block product for longer rows: L lanes share a row (L from the mean
// row length, as for the column MV), each lane takes every L-th entry and
// applies it to SPMM_LC columns of Z at once, so an entry is read once per
// column group; the lanes' sums are then combined with shuffles.  Grid:
// (row groups of 256 / L rows, column groups of SPMM_LC).
template <typename T, int L>
__global__ __launch_bounds__(256) void k_csr_spmm_lanes(int64_t m, int64_t n,
                                                        const int32_t *__restrict__ row_ptr,
                                                        const int32_t *__restrict__ col_idx,
                                                        const T *__restrict__ vals,
                                                        const T *__restrict__ Z, int64_t ldz,
                                                        T *__restrict__ X, int64_t ldx)
{
    constexpr int C = SPMM_LC;
    constexpr int E = 4;   // entries per lane in flight
    const int g = threadIdx.x / L, lig = threadIdx.x % L;
    const int64_t row = (int64_t)blockIdx.x * (256 / L) + g;
    const int64_t c0 = (int64_t)blockIdx.y * C;
    const int nc = (int)(n - c0 < C ? n - c0 : C);
    const bool live = row < m;   // uniform over the L lanes of a row
    T acc[C];
#pragma unroll
    for (int c = 0; c < C; ++c) acc[c] = 0;
    if (live) {
        const int32_t e0 = row_ptr[row], e1 = row_ptr[row + 1];
        const T *__restrict__ Zc = Z + c0 * ldz;
        for (int32_t eb = e0 + lig; eb < e1; eb += E * L) {
            int64_t l[E];
            T v[E];
#pragma unroll
            for (int t = 0; t < E; ++t) {
                const bool in = eb + t * L < e1;
                l[t] = in ? col_idx[eb + t * L] : row;
                v[t] = in ? vals[eb + t * L] : (T)0;
            }
            T zg[E][C];
#pragma unroll
            for (int t = 0; t < E; ++t)
#pragma unroll
                for (int c = 0; c < C; ++c) zg[t][c] = c < nc ? Zc[l[t] + c * ldz] : (T)0;
            // entries past the row's end are skipped, not multiplied by zero
#pragma unroll
            for (int t = 0; t < E; ++t)
                if (eb + t * L < e1)
#pragma unroll
                    for (int c = 0; c < C; ++c) acc[c] += v[t] * zg[t][c];
        }
    }
#pragma unroll
    for (int c = 0; c < C; ++c)
#pragma unroll
        for (int off = L / 2; off >= 1; off >>= 1) acc[c] += __shfl_xor(acc[c], off, L);
    if (live && lig == 0) {
        // X is not read again by this kernel: streamed past the caches, which
        // keep the gathered rows of Z
#pragma unroll
        for (int c = 0; c < C; ++c)
            if (c < nc) __builtin_nontemporal_store(acc[c], X + row + (c0 + c) * ldx);
    }
}

// --------------------------------------------------------- CSR validation
__global__ __launch_bounds__(256) void k_csr_check(int64_t m, int64_t nnz, const int32_t *__restrict__ row_ptr,
                                                   const int32_t *__restrict__ col_idx,
                                                   int32_t *flag)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t t0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    bool bad = false;
    if (t0 == 0) bad = row_ptr[0] != 0 || row_ptr[m] != nnz;
    for (int64_t k = t0; k < m; k += stride) bad |= row_ptr[k + 1] < row_ptr[k];
    for (int64_t e = t0; e < nnz; e += stride) bad |= col_idx[e] < 0 || col_idx[e] >= m;
    if (bad) *flag = 1;
}

__global__ void k_set_i32(int32_t *p, int32_t v) { *p = v; }

// ====================================================================
// Host launchers
// ====================================================================
template <typename T>
void launch_init(const Ctx &c, int64_t ncopy)
{
    const int64_t nn = c.n - c.first;
    int64_t work = ncopy > 0 ? c.m * ncopy : c.n * nn;
    int64_t blocks = (work + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(k_init<T>, dim3((unsigned)blocks), dim3(256), 0, c.stream, c.m, c.n,
                       c.first, (const T *)c.Z, c.ldz, (T *)c.Q, c.ldq, c.R, c.ldr, c.info, ncopy,
                       c.ell_k ? c.ell_wide : nullptr);
}

// The padded copy of A used by the short-row column MV: one workgroup per
// tile of MV_TILE rows.
template <typename T>
void launch_csr_to_ell(const Ctx &c)
{
    const int64_t tiles = (c.m + MV_TILE - 1) / MV_TILE;
    hipLaunchKernelGGL(k_csr_to_ell<T>, dim3((unsigned)tiles), dim3(MV_TILE), 0, c.stream, c.m,
                       c.ell_k, c.row_ptr, c.col_idx, (const T *)c.vals, c.ell_col,
                       (T *)c.ell_val, c.tile_long, c.ell_d16, c.ell_wide);
}

template <typename T>
void launch_publish(const Ctx &c, int64_t jrow)
{
    const int64_t ncols = c.n - c.first;
    const int64_t blocks = (ncols + 3) / 4;
    hipLaunchKernelGGL(k_publish<T>, dim3((unsigned)(blocks > 0 ? blocks : 1)), dim3(256), 0,
                       c.stream, c.sp, jrow, c.first, c.n, c.R, c.ldr, c.info);
}

// Launch on the context's stream; with profiling events set, the events are
// bound to the kernel's own dispatch.
template <typename K, typename A>
static void launch_k(const Ctx &c, K kernel, dim3 grid, dim3 block, const A &args)
{
    if (c.ev_start) hipExtLaunchKernelGGL(kernel, grid, block, 0, c.stream, c.ev_start, c.ev_stop, 0, args);
    else hipLaunchKernelGGL(kernel, grid, block, 0, c.stream, args);
}

template <typename T, int SRC, bool RR>
static void launch_csr_mv_L(const Ctx &c, CsrMvArgs &a)
{
    const dim3 grid((unsigned)c.geo.g_csr), block(512);
    // short rows go through the padded copy; without one, a lane per row
    switch (c.geo.lanes == 0 && c.ell_k == 0 ? 1 : c.geo.lanes) {
    case 0:
        // two rows per thread once every workgroup has two tiles or more
        if (c.m > 2 * (int64_t)c.geo.g_csr * MV_TILE - MV_TILE) {
            if (c.ell_k == 7) launch_k(c, k_csr_mv_ell<T, SRC, RR, 2, 7>, grid, dim3(MV_TILE), a);
            else launch_k(c, k_csr_mv_ell<T, SRC, RR, 2, ELL_K>, grid, dim3(MV_TILE), a);
        } else {
            if (c.ell_k == 7) launch_k(c, k_csr_mv_ell<T, SRC, RR, 1, 7>, grid, dim3(MV_TILE), a);
            else launch_k(c, k_csr_mv_ell<T, SRC, RR, 1, ELL_K>, grid, dim3(MV_TILE), a);
        }
        break;
    case 1: launch_k(c, k_csr_mv<T, 1, SRC, RR>, grid, block, a); break;
    case 2: launch_k(c, k_csr_mv<T, 2, SRC, RR>, grid, block, a); break;
    case 4: launch_k(c, k_csr_mv<T, 4, SRC, RR>, grid, block, a); break;
    case 8: launch_k(c, k_csr_mv<T, 8, SRC, RR>, grid, block, a); break;
    case 16: launch_k(c, k_csr_mv<T, 16, SRC, RR>, grid, block, a); break;
    case 32: launch_k(c, k_csr_mv<T, 32, SRC, RR>, grid, block, a); break;
    default: launch_k(c, k_csr_mv<T, 64, SRC, RR>, grid, block, a); break;
    }
}

// MV of the column kernel / naive second MV.  src_mode: SRC_UPD (column
// kernel, builds zt and x), SRC_VEC (after the second pass), SRC_DIV (naive
// p_j = A q_j).
template <typename T>
void launch_mv(const Ctx &c, int64_t j, int src_mode)
{
    const T *Q = (const T *)c.Q;
    if (c.is_dense) {
        DenseMvArgs a{};
        a.m = c.m; a.n = c.n_pub; a.j = j; a.A = c.A; a.lda = c.lda;
        a.info = c.info; a.R = c.R; a.ldr = c.ldr; a.sp = c.sp;
        a.rr_part = c.rr_part; a.n_rr = c.n_rr_mv; a.rr_out = c.rr_part;
        if (src_mode == SRC_UPD) {
            a.src = Q + j * c.ldq; a.qprev = j > 0 ? Q + (j - 1) * c.ldq : nullptr;
            a.y = c.xv; a.zt = c.zt;
            launch_k(c, k_dense_mv<T, DENSE_CB, SRC_UPD, true>, dim3((unsigned)c.geo.g_dense), dim3(256), a);
        } else if (src_mode == SRC_VEC) {
            a.src = c.zt; a.y = c.xv;
            launch_k(c, k_dense_mv<T, DENSE_CB, SRC_VEC, true>, dim3((unsigned)c.geo.g_dense), dim3(256), a);
        } else {
            a.src = c.zt; a.y = (T *)c.P + j * c.ldp;
            launch_k(c, k_dense_mv<T, DENSE_CB, SRC_DIV, false>, dim3((unsigned)c.geo.g_dense), dim3(256), a);
        }
    } else {
        CsrMvArgs a{};
        a.m = c.m; a.n = c.n_pub; a.j = j; a.row_ptr = c.row_ptr; a.col_idx = c.col_idx; a.vals = c.vals;
        a.ell_col = c.ell_col; a.ell_val = c.ell_val; a.tile_long = c.tile_long; a.ell_k = c.ell_k;
        a.ell_d16 = c.ell_d16; a.ell_wide = c.ell_wide;
        a.info = c.info; a.R = c.R; a.ldr = c.ldr; a.sp = c.sp;
        a.rr_part = c.rr_part; a.n_rr = c.n_rr_mv; a.rr_out = c.rr_part;
        if (src_mode == SRC_UPD) {
            a.src = Q + j * c.ldq; a.qprev = j > 0 ? Q + (j - 1) * c.ldq : nullptr;
            a.y = c.xv; a.zt = c.zt;
            launch_csr_mv_L<T, SRC_UPD, true>(c, a);
        } else if (src_mode == SRC_VEC) {
            a.src = c.zt; a.y = c.xv;
            launch_csr_mv_L<T, SRC_VEC, true>(c, a);
        } else {
            a.src = c.zt; a.y = (T *)c.P + j * c.ldp;
            launch_csr_mv_L<T, SRC_DIV, false>(c, a);
        }
    }
}

static RowArgs row_args(const Ctx &c, int64_t j)
{
    RowArgs a{};
    a.m = c.m; a.n = c.n_pub; a.j = j; a.x_from = c.x_from;
    a.pend = (c.cgs || c.no_pend) ? 0 : 1;
    a.z_in_zt = c.z_in_zt; a.Q = c.Q; a.ldq = c.ldq; a.P = c.P; a.ldp = c.ldp;
    a.X = c.X; a.ldx = c.m; a.zt = c.zt; a.R = c.R; a.ldr = c.ldr; a.info = c.info;
    a.sp = c.sp; a.rr_out = c.rr_part; a.s_part = c.s_part; a.S = c.S; a.re_lo = c.re_lo;
    return a;
}

#define AMGS_DISPATCH_U(U_, ...)                                                                  \
    switch (U_) {                                                                                 \
    case 1: { constexpr int UU = 1; __VA_ARGS__; } break;                                         \
    case 2: { constexpr int UU = 2; __VA_ARGS__; } break;                                         \
    case 4: { constexpr int UU = 4; __VA_ARGS__; } break;                                         \
    default: { constexpr int UU = 8; __VA_ARGS__; } break;                                        \
    }

#define AMGS_DISPATCH_U2(U_, ...)                                                                 \
    switch (U_) {                                                                                 \
    case 1: { constexpr int UU = 1; __VA_ARGS__; } break;                                         \
    case 2: { constexpr int UU = 2; __VA_ARGS__; } break;                                         \
    default: { constexpr int UU = 4; __VA_ARGS__; } break;                                        \
    }

template <typename T>
void launch_col_hp(const Ctx &c, int64_t j, bool reorth_a)
{
    RowArgs a = row_args(c, j);
    const dim3 grid((unsigned)c.geo.g_rows2), block(256);
    if (reorth_a) {
        const dim3 grid2((unsigned)c.geo.g_rows2, (unsigned)((j - c.re_lo + RE_GROUP - 1) / RE_GROUP));
        AMGS_DISPATCH_U2(c.geo.U2, hipLaunchKernelGGL((k_col_hp<T, UU, true>), grid2, block, 0, c.stream, a));
    } else {
        AMGS_DISPATCH_U2(c.geo.U2, hipLaunchKernelGGL((k_col_hp<T, UU, false>), grid, block, 0, c.stream, a));
    }
}

template <typename T>
void launch_reorth_a(const Ctx &c, int64_t j)
{
    RowArgs a = row_args(c, j);
    const dim3 grid((unsigned)c.geo.g_rows2, (unsigned)((j - c.re_lo + RE_GROUP - 1) / RE_GROUP)),
        block(256);
    AMGS_DISPATCH_U2(c.geo.U2, hipLaunchKernelGGL((k_reorth_a<T, UU>), grid, block, 0, c.stream, a));
}

void launch_reorth_fin(const Ctx &c, int64_t j)
{
    const int64_t blocks = (j - c.re_lo + 3) / 4;
    hipLaunchKernelGGL(k_reorth_fin, dim3((unsigned)blocks), dim3(256), 0, c.stream,
                       (const double *)c.s_part, c.geo.g_rows2, c.re_lo, j, c.S, c.R, c.ldr,
                       c.info);
}

// One row per thread: the pass reads j earlier columns per row, so the
// kernel needs many resident waves rather than several rows per thread.
template <typename T>
void launch_reorth_b(const Ctx &c, int64_t j, bool hp)
{
    RowArgs a = row_args(c, j);
    const dim3 grid((unsigned)c.geo.g_rows1), block(256);
    if (hp) hipLaunchKernelGGL((k_reorth_b<T, 1, true>), grid, block, 0, c.stream, a);
    else hipLaunchKernelGGL((k_reorth_b<T, 1, false>), grid, block, 0, c.stream, a);
}

// Column groups of the sweep: enough workgroups to fill the chip even when
// there are few row chunks; each group is a multiple of 4 columns.
static void sweep_cols(const Ctx &c, int64_t ncols, int64_t &gy, int64_t &cpw)
{
    if (ncols <= 0) {
        gy = 1;
        cpw = SWEEP_CB;
        return;
    }
    gy = (SWEEP_TARGET_WG + c.geo.g_rows - 1) / c.geo.g_rows;
    const int64_t max_gy = (ncols + SWEEP_CB - 1) / SWEEP_CB;
    if (gy > max_gy) gy = max_gy;
    if (gy < 1) gy = 1;
    cpw = (ncols + gy - 1) / gy;
    cpw = (cpw + SWEEP_CB - 1) / SWEEP_CB * SWEEP_CB;
    if (cpw > MAX_CPW) cpw = MAX_CPW;
    gy = (ncols + cpw - 1) / cpw;
}

template <typename T>
void launch_sweep(const Ctx &c, int64_t j, int variant, int64_t n_rr)
{
    SweepArgs a{};
    a.m = c.m; a.n = c.n; a.j = j; a.Q = c.Q; a.ldq = c.ldq; a.P = c.P; a.ldp = c.ldp;
    a.X = c.X; a.ldx = c.m; a.zt = c.zt; a.xv = c.xv; a.R = c.R; a.ldr = c.ldr;
    a.info = c.info; a.sp = c.sp; a.rr_part = c.rr_part; a.n_rr = n_rr;
    // a column before c.first is final: only its projections onto the new
    // columns [first, n) remain
    a.norm = j >= c.first ? 1 : 0;
    a.c_lo = j >= c.first ? j + 1 : c.first;
    int64_t gy, cpw;
    sweep_cols(c, c.n - a.c_lo, gy, cpw);
    a.cpw = cpw;
    const dim3 grid((unsigned)c.geo.g_rows, (unsigned)gy), block(256);
    // later columns that no longer fit the last-level cache are streamed with
    // non-temporal loads and stores; smaller trailing blocks stay cached for
    // the next step
    const bool nts = (double)(c.n - a.c_lo) * (double)c.m * sizeof(T) > SWEEP_NT_BYTES;
#define AMGS_SWEEP_V(V_, NT_)                                                                     \
    AMGS_DISPATCH_U(c.geo.U, if (c.ev_start) hipExtLaunchKernelGGL((k_sweep<T, UU, V_, NT_>),     \
        grid, block, 0, c.stream, c.ev_start, c.ev_stop, 0, a);                                   \
        else hipLaunchKernelGGL((k_sweep<T, UU, V_, NT_>), grid, block, 0, c.stream, a))
    if (nts) {
        if (variant == VAR_NAIVE) { AMGS_SWEEP_V(VAR_NAIVE, true); }
        else if (variant == VAR_HA) { AMGS_SWEEP_V(VAR_HA, true); }
        else { AMGS_SWEEP_V(VAR_HP, true); }
    } else {
        if (variant == VAR_NAIVE) { AMGS_SWEEP_V(VAR_NAIVE, false); }
        else if (variant == VAR_HA) { AMGS_SWEEP_V(VAR_HA, false); }
        else { AMGS_SWEEP_V(VAR_HP, false); }
    }
#undef AMGS_SWEEP_V
}

template <typename T>
bool launch_hp_xblock(const Ctx &c, int64_t s, int64_t c_from)
{
    // terms [s - HP_XB, s) on the columns c >= c_from (and >= first)
    const int64_t c_lo = c_from > c.first ? c_from : c.first;
    if (s < HP_XB || s % HP_XB != 0 || c_lo >= c.n) return false;
    const int64_t ncols = c.n - c_lo;
    const int64_t gx = (c.m + 255) / 256;
    int64_t gy = (SWEEP_TARGET_WG + gx - 1) / gx;
    const int64_t max_gy = (ncols + 3) / 4;
    if (gy > max_gy) gy = max_gy;
    if (gy < 1) gy = 1;
    int64_t cpw = (ncols + gy - 1) / gy;
    gy = (ncols + cpw - 1) / cpw;
    hipLaunchKernelGGL(k_hp_xblock<T>, dim3((unsigned)gx, (unsigned)gy), dim3(256), 0, c.stream,
                       c.m, c.n, s, c_lo, cpw, (const T *)c.P, c.ldp, (T *)c.X, c.m, c.R, c.ldr,
                       c.info);
    return true;
}

template <typename T>
void launch_csr_spmm(const Ctx &c)
{
    // the new columns [first, n) only, read from Z (the working copy in Q
    // may not hold them yet)
    const int64_t nn = c.n - c.first;
    const T *Zn = (const T *)c.Z + c.first * c.ldz;
    T *Xn = (T *)c.X + c.first * c.m;
    const int L = c.geo.lanes;
    if (L <= 1) {
        // short rows: a thread per row (entries in registers for <= 8)
        const dim3 grid((unsigned)((c.m + 255) / 256)), block(256);
        hipLaunchKernelGGL(k_csr_spmm<T>, grid, block, 0, c.stream, c.m, nn, c.nnz, c.row_ptr,
                           c.col_idx, (const T *)c.vals, Zn, c.ldz, Xn, c.m);
        return;
    }
    const int64_t rows = 256 / L;
    const dim3 grid((unsigned)((c.m + rows - 1) / rows), (unsigned)((nn + SPMM_LC - 1) / SPMM_LC));
    const dim3 block(256);
#define AMGS_SPMM_L(LL)                                                                            \
    hipLaunchKernelGGL((k_csr_spmm_lanes<T, LL>), grid, block, 0, c.stream, c.m, nn, c.row_ptr,   \
                       c.col_idx, (const T *)c.vals, Zn, c.ldz, Xn, c.m)
    switch (L) {
    case 2: AMGS_SPMM_L(2); break;
    case 4: AMGS_SPMM_L(4); break;
    case 8: AMGS_SPMM_L(8); break;
    case 16: AMGS_SPMM_L(16); break;
    case 32: AMGS_SPMM_L(32); break;
    default: AMGS_SPMM_L(64); break;
    }
#undef AMGS_SPMM_L
}

void launch_csr_check(int64_t m, int64_t nnz, const int32_t *row_ptr, const int32_t *col_idx,
                      int32_t *flag, hipStream_t s)
{
    hipLaunchKernelGGL(k_set_i32, dim3(1), dim3(1), 0, s, flag, 0);
    int64_t work = m > nnz ? m : nnz;
    int64_t blocks = (work + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(k_csr_check, dim3((unsigned)blocks), dim3(256), 0, s, m, nnz, row_ptr,
                       col_idx, flag);
}

template void launch_init<double>(const Ctx &, int64_t);
template void launch_init<float>(const Ctx &, int64_t);
template void launch_csr_to_ell<double>(const Ctx &);
template void launch_csr_to_ell<float>(const Ctx &);
template void launch_publish<double>(const Ctx &, int64_t);
template void launch_publish<float>(const Ctx &, int64_t);
template void launch_mv<double>(const Ctx &, int64_t, int);
template void launch_mv<float>(const Ctx &, int64_t, int);
template void launch_col_hp<double>(const Ctx &, int64_t, bool);
template void launch_col_hp<float>(const Ctx &, int64_t, bool);
template void launch_reorth_a<double>(const Ctx &, int64_t);
template void launch_reorth_a<float>(const Ctx &, int64_t);
template void launch_reorth_b<double>(const Ctx &, int64_t, bool);
template void launch_reorth_b<float>(const Ctx &, int64_t, bool);
template void launch_sweep<double>(const Ctx &, int64_t, int, int64_t);
template void launch_sweep<float>(const Ctx &, int64_t, int, int64_t);
template bool launch_hp_xblock<double>(const Ctx &, int64_t, int64_t);
template bool launch_hp_xblock<float>(const Ctx &, int64_t, int64_t);
template void launch_csr_spmm<double>(const Ctx &);
template void launch_csr_spmm<float>(const Ctx &);

} // namespace amgs
