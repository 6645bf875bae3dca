// amgs_panel.hip -- kernels of the panel schedule (opts->panel).
//
// Columns are taken in panels of PANEL_B.  Inside a panel every step is the
// column algorithm's (Algs. 3/5/6): the column kernel, then a sweep that
// normalises column j (eqs. (4), (10)), applies the pending update to the
// later columns of the panel and forms their dots with p_j (eq. (9)).
// After the last column of panel I a single sweep over every later column c
// applies panel I-1 as one block (its coefficients r_{I-1,c} are final in R)
// and forms W_c = P_I^T z_c; k_pfin then solves (I + L) r_{I,c} = W_c with
// L = strict_lower(P_I^T Q_I).  Since z_c^{(i-1)} = z_c - sum_{k<i} r_kc q_k,
// r_ic = p_i^T z_c^{(i-1)} = W_ic - sum_{k<i} (p_i^T q_k) r_kc: the same
// coefficients as the column algorithm in exact arithmetic, obtained with one
// pass over the later columns per panel instead of one per column.
//
// For HP the sweeps leave the x columns alone.  The recurrence of eq. (5)
// is applied as in the column schedule: after every second panel (once the
// coefficients are final) k_hp_xblock applies the last HP_XB terms to every
// later x column, and the column kernels add the terms since then, so each
// x_c receives every term once, in ascending i.  The x columns are streamed
// once per HP_XB columns instead of once per panel.
#include <hip/hip_ext.h>

#include "amgs_device.h"
#include "amgs_internal.h"

namespace amgs {

// Rows per thread of the panel kernels: each thread holds, per row, the
// pending q_k and the dot vectors p_d in registers.
template <typename T>
constexpr int panel_rows() { return sizeof(T) == 8 ? 2 : 4; }

// One step of the panel schedule.  DB = 1: a step inside a panel (dots with
// p_j only, partials in the column-schedule layout part[c * g + w]).
// DB = PANEL_B: the sweep after the last column j of a panel (dots with
// p_d, d in [d0, j], partials part[(c * PANEL_B + d - d0) * g + w]).
// Every launch also writes the partials of p_j^T q_k, k in [l0, j) (one row
// of strict_lower(P_I^T Q_I)), from the workgroups of grid row 0.
// KB: most pending columns; LB: most columns of the panel whose L row is
// formed (PANEL_B for the one-level schedule, PANEL_B1 for two levels).
template <typename T, int U, int VAR, bool NTS, int DB, int KB, int LB>
__global__ __launch_bounds__(256) void k_psweep(PSweepArgs a)
{
    constexpr int DL = DB > 1 ? DB - 1 : 1;
    static_assert(DB == 1 || DB == 4, "block dots are reduced four at a time");
    __shared__ T red[256 / WAVE][PS_MAXC * DB];
    __shared__ T lred[256 / WAVE][LB];
    __shared__ double s_rr;
    if (*a.info) return;
    const int64_t j = a.j, m = a.m;
    const int tid = threadIdx.x, wave = tid / WAVE, lane = tid & (WAVE - 1);
    T *__restrict__ Q = (T *)a.Q;
    T *__restrict__ P = (T *)a.P;
    T *__restrict__ X = (T *)a.X;
    const int64_t row0 = (int64_t)blockIdx.x * 256 * U;
    const bool own = blockIdx.y == 0;
    const int kw = (int)(a.k1 - a.k0);
    const int bd = (int)(j - a.d0 + 1);
    const T *__restrict__ zsrc = VAR == VAR_HP ? Q + j * a.ldq : (const T *)a.zt;
    const T *__restrict__ xsrc = VAR == VAR_HP ? (const T *)X + j * a.ldx : (const T *)a.xv;
    // every vector load is issued before waiting for r_jj
    T xs[U], zs[U], qk[KB][U], pd[DL][U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const int64_t k = row0 + u * 256 + tid;
        const bool in = k < m;
        xs[u] = in ? (VAR == VAR_NAIVE ? P[k + j * a.ldp] : xsrc[k]) : (T)0;
        zs[u] = (in && own) ? zsrc[k] : (T)0;
#pragma unroll
        for (int t = 0; t < KB; ++t) qk[t][u] = (in && t < kw) ? Q[k + (a.k0 + t) * a.ldq] : (T)0;
#pragma unroll
        for (int t = 0; t < DL; ++t) pd[t][u] = (in && t < bd - 1) ? P[k + (a.d0 + t) * a.ldp] : (T)0;
    }
    // q_k for the row of strict_lower(P_I^T Q_I), k in [l0, j)
    const int nl = (int)(j - a.l0);
    T ql[LB - 1][U];
#pragma unroll
    for (int i = 0; i < LB - 1; ++i)
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t k = row0 + u * 256 + tid;
            ql[i][u] = (own && i < nl && k < m) ? Q[k + (a.l0 + i) * a.ldq] : (T)0;
        }
    const int64_t c0 = a.c0 + (int64_t)blockIdx.y * a.cpw;
    const int64_t c1 = (c0 + a.cpw < a.c1) ? c0 + a.cpw : a.c1;
    const bool full_rows = row0 + 256 * U <= m;
    // the first group of later columns is requested before waiting for r_jj
    T zv[PS_CB][U];
    auto load_group = [&](int64_t cb) {
#pragma unroll
        for (int t = 0; t < PS_CB; ++t) {
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int64_t k = row0 + u * 256 + tid;
                const bool in = cb + t < c1 && (full_rows || k < m);
                zv[t][u] = in ? ld_stream<NTS>(Q + (cb + t) * a.ldq + k) : (T)0;
            }
        }
    };
    load_group(c0);
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
    T pj[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const int64_t k = row0 + u * 256 + tid;
        pj[u] = VAR == VAR_NAIVE ? xs[u] : scale_div(xs[u], rjj);
        if (own && k < m) {
            Q[k + j * a.ldq] = scale_div(zs[u], rjj);
            if (VAR != VAR_NAIVE) P[k + j * a.ldp] = pj[u];
        }
    }
    for (int64_t cb = c0; cb < c1; cb += PS_CB) {
        if (cb > c0) load_group(cb);
        // the group's pending coefficients; in binary32 they are requested
        // together (the compiler would otherwise wait for each one where it
        // is converted; a coefficient past the group or the block reads R[0],
        // unused)
        double rcd[PS_CB][KB];
        if constexpr (sizeof(T) == 4) {
#pragma unroll
            for (int t = 0; t < PS_CB; ++t)
#pragma unroll
                for (int i = 0; i < KB; ++i)
                    rcd[t][i] = ld_fix(a.R, (a.k0 + i) + (cb + t) * a.ldr, 0, cb + t < c1 && i < kw);
            pin();
        }
        T acc[PS_CB][DB];
#pragma unroll
        for (int t = 0; t < PS_CB; ++t) {
            const bool cin = cb + t < c1;
            T rc[KB];
#pragma unroll
            for (int i = 0; i < KB; ++i)
                rc[i] = sizeof(T) == 4 ? (T)rcd[t][i]
                                       : ((cin && i < kw) ? (T)a.R[(a.k0 + i) + (cb + t) * a.ldr] : (T)0);
#pragma unroll
            for (int d = 0; d < DB; ++d) acc[t][d] = 0;
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int64_t k = row0 + u * 256 + tid;
                if (!(cin && (full_rows || k < m))) continue;
                T z = zv[t][u];
                if (kw > 0) {
                    // pending terms in ascending column order
#pragma unroll
                    for (int i = 0; i < KB; ++i)
                        if (i < kw) z = upd(z, rc[i], qk[i][u]);
                    st_stream<NTS>(Q + (cb + t) * a.ldq + k, z);
                }
#pragma unroll
                for (int d = 0; d < DB; ++d) {
                    if (d == bd - 1) acc[t][d] += pj[u] * z;
                    else if (d < DL && d < bd - 1) acc[t][d] += pd[d < DL ? d : 0][u] * z;
                }
            }
        }
        if constexpr (DB == 4) {
#pragma unroll
            for (int t = 0; t < PS_CB; ++t) {
                const T v = wave_sum4(acc[t][0], acc[t][1], acc[t][2], acc[t][3]);
                if (lane < 4 && cb + t < c1 && lane < bd) red[wave][(cb - c0 + t) * DB + lane] = v;
            }
        } else {
#pragma unroll
            for (int t = 0; t < PS_CB; ++t)
#pragma unroll
                for (int d = 0; d < DB; ++d) {
                    const T v = wave_sum(acc[t][d]);
                    if (lane == 0 && cb + t < c1 && d < bd) red[wave][(cb - c0 + t) * DB + d] = v;
                }
        }
    }
    __syncthreads();
    const int ncols = c0 < c1 ? (int)(c1 - c0) : 0;
    for (int idx = tid; idx < ncols * bd; idx += 256) {
        const int cl = idx / bd, d = idx - cl * bd;
        T s = red[0][cl * DB + d];
#pragma unroll
        for (int w = 1; w < 256 / WAVE; ++w) s += red[w][cl * DB + d];
        ((T *)a.part)[((c0 + cl) * a.pstride + d) * a.g + blockIdx.x] = s;
    }
    // row j of strict_lower(P_I^T Q_I): p_j^T q_k for k in [l0, j)
    if (own && nl > 0) {
#pragma unroll
        for (int i = 0; i < LB - 1; ++i) {
            if (i < nl) {
                T s = 0;
#pragma unroll
                for (int u = 0; u < U; ++u) s += pj[u] * ql[i][u];
                s = wave_sum(s);
                if (lane == 0) lred[wave][i] = s;
            }
        }
        __syncthreads();
        if (tid < nl) {
            T s = lred[0][tid];
#pragma unroll
            for (int w = 1; w < 256 / WAVE; ++w) s += lred[w][tid];
            ((T *)a.lpart)[(nl * a.lstride + tid) * a.g + blockIdx.x] = s;
        }
    }
}

// r_{I,c} for every later column c = e + blockIdx.x: the dots W_c and the
// entries of L are re-reduced from their partials (fixed order, so every
// workgroup obtains the same L), then (I + L) r = W is solved by forward
// substitution in binary64 and r is written to R[s.., c].
template <typename T>
__global__ __launch_bounds__(16 * WAVE) void k_pfin(int64_t s, int64_t e, const T *__restrict__ wpart,
                                              const T *__restrict__ lpart, int64_t g,
                                              double *__restrict__ R, int64_t ldr,
                                              const int32_t *info)
{
    constexpr int B = PANEL_B;
    __shared__ T vals[B + B * B];
    if (*info) return;
    const int64_t c = e + blockIdx.x;
    const int b = (int)(e - s);
    const int wave = threadIdx.x / WAVE, lane = threadIdx.x & (WAVE - 1);
    // one wave per item (at most 4 + 6), all of them at once
    const int nitems = b + b * (b - 1) / 2;
    for (int it = wave; it < nitems; it += 16) {
        const T *src;
        int slot;
        if (it < b) {
            src = wpart + (c * B + it) * g;
            slot = it;
        } else {
            int q = it - b, i = 1;
            while (q >= i) {
                q -= i;
                ++i;
            }
            src = lpart + ((int64_t)i * B + q) * g;
            slot = B + i * B + q;
        }
        const T v = wave_reduce_seq_deep<16>(src, g);
        if (lane == 0) vals[slot] = v;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double r[B];
#pragma unroll
        for (int i = 0; i < B; ++i) {
            if (i < b) {
                double t = (double)vals[i];
#pragma unroll
                for (int k = 0; k < B; ++k)
                    if (k < i) t = __builtin_fma(-(double)vals[B + i * B + k], r[k], t);
                r[i] = t;
                R[(s + i) + c * ldr] = t;
            }
        }
    }
}

// First column j of a panel: z_j -= sum_k r_kj q_k over the previous panel
// [k0, k1) (coefficients final in R, ascending k); for HP also
// x_j -= sum_k r_kj p_k for the terms k >= a.x_from that no x-block pass has
// applied, both in place, and the partial of z_j^T x_j.  For naive / HA the
// corrected z_j goes to zt, from where the column MV reads it.
template <typename T, int U, int VAR, int KB>
__global__ __launch_bounds__(256) void k_pcol_blk(RowArgs a, int64_t k0, int64_t k1)
{
    constexpr bool HP = VAR == VAR_HP;
    __shared__ double lds[256 / WAVE];
    if (*a.info) return;
    const int64_t j = a.j;
    T *__restrict__ Q = (T *)a.Q;
    const T *__restrict__ P = (const T *)a.P;
    T *__restrict__ X = (T *)a.X;
    T *__restrict__ zt = (T *)a.zt;
    const int kw = (int)(k1 - k0);
    const int tid = threadIdx.x;
    const int64_t row0 = (int64_t)blockIdx.x * 256 * U;
    T r[KB];
#pragma unroll
    for (int i = 0; i < KB; ++i) r[i] = i < kw ? (T)a.R[(k0 + i) + j * a.ldr] : (T)0;
    T z[U], x[U], qv[KB][U], pv[HP ? KB : 1][U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const int64_t k = row0 + u * 256 + tid;
        const bool in = k < a.m;
        z[u] = in ? Q[k + j * a.ldq] : (T)0;
        x[u] = (HP && in) ? X[k + j * a.ldx] : (T)0;
#pragma unroll
        for (int i = 0; i < KB; ++i) {
            qv[i][u] = (in && i < kw) ? Q[k + (k0 + i) * a.ldq] : (T)0;
            if (HP) pv[i][u] = (in && i < kw && k0 + i >= a.x_from) ? P[k + (k0 + i) * a.ldp] : (T)0;
        }
    }
    double acc = 0.0;
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const int64_t k = row0 + u * 256 + tid;
        if (k >= a.m) continue;
#pragma unroll
        for (int i = 0; i < KB; ++i) {
            if (i < kw) {
                z[u] = upd(z[u], r[i], qv[i][u]);
                if (HP && k0 + i >= a.x_from) x[u] = upd(x[u], r[i], pv[i][u]);
            }
        }
        if (HP) {
            Q[k + j * a.ldq] = z[u];
            X[k + j * a.ldx] = x[u];
            acc += (double)z[u] * (double)x[u];
        } else {
            zt[k] = z[u];
        }
    }
    if (HP) {
        const double t = block_sum<double, 256>(acc, lds);
        if (tid == 0) a.rr_out[blockIdx.x] = t;
    }
}

// The coefficients of a finished block [s, s + b) for the later columns
// [c0, c1) come from the partials k_bsweep wrote (XCD order, one entry per
// row chunk) in two stages.  Stage one, k_wred: every partial row -- the
// dots W_c (row (c - c0) B + d) and then the entries of
// L = strict_lower(P_I^T Q_I) (row nW + t for the t-th entry (i, k), k < i,
// in row-major order) -- is reduced per XCD segment x, one wave per row and
// segment, into out[row * 8 + x]: the whole GPU takes part, not one
// workgroup per later column.
template <typename T, int B>
__global__ __launch_bounds__(16 * WAVE) void k_wred(const T *__restrict__ wpart,
                                                    const T *__restrict__ lpart, int64_t g,
                                                    int64_t c0, int64_t nW, int64_t nL,
                                                    T *__restrict__ out, const int32_t *info)
{
    if (*info) return;
    const int64_t r = (int64_t)blockIdx.x * 16 + threadIdx.x / WAVE;
    if (r >= nW + nL) return;
    const int x = blockIdx.y;
    const int64_t span = xcd_span(g), g8 = (g + 7) / 8;
    const T *__restrict__ row;
    if (r < nW) {
        row = wpart + ((c0 + r / B) * B + r % B) * span;
    } else {
        int q = (int)(r - nW), i = 1;
        while (q >= i) {
            q -= i;
            ++i;
        }
        row = lpart + (int64_t)(i * B + q) * span;
    }
    const T v = wave_reduce_seq(row + x * g8, (g - x + 7) / 8);
    if ((threadIdx.x & (WAVE - 1)) == 0) out[r * 8 + x] = v;
}

// Stage two: r_{[s, s+b), c} for the later column c = c0 + blockIdx.x.
// W_c and L are the eight segment sums of their rows, added in segment order
// (every workgroup forms the same L), then (I + L) r = W is solved by
// forward substitution in binary64 and r is written to R.
template <typename T, int B>
__global__ __launch_bounds__(256) void k_pfin2(int64_t s, int b, int64_t c0,
                                               const T *__restrict__ wred, int64_t nW,
                                               double *__restrict__ R, int64_t ldr,
                                               const int32_t *info)
{
    __shared__ double wv[B];
    __shared__ double lv[B * B];
    if (*info) return;
    const int64_t c = c0 + blockIdx.x;
    const int tid = threadIdx.x;
    auto seg_sum = [&](int64_t row) {
        T v = 0;
#pragma unroll
        for (int x = 0; x < 8; ++x) v += wred[row * 8 + x];
        return (double)v;
    };
    if (tid < b) wv[tid] = seg_sum((int64_t)blockIdx.x * B + tid);
    const int nl = b * (b - 1) / 2;
    for (int t = tid; t < nl; t += 256) {
        int q = t, i = 1;
        while (q >= i) {
            q -= i;
            ++i;
        }
        lv[i * B + q] = seg_sum(nW + t);
    }
    __syncthreads();
    if (tid == 0) {
        double r[B];
#pragma unroll
        for (int i = 0; i < B; ++i) {
            if (i < b) {
                double t = wv[i];
#pragma unroll
                for (int k = 0; k < B; ++k)
                    if (k < i) t = __builtin_fma(-lv[i * B + k], r[k], t);
                r[i] = t;
                R[(s + i) + c * ldr] = t;
            }
        }
    }
}

// ------------------------------------------ blocked second pass (reorth = 2)
// When an outer panel [s, s + nz) of the two-level schedule starts, its
// columns have every first-pass projection onto the columns before s.  Each
// of them gets the classical second pass against all i < s at once:
// s_ic = p_i^T z_c accumulated in binary64, z_c -= sum_i s_ic q_i in binary64
// rounded once to storage, r_ic += s_ic, and for HP x_c -= sum_i s_ic p_i.
// The dots run on the binary64 matrix cores (binary32 data is widened on
// the way in, so the products are exact and the sums binary64), on the
// tiles and LDS staging of k_bsweep: a wave owns 64 rows of the panel's
// columns and streams the earlier columns 16 at a time.  The update runs
// on the vector units (k_rb_updv).
template <typename T>
__global__ __launch_bounds__(256) void k_rb_dots(RbArgs a)
{
    typedef Mfma<double>::acc_t acc_t;
    constexpr int WR = 64, LD = WR + 4, BB = PANEL_B1, NG = RB_GROUPS;
    __shared__ double red[256 / WAVE][16 * BB];
    __shared__ __attribute__((aligned(16))) T tile[256 / WAVE][16][LD];
    if (*a.info) return;
    const int tid = threadIdx.x, wave = tid / WAVE, lane = tid & (WAVE - 1);
    const int g4 = lane >> 4, jl = lane & 15;
    const T *__restrict__ Q = (const T *)a.Q;
    const T *__restrict__ P = (const T *)a.P;
    const int64_t myrow = ((int64_t)blockIdx.x * (256 / WAVE) + wave) * WR + lane;
    const bool rin = myrow < a.m;
    const int nz = (int)a.nz;
    T(*tl)[LD] = tile[wave];
    // B operands: z_{s+l%16} at matrix row 4 (l/16) + v of each 16-row tile
#pragma unroll
    for (int c = 0; c < BB; ++c) tl[c][lane] = (rin && c < nz) ? Q[myrow + (a.s + c) * a.ldq] : (T)0;
    __syncthreads();
    double zb[4][4];
#pragma unroll
    for (int st = 0; st < 4; ++st)
#pragma unroll
        for (int v = 0; v < 4; ++v) zb[st][v] = jl < BB ? (double)tl[jl][st * 16 + 4 * g4 + v] : 0.0;
    // the earlier columns 16 at a time, NG groups per round: the next group's
    // columns are loaded while the current one's products run, and the
    // round's products stay in registers until its sums are written
    T nxt[16];
    auto load = [&](int64_t ig) {
#pragma unroll
        for (int c = 0; c < 16; ++c)
            nxt[c] = (rin && ig + c < a.s) ? P[myrow + (ig + c) * a.ldp] : (T)0;
    };
    load(0);
    for (int64_t ig0 = 0; ig0 < a.s; ig0 += 16 * NG) {
        acc_t w[NG];
#pragma unroll
        for (int q = 0; q < NG; ++q) {
            w[q] = acc_t{0, 0, 0, 0};
            const int64_t ig = ig0 + 16 * q;
            if (ig >= a.s) continue;
            __syncthreads();   // the previous group's LDS reads are done
#pragma unroll
            for (int c = 0; c < 16; ++c) tl[c][lane] = nxt[c];
            __syncthreads();
            if (ig + 16 < a.s) load(ig + 16);
#pragma unroll
            for (int st = 0; st < 4; ++st)
#pragma unroll
                for (int v = 0; v < 4; ++v)
                    w[q] = Mfma<double>::op((double)tl[jl][st * 16 + 4 * g4 + v], zb[st][v], w[q]);
        }
        // W[i, c] for i = ig + Mfma<double>::row(lane, v), c = l%16 < PANEL_B1
#pragma unroll
        for (int q = 0; q < NG; ++q) {
            const int64_t ig = ig0 + 16 * q;
            if (ig >= a.s) continue;
            __syncthreads();
#pragma unroll
            for (int v = 0; v < 4; ++v)
                if (jl < BB) red[wave][Mfma<double>::row(lane, v) * BB + jl] = w[q][v];
            __syncthreads();
            if (tid < 16 * BB) {
                const int il = tid / BB, c = tid - il * BB;
                if (ig + il < a.s && c < nz) {
                    double sum = red[0][tid];
#pragma unroll
                    for (int wv = 1; wv < 256 / WAVE; ++wv) sum += red[wv][tid];
                    ((double *)a.part)[((ig + il) * BB + c) * xcd_span(a.g) + xcd_pos(blockIdx.x, a.g)] = sum;
                }
            }
        }
    }
}

// s_ic from its partials (one wave each, fixed order; stored in XCD order),
// kept for the update and added into R.
__global__ __launch_bounds__(256) void k_rb_fin(RbArgs a, double *__restrict__ R, int64_t ldr)
{
    if (*a.info) return;
    const int64_t idx = (int64_t)blockIdx.x * (256 / WAVE) + threadIdx.x / WAVE;
    const int nz = (int)a.nz;
    if (idx >= a.s * nz) return;
    const int64_t i = idx / nz, c = idx - i * nz;
    const double v = wave_reduce_xcd((const double *)a.part + (i * PANEL_B1 + c) * xcd_span(a.g), a.g);
    if ((threadIdx.x & (WAVE - 1)) == 0) {
        ((double *)a.S)[i * PANEL_B1 + c] = v;
        R[i + (a.s + c) * ldr] += v;
    }
}

// z_c (HP: and x_c) -= sum_{i < s} s_ic q_i (p_i), binary64 accumulation
// rounded once to storage, on the vector units: one row per thread, the
// panel's columns in binary64 registers, the earlier columns streamed
// sixteen at a time with every coefficient s_ic a wave-uniform operand.
// Each earlier element is used by eight fused multiply-adds (one per panel
// column), so no product is wasted (on the 16x16x4 matrix cores half of
// them would be), and the kernel needs neither LDS nor barriers.  The
// loads are unconditional (a column index past the end is clamped, its
// value dropped by a select or a uniform test) so that they are all in
// flight together.
template <typename T, bool HP, bool FULL>
__device__ __forceinline__ void rb_updv_group(const T *__restrict__ Q, int64_t ldq,
                                              const T *__restrict__ P, int64_t ldp,
                                              const double *__restrict__ S, int64_t row,
                                              int64_t ib, int64_t s, double (&z)[PANEL_B1],
                                              double (&x)[PANEL_B1])
{
    constexpr int BB = PANEL_B1, G = 16;
    T qv[G], pv[HP ? G : 1];
#pragma unroll
    for (int t = 0; t < G; ++t) {
        const int64_t i = FULL ? ib + t : (ib + t < s ? ib + t : s - 1);
        qv[t] = Q[row + i * ldq];
        if (HP) pv[HP ? t : 0] = P[row + i * ldp];
    }
#pragma unroll
    for (int t = 0; t < G; ++t) {
        if (FULL || ib + t < s) {
            const double qd = (double)qv[t];
            const double pd = HP ? (double)pv[HP ? t : 0] : 0.0;
#pragma unroll
            for (int c = 0; c < BB; ++c) {
                const double sc = S[(ib + t) * BB + c];
                z[c] = __builtin_fma(-sc, qd, z[c]);
                if (HP) x[c] = __builtin_fma(-sc, pd, x[c]);
            }
        }
    }
}

template <typename T, bool HP>
__global__ __launch_bounds__(256) void k_rb_updv(RbArgs a)
{
    constexpr int BB = PANEL_B1, G = 16;
    if (*a.info) return;
    const int64_t row = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (row >= a.m) return;
    T *__restrict__ Q = (T *)a.Q;
    const T *__restrict__ P = (const T *)a.P;
    T *__restrict__ X = (T *)a.X;
    const int nz = (int)a.nz;
    const int64_t s = a.s;
    double z[BB], x[BB];
#pragma unroll
    for (int c = 0; c < BB; ++c) {
        const int64_t cc = s + (c < nz ? c : nz - 1);
        const T zv = Q[row + cc * a.ldq];
        const T xv = HP ? X[row + cc * a.ldx] : (T)0;
        z[c] = c < nz ? (double)zv : 0.0;
        x[c] = (HP && c < nz) ? (double)xv : 0.0;
    }
    int64_t ib = 0;
    for (; ib + G <= s; ib += G)
        rb_updv_group<T, HP, true>(Q, a.ldq, P, a.ldp, a.S, row, ib, s, z, x);
    if (ib < s) rb_updv_group<T, HP, false>(Q, a.ldq, P, a.ldp, a.S, row, ib, s, z, x);
#pragma unroll
    for (int c = 0; c < BB; ++c)
        if (c < nz) {
            Q[row + (s + c) * a.ldq] = (T)z[c];
            if (HP) X[row + (s + c) * a.ldx] = (T)x[c];
        }
}

// ------------------------------------------------------------- launchers
template <typename T>
void launch_psweep(const Ctx &c, int variant, int64_t j, int64_t k0, int64_t k1, int64_t d0,
                   int64_t l0, int64_t c0, int64_t c1, int64_t n_rr)
{
    constexpr int U = panel_rows<T>();
    PSweepArgs a{};
    a.m = c.m; a.n = c.n; a.j = j; a.Q = c.Q; a.ldq = c.ldq; a.P = c.P; a.ldp = c.ldp;
    a.X = c.X; a.ldx = c.m; a.zt = c.zt; a.xv = c.xv; a.R = c.R; a.ldr = c.ldr;
    a.info = c.info; a.rr_part = c.rr_part; a.n_rr = n_rr;
    a.k0 = k0; a.k1 = k1; a.d0 = d0; a.l0 = l0; a.c0 = c0; a.c1 = c1 > c0 ? c1 : c0;
    const bool block_dots = d0 < j;
    a.part = block_dots ? c.wpart : c.sp.part;
    a.pstride = block_dots ? PANEL_B : 1;
    a.g = c.g_p;
    a.lpart = c.lpart;
    // a pending block wider than PANEL_B (the previous outer panel) needs the
    // wider kernel; every other step uses the one-level kernels
    const bool two = k1 - k0 > PANEL_B;
    a.lstride = PANEL_B;
    const int64_t ncols = a.c1 - a.c0;
    int64_t gy = 1, cpw = PS_CB;
    if (ncols > 0) {
        gy = (SWEEP_TARGET_WG + c.g_p - 1) / c.g_p;
        const int64_t max_gy = (ncols + PS_CB - 1) / PS_CB;
        if (gy > max_gy) gy = max_gy;
        if (gy < 1) gy = 1;
        cpw = (ncols + gy - 1) / gy;
        cpw = (cpw + PS_CB - 1) / PS_CB * PS_CB;
        if (cpw > PS_MAXC) cpw = PS_MAXC;
        gy = (ncols + cpw - 1) / cpw;
    }
    a.cpw = cpw;
    const dim3 grid((unsigned)c.g_p, (unsigned)gy), block(256);
    const bool nts = (double)ncols * (double)c.m * sizeof(T) > SWEEP_NT_BYTES;
#define AMGS_PS_LAUNCH2(V_, NT_, DB_, KB_)                                                       \
    do {                                                                                          \
        if (c.ev_start)                                                                           \
            hipExtLaunchKernelGGL((k_psweep<T, U, V_, NT_, DB_, KB_, PANEL_B>), grid, block, 0,   \
                                  c.stream, c.ev_start, c.ev_stop, 0, a);                         \
        else                                                                                      \
            hipLaunchKernelGGL((k_psweep<T, U, V_, NT_, DB_, KB_, PANEL_B>), grid, block, 0,      \
                               c.stream, a);                                                      \
    } while (0)
#define AMGS_PS_LAUNCH(V_, NT_, DB_)                                                              \
    do {                                                                                          \
        if (two) AMGS_PS_LAUNCH2(V_, NT_, DB_, PANEL_B1);                                         \
        else AMGS_PS_LAUNCH2(V_, NT_, DB_, PANEL_B);                                              \
    } while (0)
#define AMGS_PS_DB(V_, NT_)                                                                       \
    do {                                                                                          \
        if (block_dots) AMGS_PS_LAUNCH(V_, NT_, PANEL_B);                                         \
        else AMGS_PS_LAUNCH(V_, NT_, 1);                                                          \
    } while (0)
#define AMGS_PS_NT(V_)                                                                            \
    do {                                                                                          \
        if (nts) AMGS_PS_DB(V_, true);                                                            \
        else AMGS_PS_DB(V_, false);                                                               \
    } while (0)
    if (variant == VAR_NAIVE) AMGS_PS_NT(VAR_NAIVE);
    else if (variant == VAR_HA) AMGS_PS_NT(VAR_HA);
    else AMGS_PS_NT(VAR_HP);
#undef AMGS_PS_NT
#undef AMGS_PS_DB
#undef AMGS_PS_LAUNCH
#undef AMGS_PS_LAUNCH2
}

template <typename T>
void launch_pfin(const Ctx &c, int64_t s, int64_t e, int64_t c1)
{
    if (e >= c1) return;
    hipLaunchKernelGGL(k_pfin<T>, dim3((unsigned)(c1 - e)), dim3(16 * WAVE), 0, c.stream, s, e,
                       (const T *)c.wpart, (const T *)c.lpart, c.g_p, c.R, c.ldr, c.info);
}

// The block's coefficients for the later columns [c0, c1): k_wred, then
// k_pfin2 (two launches).
template <typename T, int B>
static void launch_pfin2_b(const Ctx &c, int64_t s, int64_t e, int64_t c0, int64_t c1)
{
    const int b = (int)(e - s);
    const int64_t nW = (c1 - c0) * B, nL = (int64_t)b * (b - 1) / 2;
    const dim3 gw((unsigned)((nW + nL + 15) / 16), 8);
    hipLaunchKernelGGL((k_wred<T, B>), gw, dim3(16 * WAVE), 0, c.stream, (const T *)c.wpart,
                       (const T *)c.lpart8, c.g_b, c0, nW, nL, (T *)c.wred, c.info);
    hipLaunchKernelGGL((k_pfin2<T, B>), dim3((unsigned)(c1 - c0)), dim3(256), 0, c.stream, s, b, c0,
                       (const T *)c.wred, nW, c.R, c.ldr, c.info);
}

template <typename T>
void launch_pfin2(const Ctx &c, int64_t s, int64_t e, int64_t c0, int64_t c1, int bb)
{
    if (c1 <= c0) return;
    if (bb == PANEL_B2) launch_pfin2_b<T, PANEL_B2>(c, s, e, c0, c1);
    else launch_pfin2_b<T, PANEL_B1>(c, s, e, c0, c1);
}

// The blocked second pass of the outer panel [s, e) against the columns
// before s (reorth = 2).
template <typename T>
void launch_rb(const Ctx &c, int64_t s, int64_t e, int variant)
{
    if (s <= 0 || e <= s) return;
    RbArgs a{};
    a.m = c.m; a.Q = c.Q; a.ldq = c.ldq; a.P = c.P; a.ldp = c.ldp; a.X = c.X; a.ldx = c.m;
    a.s = s; a.nz = e - s; a.part = c.rb_part; a.g = c.g_b; a.S = c.rb_s; a.info = c.info;
    const dim3 grid((unsigned)c.g_b), block(256);
    hipLaunchKernelGGL(k_rb_dots<T>, grid, block, 0, c.stream, a);
    const int64_t waves = s * (e - s);
    hipLaunchKernelGGL(k_rb_fin, dim3((unsigned)((waves + 3) / 4)), block, 0, c.stream, a, c.R,
                       c.ldr);
    const dim3 gv((unsigned)((c.m + 255) / 256));
    if (variant == VAR_HP) hipLaunchKernelGGL((k_rb_updv<T, true>), gv, block, 0, c.stream, a);
    else hipLaunchKernelGGL((k_rb_updv<T, false>), gv, block, 0, c.stream, a);
}

int64_t pcol_blk_partials(const Ctx &c) { return c.geo.g_rows2; }

template <typename T>
void launch_pcol_blk(const Ctx &c, int variant, int64_t j, int64_t k0, int64_t k1, int64_t xk0)
{
    RowArgs a{};
    a.m = c.m; a.n = c.n; a.j = j; a.Q = c.Q; a.ldq = c.ldq; a.P = c.P; a.ldp = c.ldp;
    a.X = c.X; a.ldx = c.m; a.zt = c.zt; a.R = c.R; a.ldr = c.ldr; a.info = c.info;
    a.sp = c.sp; a.rr_out = c.rr_part; a.x_from = xk0;
    const dim3 grid((unsigned)c.geo.g_rows2), block(256);
#define AMGS_PCB2(V_, KB_)                                                                        \
    switch (c.geo.U2) {                                                                           \
    case 1: hipLaunchKernelGGL((k_pcol_blk<T, 1, V_, KB_>), grid, block, 0, c.stream, a, k0, k1); break; \
    case 2: hipLaunchKernelGGL((k_pcol_blk<T, 2, V_, KB_>), grid, block, 0, c.stream, a, k0, k1); break; \
    default: hipLaunchKernelGGL((k_pcol_blk<T, 4, V_, KB_>), grid, block, 0, c.stream, a, k0, k1); break; \
    }
#define AMGS_PCB(V_)                                                                              \
    do {                                                                                          \
        if (k1 - k0 > PANEL_B) { AMGS_PCB2(V_, PANEL_B1); }                                       \
        else { AMGS_PCB2(V_, PANEL_B); }                                                          \
    } while (0)
    if (variant == VAR_HP) { AMGS_PCB(VAR_HP); }
    else { AMGS_PCB(VAR_HA); }
#undef AMGS_PCB
#undef AMGS_PCB2
}

template void launch_psweep<double>(const Ctx &, int, int64_t, int64_t, int64_t, int64_t, int64_t,
                                    int64_t, int64_t, int64_t);
template void launch_psweep<float>(const Ctx &, int, int64_t, int64_t, int64_t, int64_t, int64_t,
                                   int64_t, int64_t, int64_t);
template void launch_pfin<double>(const Ctx &, int64_t, int64_t, int64_t);
template void launch_pfin2<double>(const Ctx &, int64_t, int64_t, int64_t, int64_t, int);
template void launch_pfin2<float>(const Ctx &, int64_t, int64_t, int64_t, int64_t, int);
template void launch_rb<double>(const Ctx &, int64_t, int64_t, int);
template void launch_rb<float>(const Ctx &, int64_t, int64_t, int);
template void launch_pfin<float>(const Ctx &, int64_t, int64_t, int64_t);
template void launch_pcol_blk<double>(const Ctx &, int, int64_t, int64_t, int64_t, int64_t);
template void launch_pcol_blk<float>(const Ctx &, int, int64_t, int64_t, int64_t, int64_t);

int panel_rows_for(int fp64) { return fp64 ? panel_rows<double>() : panel_rows<float>(); }

} // namespace amgs
