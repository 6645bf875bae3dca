// amgs_batched.hip -- many independent A-orthonormalisations in one
// persistent launch (the single-problem computation of Alg. 3 / 5 / 6 per
// instance, one workgroup per instance, every reduction inside the
// workgroup).
//
// Column order.  An instance is processed left-looking in blocks of B
// columns held in registers: for every earlier column i the workgroup streams
// p_i and q_i once, forms the B dots p_i^T z_c with one workgroup reduction,
// and applies z_c -= r_ic q_i (HP also x_c -= r_ic p_i).  The block's own
// columns are then finished right-looking.  Each column therefore receives
// exactly the updates of the column algorithm in ascending i, while p_i and
// q_i are read once per block instead of once per column.
//
// Work list.  Instances are taken largest-first (cost m n^2) from an atomic
// counter; every workgroup leaves when the list is exhausted, so the grid
// always drains.  The counter is reset by a one-thread kernel in the same
// graph (no memset node).
#include "amgs_batched.h"
#include "amgs_device.h"
#include "amgs_internal.h"

#include <algorithm>
#include <cmath>
#include <new>
#include <vector>

namespace amgs {

template <typename A>
__device__ __forceinline__ void bt_zero(A *v, int n)
{
    for (int i = threadIdx.x; i < n; i += BT_NT) v[i] = 0;
}

// Sum NV per-thread values across the workgroup (only the first nv <= NV
// are used) with a single barrier: each wave's DPP sum goes to LDS slot
// buffer `buf` (callers alternate 0/1 between consecutive reductions, so a
// slot is never rewritten while another thread may still read it), then
// every thread adds the wave sums in wave order.  out[v] receives the sum of
// value v in every thread (registers, no second barrier).
template <typename A, int NV>
__device__ __forceinline__ void bt_reduce(const A (&vals)[NV], int nv, A (*red)[BT_NT / WAVE][BT_RED],
                                          int &buf, A (&out)[NV])
{
    const int lane = threadIdx.x & (WAVE - 1), wave = threadIdx.x / WAVE;
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        if (v < nv) {
            A s = wave_sum(vals[v]);
            if (lane == 0) red[buf][wave][v] = s;
        }
    }
    __syncthreads();
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        A s = 0;
        if (v < nv) {
            s = red[buf][0][v];
#pragma unroll
            for (int w = 1; w < BT_NT / WAVE; ++w) s += red[buf][w][v];
        }
        out[v] = s;
    }
    buf ^= 1;
}

template <typename T, int VAR, int BMAX>
__global__ __launch_bounds__(BT_NT) void k_batched(const amgs_batch_desc_t *__restrict__ desc,
                                                   const BatchItem *__restrict__ items,
                                                   int32_t count, T *__restrict__ work,
                                                   int32_t *__restrict__ info,
                                                   uint32_t *__restrict__ counter, int reorth)
{
    __shared__ T vec[BT_MAX_M];                 // one column for the in-workgroup MV
    __shared__ T redT[2][BT_NT / WAVE][BT_RED];
    __shared__ double redD[2][BT_NT / WAVE][BT_RED];
    __shared__ int32_t s_idx;
    const int tid = threadIdx.x;
    int bufT = 0, bufD = 0;

    for (;;) {
        if (tid == 0) s_idx = (int32_t)atomicAdd(counter, 1u);
        __syncthreads();
        const int32_t idx = s_idx;
        __syncthreads();
        if (idx >= count) break;
        const BatchItem it = items[idx];
        const amgs_batch_desc_t d = desc[it.k];
        const int64_t m = d.m, n = d.n, ldq = d.ldq, ldr = d.ldr, ldz = d.ldz;
        const int32_t *__restrict__ rp = d.row_ptr;
        const int32_t *__restrict__ ci = d.col_idx;
        const T *__restrict__ av = (const T *)d.vals;
        const T *__restrict__ Z = (const T *)d.Z;
        T *__restrict__ Q = (T *)d.Q;
        double *__restrict__ R = d.R;
        T *__restrict__ P = work + it.ws;                   // m x n, ld m
        T *__restrict__ X = P + m * n;                      // HP: m x n, ld m
        const int B = it.B < 1 ? 1 : (it.B > BMAX ? BMAX : it.B);

        for (int64_t e = tid; e < n * n; e += BT_NT) R[(e % n) + (e / n) * ldr] = 0.0;
        // HP block product X = A Z, then Q <- Z (Z may alias Q)
        if (VAR == VAR_HP) {
            for (int64_t c = 0; c < n; ++c) {
#pragma unroll
                for (int u = 0; u < BT_RPT; ++u) {
                    const int64_t r = tid + u * BT_NT;
                    if (r < m) {
                        T s = 0;
                        for (int32_t e = rp[r]; e < rp[r + 1]; ++e) s += av[e] * Z[ci[e] + c * ldz];
                        X[r + c * m] = s;
                    }
                }
            }
            __syncthreads();
        }
        bool broke = false;
        for (int64_t j0 = 0; j0 < n && !broke; j0 += B) {
            const int bw = (int)(n - j0 < B ? n - j0 : B);
            T zb[BMAX][BT_RPT], xb[VAR == VAR_HP ? BMAX : 1][BT_RPT];
#pragma unroll
            for (int b = 0; b < BMAX; ++b)
#pragma unroll
                for (int u = 0; u < BT_RPT; ++u) {
                    const int64_t r = tid + u * BT_NT;
                    const bool in = b < bw && r < m;
                    zb[b][u] = in ? Z[r + (j0 + b) * ldz] : (T)0;
                    if (VAR == VAR_HP) xb[b][u] = in ? X[r + (j0 + b) * m] : (T)0;
                }
            // earlier columns, i ascending: one reduction of bw dots per i.
            // The loads of p_{i+1}, q_{i+1} are issued before the reduction,
            // except in binary32 once the block (z, and x for HP) holds 4 or
            // more columns: there the registers they take cost a wave per
            // SIMD or more than the overlap gains, while in binary64 the
            // overlap pays even where it spills.
            constexpr bool PF = (BMAX * (VAR == VAR_HP ? 2 : 1) < 4) || sizeof(T) == 8;
            T pn[PF ? BT_RPT : 1], qn[PF ? BT_RPT : 1];
            if (PF) {
#pragma unroll
                for (int u = 0; u < BT_RPT; ++u) {
                    const int64_t r = tid + u * BT_NT;
                    pn[PF ? u : 0] = (j0 > 0 && r < m) ? P[r] : (T)0;
                    qn[PF ? u : 0] = (j0 > 0 && r < m) ? Q[r] : (T)0;
                }
            }
            for (int64_t i = 0; i < j0; ++i) {
                T pr[BT_RPT], qr[BT_RPT], dots[BMAX], rvals[BMAX];
#pragma unroll
                for (int u = 0; u < BT_RPT; ++u) {
                    const int64_t r = tid + u * BT_NT;
                    if (PF) {
                        pr[u] = pn[PF ? u : 0];
                        qr[u] = qn[PF ? u : 0];
                        pn[PF ? u : 0] = (i + 1 < j0 && r < m) ? P[r + (i + 1) * m] : (T)0;
                        qn[PF ? u : 0] = (i + 1 < j0 && r < m) ? Q[r + (i + 1) * ldq] : (T)0;
                    } else {
                        pr[u] = r < m ? P[r + i * m] : (T)0;
                        qr[u] = r < m ? Q[r + i * ldq] : (T)0;
                    }
                }
#pragma unroll
                for (int b = 0; b < BMAX; ++b) {
                    T s = 0;
#pragma unroll
                    for (int u = 0; u < BT_RPT; ++u) s += pr[u] * zb[b][u];
                    dots[b] = s;
                }
                bt_reduce<T, BMAX>(dots, bw, redT, bufT, rvals);
#pragma unroll
                for (int b = 0; b < BMAX; ++b) {
                    if (b < bw) {
                        const T rib = rvals[b];
#pragma unroll
                        for (int u = 0; u < BT_RPT; ++u) {
                            zb[b][u] = upd(zb[b][u], rib, qr[u]);
                            if (VAR == VAR_HP) xb[b][u] = upd(xb[b][u], rib, pr[u]);
                        }
                        if (tid == 0) R[i + (j0 + b) * ldr] = (double)rib;
                    }
                }
            }
            // the block's own columns, right-looking
#pragma unroll
            for (int b = 0; b < BMAX; ++b) {
                if (b >= bw || broke) continue;
                const int64_t j = j0 + b;
                if (reorth && j > 0) {
                    // second pass: s_i = p_i^T z_j (binary64), z_j -= sum s_i q_i,
                    // HP x_j -= sum s_i p_i, r_ij += s_i; BT_RED coefficients at a time
                    double zd[BT_RPT], xd[BT_RPT];
#pragma unroll
                    for (int u = 0; u < BT_RPT; ++u) {
                        zd[u] = (double)zb[b][u];
                        xd[u] = VAR == VAR_HP ? (double)xb[b][u] : 0.0;
                    }
                    for (int64_t i0 = 0; i0 < j; i0 += BT_RED) {
                        const int ni = (int)(j - i0 < BT_RED ? j - i0 : BT_RED);
                        double sp[BT_RED];
#pragma unroll
                        for (int t = 0; t < BT_RED; ++t) {
                            double sacc = 0.0;
                            if (t < ni) {
#pragma unroll
                                for (int u = 0; u < BT_RPT; ++u) {
                                    const int64_t r = tid + u * BT_NT;
                                    if (r < m) sacc += (double)P[r + (i0 + t) * m] * (double)zb[b][u];
                                }
                            }
                            sp[t] = sacc;
                        }
                        double sv[BT_RED];
                        bt_reduce<double, BT_RED>(sp, ni, redD, bufD, sv);
#pragma unroll
                        for (int t = 0; t < BT_RED; ++t) {
                            if (t < ni) {
                                const double sc = sv[t];
#pragma unroll
                                for (int u = 0; u < BT_RPT; ++u) {
                                    const int64_t r = tid + u * BT_NT;
                                    if (r < m) {
                                        zd[u] -= sc * (double)Q[r + (i0 + t) * ldq];
                                        if (VAR == VAR_HP) xd[u] -= sc * (double)P[r + (i0 + t) * m];
                                    }
                                }
                                if (tid == 0) R[(i0 + t) + j * ldr] += sc;
                            }
                        }
                    }
#pragma unroll
                    for (int u = 0; u < BT_RPT; ++u) {
                        zb[b][u] = (T)zd[u];
                        if (VAR == VAR_HP) xb[b][u] = (T)xd[u];
                    }
                }
                // x_j: MV through LDS (naive, HA) or the recurrence result (HP)
                T xr[BT_RPT];
                if (VAR == VAR_HP) {
#pragma unroll
                    for (int u = 0; u < BT_RPT; ++u) xr[u] = xb[b][u];
                } else {
#pragma unroll
                    for (int u = 0; u < BT_RPT; ++u) {
                        const int64_t r = tid + u * BT_NT;
                        if (r < m) vec[r] = zb[b][u];
                    }
                    __syncthreads();
#pragma unroll
                    for (int u = 0; u < BT_RPT; ++u) {
                        const int64_t r = tid + u * BT_NT;
                        T s = 0;
                        if (r < m)
                            for (int32_t e = rp[r]; e < rp[r + 1]; ++e) s += av[e] * vec[ci[e]];
                        xr[u] = s;
                    }
                    __syncthreads();
                }
                double nrm[1];
                nrm[0] = 0.0;
#pragma unroll
                for (int u = 0; u < BT_RPT; ++u) nrm[0] += (double)zb[b][u] * (double)xr[u];
                double rrv[1];
                bt_reduce<double, 1>(nrm, 1, redD, bufD, rrv);
                const double rr = rrv[0];
                if (!norm_ok(rr)) {
                    if (tid == 0) info[it.k] = (int32_t)(j + 1);
                    broke = true;
                    continue;
                }
                const double rjj = sqrt(rr);
                if (tid == 0) R[j + j * ldr] = rjj;
                T qv[BT_RPT], pv[BT_RPT];
#pragma unroll
                for (int u = 0; u < BT_RPT; ++u) {
                    const int64_t r = tid + u * BT_NT;
                    qv[u] = scale_div(zb[b][u], rjj);
                    if (r < m) Q[r + j * ldq] = qv[u];
                }
                if (VAR == VAR_NAIVE) {
                    // second MV: p_j = A q_j
#pragma unroll
                    for (int u = 0; u < BT_RPT; ++u) {
                        const int64_t r = tid + u * BT_NT;
                        if (r < m) vec[r] = qv[u];
                    }
                    __syncthreads();
#pragma unroll
                    for (int u = 0; u < BT_RPT; ++u) {
                        const int64_t r = tid + u * BT_NT;
                        T s = 0;
                        if (r < m)
                            for (int32_t e = rp[r]; e < rp[r + 1]; ++e) s += av[e] * vec[ci[e]];
                        pv[u] = s;
                    }
                    __syncthreads();
                } else {
#pragma unroll
                    for (int u = 0; u < BT_RPT; ++u) pv[u] = scale_div(xr[u], rjj);
                }
#pragma unroll
                for (int u = 0; u < BT_RPT; ++u) {
                    const int64_t r = tid + u * BT_NT;
                    if (r < m) P[r + j * m] = pv[u];
                }
                // project the block's later columns on q_j
                if (b + 1 < bw) {
                    T dots[BMAX];
#pragma unroll
                    for (int c = 0; c < BMAX; ++c) {
                        T s = 0;
                        if (c > b && c < bw) {
#pragma unroll
                            for (int u = 0; u < BT_RPT; ++u) s += pv[u] * zb[c][u];
                        }
                        dots[c] = s;
                    }
                    T rv[BMAX];
                    bt_reduce<T, BMAX>(dots, bw, redT, bufT, rv);
#pragma unroll
                    for (int c = 0; c < BMAX; ++c) {
                        if (c > b && c < bw) {
                            const T rjc = rv[c];
#pragma unroll
                            for (int u = 0; u < BT_RPT; ++u) {
                                zb[c][u] = upd(zb[c][u], rjc, qv[u]);
                                if (VAR == VAR_HP) xb[c][u] = upd(xb[c][u], rjc, pv[u]);
                            }
                            if (tid == 0) R[j + (j0 + c) * ldr] = (double)rjc;
                        }
                    }
                }
            }
            // P and Q of this block are read by later blocks
            __syncthreads();
        }
        if (!broke && tid == 0) info[it.k] = 0;
    }
}

__global__ void k_reset_counter(uint32_t *c) { *c = 0u; }

template <typename T, int VAR, int BMAX>
static void launch_t(int grid, const amgs_batch_desc_t *desc, const BatchItem *items,
                     int32_t count, void *work, int32_t *info, uint32_t *counter, int reorth,
                     hipStream_t s)
{
    hipLaunchKernelGGL((k_batched<T, VAR, BMAX>), dim3(grid), dim3(BT_NT), 0, s, desc, items,
                       count, (T *)work, info, counter, reorth);
}

// Widest tile compiled for a variant: HP keeps two register blocks (z and
// x), so its limit is lower, to stay clear of register spills.
static int max_tile(int variant) { return variant == VAR_HP ? BT_TILE_HP : BT_TILE_HA; }

template <int VAR> constexpr int tile_cap() { return VAR == VAR_HP ? BT_TILE_HP : BT_TILE_HA; }
template <int B, int CAP> constexpr int tile_clip() { return B < CAP ? B : CAP; }

template <typename T, int VAR>
static void launch_v(int bmax, int grid, const amgs_batch_desc_t *desc, const BatchItem *items,
                     int32_t count, void *work, int32_t *info, uint32_t *counter, int reorth,
                     hipStream_t s)
{
    constexpr int CAP = tile_cap<VAR>();
    if (bmax <= 1) launch_t<T, VAR, 1>(grid, desc, items, count, work, info, counter, reorth, s);
    else if (bmax <= 2) launch_t<T, VAR, tile_clip<2, CAP>()>(grid, desc, items, count, work, info, counter, reorth, s);
    else if (bmax <= 4) launch_t<T, VAR, tile_clip<4, CAP>()>(grid, desc, items, count, work, info, counter, reorth, s);
    else launch_t<T, VAR, tile_clip<8, CAP>()>(grid, desc, items, count, work, info, counter, reorth, s);
}

void launch_batched(int precision, int variant, int bmax, int reorth, int grid,
                    const amgs_batch_desc_t *desc, const BatchItem *items, int32_t count,
                    void *work, int32_t *info, uint32_t *counter, hipStream_t s)
{
    hipLaunchKernelGGL(k_reset_counter, dim3(1), dim3(1), 0, s, counter);
    if (precision == AMGS_FP64) {
        if (variant == VAR_NAIVE) launch_v<double, VAR_NAIVE>(bmax, grid, desc, items, count, work, info, counter, reorth, s);
        else if (variant == VAR_HA) launch_v<double, VAR_HA>(bmax, grid, desc, items, count, work, info, counter, reorth, s);
        else launch_v<double, VAR_HP>(bmax, grid, desc, items, count, work, info, counter, reorth, s);
    } else {
        if (variant == VAR_NAIVE) launch_v<float, VAR_NAIVE>(bmax, grid, desc, items, count, work, info, counter, reorth, s);
        else if (variant == VAR_HA) launch_v<float, VAR_HA>(bmax, grid, desc, items, count, work, info, counter, reorth, s);
        else launch_v<float, VAR_HP>(bmax, grid, desc, items, count, work, info, counter, reorth, s);
    }
}

template <typename T, int VAR, int BMAX>
static int occ_t()
{
    int blocks = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, k_batched<T, VAR, BMAX>, BT_NT, 0) != hipSuccess)
        return 1;
    return blocks > 0 ? blocks : 1;
}

template <typename T, int VAR>
static int occ_v(int bmax)
{
    constexpr int CAP = tile_cap<VAR>();
    return bmax <= 1 ? occ_t<T, VAR, 1>()
         : bmax <= 2 ? occ_t<T, VAR, tile_clip<2, CAP>()>()
         : bmax <= 4 ? occ_t<T, VAR, tile_clip<4, CAP>()>() : occ_t<T, VAR, tile_clip<8, CAP>()>();
}

int batched_resident_wgs(int device, int precision, int variant, int bmax)
{
    hipDeviceProp_t prop;
    int cus = 256;
    if (hipGetDeviceProperties(&prop, device) == hipSuccess) cus = prop.multiProcessorCount;
    int per;
    if (precision == AMGS_FP64)
        per = variant == VAR_NAIVE ? occ_v<double, VAR_NAIVE>(bmax)
            : variant == VAR_HA ? occ_v<double, VAR_HA>(bmax) : occ_v<double, VAR_HP>(bmax);
    else
        per = variant == VAR_NAIVE ? occ_v<float, VAR_NAIVE>(bmax)
            : variant == VAR_HA ? occ_v<float, VAR_HA>(bmax) : occ_v<float, VAR_HP>(bmax);
    return cus * per;
}

} // namespace amgs

// ====================================================================
// Plan, autotuner and graph (host)
// ====================================================================
#include "amgs_handle.h"

struct amgs_batch_plan {
    amgs_handle_t h;
    int32_t batch;
    int variant, precision, reorth;
    std::vector<int64_t> m, n;
    std::vector<amgs::BatchItem> items;   // host copy, largest-first
    amgs::BatchItem *d_items;
    uint32_t *d_counter;
    size_t ws_bytes;
    int bmax;
    int grid;
    int class_B[amgs::BT_NCLASS];
    // cached graph for one (desc, work, info); it replays on any stream
    hipStream_t cap_stream;
    // recorded after every launch: the next launch (on whatever stream) waits
    // for it, so two passes never share the work-queue counter at once
    hipEvent_t done;
    int launched;
    hipGraph_t graph;
    hipGraphExec_t exec;
    const void *g_desc;
    void *g_work;
    int32_t *g_info;
};

namespace {

using namespace amgs;

struct DevGuard {
    int prev = -1;
    explicit DevGuard(int dev)
    {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        if (prev != dev) (void)hipSetDevice(dev);
    }
    ~DevGuard()
    {
        int cur = -1;
        if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
    }
};

// Default tile per size class when not autotuning: wide blocks pay off once
// an instance has many columns.
int default_B(int cls, int variant)
{
    const bool wide_n = cls & 1;
    if (!wide_n) return 2;
    return variant == VAR_HP ? 2 : 4;
}

// Lay out the work list: largest-first by m n^2, workspace offsets, tiles.
void build_items(amgs_batch_plan *pl)
{
    const size_t w = pl->precision == AMGS_FP64 ? 8 : 4;
    std::vector<int32_t> ord(pl->batch);
    for (int32_t k = 0; k < pl->batch; ++k) ord[k] = k;
    std::stable_sort(ord.begin(), ord.end(), [&](int32_t a, int32_t b) {
        const double ca = (double)pl->m[a] * pl->n[a] * pl->n[a];
        const double cb = (double)pl->m[b] * pl->n[b] * pl->n[b];
        return ca > cb;
    });
    pl->items.resize(pl->batch);
    int64_t off = 0;
    pl->bmax = 1;
    for (int32_t t = 0; t < pl->batch; ++t) {
        const int32_t k = ord[t];
        BatchItem it;
        it.k = k;
        it.B = std::min(pl->class_B[size_class(pl->m[k], pl->n[k])], max_tile(pl->variant));
        if (it.B > pl->bmax) pl->bmax = it.B;
        it.ws = off;
        const int64_t blocks = pl->variant == VAR_HP ? 2 : 1;
        off += blocks * pl->m[k] * pl->n[k];
        off = (off + 63) / 64 * 64;   // keep every instance 256-byte aligned
        pl->items[t] = it;
    }
    pl->ws_bytes = (size_t)off * w;
}

void release_graph(amgs_batch_plan *pl)
{
    // the graph may still be running from the last launch
    if (pl->launched && pl->done) (void)hipEventSynchronize(pl->done);
    if (pl->exec) (void)hipGraphExecDestroy(pl->exec);
    if (pl->graph) (void)hipGraphDestroy(pl->graph);
    pl->exec = nullptr;
    pl->graph = nullptr;
    pl->g_desc = nullptr;
    pl->g_work = nullptr;
    pl->g_info = nullptr;
}

// Synthetic instances with the plan's shapes for timing tile candidates:
// pentadiagonal, strictly diagonally dominant A and pseudo-random Z.
struct TuneSet {
    std::vector<void *> bufs;
    amgs_batch_desc_t *d_desc = nullptr;
    BatchItem *d_items = nullptr;
    int32_t *d_info = nullptr;
    void *d_work = nullptr;
    uint32_t *d_counter = nullptr;
    std::vector<BatchItem> items;
    int32_t count = 0;
    ~TuneSet()
    {
        for (void *p : bufs) (void)hipFree(p);
    }
    template <typename P>
    P *alloc(size_t bytes)
    {
        void *p = nullptr;
        if (hipMalloc(&p, bytes > 0 ? bytes : 1) != hipSuccess) return nullptr;
        bufs.push_back(p);
        return (P *)p;
    }
};

template <typename T>
bool make_tune_set(TuneSet &ts, const std::vector<int32_t> &ks, const amgs_batch_plan *pl)
{
    std::vector<amgs_batch_desc_t> desc(ks.size());
    uint64_t state = 0x9E3779B97F4A7C15ull;
    auto rnd = [&]() {
        state = state * 6364136223846793005ull + 1442695040888963407ull;
        return (double)(state >> 11) * (1.0 / 9007199254740992.0);
    };
    size_t wsz = 0;
    for (size_t t = 0; t < ks.size(); ++t) {
        const int64_t m = pl->m[ks[t]], n = pl->n[ks[t]];
        std::vector<int32_t> rp(m + 1), ci;
        std::vector<T> va;
        rp[0] = 0;
        for (int64_t r = 0; r < m; ++r) {
            for (int64_t c = r - 2; c <= r + 2; ++c) {
                if (c < 0 || c >= m) continue;
                ci.push_back((int32_t)c);
                va.push_back(c == r ? (T)(4.5 + rnd()) : (T)(-rnd()));
            }
            rp[r + 1] = (int32_t)ci.size();
        }
        std::vector<T> z((size_t)m * n);
        for (auto &v : z) v = (T)(rnd() - 0.5);
        int32_t *d_rp = ts.alloc<int32_t>(rp.size() * 4);
        int32_t *d_ci = ts.alloc<int32_t>(ci.size() * 4);
        T *d_va = ts.alloc<T>(va.size() * sizeof(T));
        T *d_z = ts.alloc<T>(z.size() * sizeof(T));
        T *d_q = ts.alloc<T>(z.size() * sizeof(T));
        double *d_r = ts.alloc<double>((size_t)n * n * 8);
        if (!d_rp || !d_ci || !d_va || !d_z || !d_q || !d_r) return false;
        if (hipMemcpy(d_rp, rp.data(), rp.size() * 4, hipMemcpyHostToDevice) != hipSuccess ||
            hipMemcpy(d_ci, ci.data(), ci.size() * 4, hipMemcpyHostToDevice) != hipSuccess ||
            hipMemcpy(d_va, va.data(), va.size() * sizeof(T), hipMemcpyHostToDevice) != hipSuccess ||
            hipMemcpy(d_z, z.data(), z.size() * sizeof(T), hipMemcpyHostToDevice) != hipSuccess)
            return false;
        amgs_batch_desc_t &d = desc[t];
        d.m = m; d.n = n; d.nnz = (int64_t)ci.size();
        d.row_ptr = d_rp; d.col_idx = d_ci; d.vals = d_va;
        d.Z = d_z; d.ldz = m; d.Q = d_q; d.ldq = m; d.R = d_r; d.ldr = n;
        BatchItem it;
        it.k = (int32_t)t;
        it.B = 1;
        it.ws = (int64_t)(wsz / sizeof(T));
        wsz += ((size_t)(pl->variant == VAR_HP ? 2 : 1) * m * n * sizeof(T) + 255) / 256 * 256;
        ts.items.push_back(it);
    }
    ts.count = (int32_t)ks.size();
    ts.d_desc = ts.alloc<amgs_batch_desc_t>(desc.size() * sizeof(amgs_batch_desc_t));
    ts.d_items = ts.alloc<BatchItem>(ts.items.size() * sizeof(BatchItem));
    ts.d_info = ts.alloc<int32_t>(ks.size() * 4);
    ts.d_work = ts.alloc<char>(wsz);
    ts.d_counter = ts.alloc<uint32_t>(4);
    if (!ts.d_desc || !ts.d_items || !ts.d_info || !ts.d_work || !ts.d_counter) return false;
    return hipMemcpy(ts.d_desc, desc.data(), desc.size() * sizeof(amgs_batch_desc_t),
                     hipMemcpyHostToDevice) == hipSuccess;
}

// Time one pass of the persistent kernel over a tune set with the tiles its
// items hold (the widest decides the kernel and its resident grid): the best
// of `reps` launches.
float time_mix(amgs_batch_plan *pl, TuneSet &ts, int reps, hipStream_t s, hipEvent_t e0,
               hipEvent_t e1)
{
    int bmax = 1;
    for (const auto &it : ts.items) bmax = std::max(bmax, it.B);
    if (hipMemcpy(ts.d_items, ts.items.data(), ts.items.size() * sizeof(BatchItem),
                  hipMemcpyHostToDevice) != hipSuccess)
        return -1.f;
    const int grid = std::min(batched_resident_wgs(pl->h->device, pl->precision, pl->variant, bmax),
                              std::max(ts.count, 1));
    float best = -1.f;
    for (int rep = 0; rep < reps; ++rep) {
        (void)hipEventRecord(e0, s);
        launch_batched(pl->precision, pl->variant, bmax, pl->reorth, grid, ts.d_desc, ts.d_items,
                       ts.count, ts.d_work, ts.d_info, ts.d_counter, s);
        (void)hipEventRecord(e1, s);
        if (hipEventSynchronize(e1) != hipSuccess) return -1.f;
        float ms = 0.f;
        (void)hipEventElapsedTime(&ms, e0, e1);
        if (best < 0.f || ms < best) best = ms;
    }
    return best;
}

// Autotuner on the batch's own mix: a stratified sample of the instances
// (every s-th in largest-first order, at most BT_TUNE_MAX, so every size
// class keeps its share of the work) is run as one persistent pass, as the
// real batch is.  Starting from the built-in widths, one width for every
// class is tried first (the widest tile decides the kernel and its resident
// grid for all classes); then each size class in turn (largest total work
// first) tries the other widths {1, 2, 4, 8} (up to the variant's register
// limit) with every other class fixed.  A change is taken only if the whole
// pass gets faster by more than BT_TUNE_GAIN, so that timing noise does not
// flip near-equal choices.  Two sweeps over the classes at most.
template <typename T>
void autotune(amgs_batch_plan *pl)
{
    std::vector<int32_t> order(pl->batch);
    for (int32_t k = 0; k < pl->batch; ++k) order[k] = k;
    auto work = [&](int32_t k) { return (double)pl->m[k] * pl->n[k] * pl->n[k]; };
    std::stable_sort(order.begin(), order.end(),
                     [&](int32_t a, int32_t b) { return work(a) > work(b); });
    const int32_t stride = (pl->batch + BT_TUNE_MAX - 1) / BT_TUNE_MAX;
    std::vector<int32_t> ks;
    for (int32_t t = 0; t < pl->batch; t += stride) ks.push_back(order[t]);
    TuneSet ts;
    if (!make_tune_set<T>(ts, ks, pl)) return;
    std::vector<int> cls_of(ks.size());
    double share[BT_NCLASS] = {0};
    for (size_t t = 0; t < ks.size(); ++t) {
        cls_of[t] = size_class(pl->m[ks[t]], pl->n[ks[t]]);
        share[cls_of[t]] += work(ks[t]);
    }
    std::vector<int> classes;
    for (int c = 0; c < BT_NCLASS; ++c)
        if (share[c] > 0) classes.push_back(c);
    std::stable_sort(classes.begin(), classes.end(),
                     [&](int a, int b) { return share[a] > share[b]; });
    hipStream_t s = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) return;
    (void)hipEventCreate(&e0);
    (void)hipEventCreate(&e1);
    int B[BT_NCLASS];
    for (int c = 0; c < BT_NCLASS; ++c) B[c] = std::min(pl->class_B[c], max_tile(pl->variant));
    auto run = [&]() {
        for (size_t t = 0; t < ts.items.size(); ++t) ts.items[t].B = B[cls_of[t]];
        return time_mix(pl, ts, BT_TUNE_REPS, s, e0, e1);
    };
    // one untimed pass first (code loading, caches)
    (void)run();
    float base = run();
    // the widest tile decides the kernel every class runs in, so start from
    // the best single width for all classes
    for (int cand : {1, 2, 4, 8}) {
        if (cand > max_tile(pl->variant) || base <= 0.f) continue;
        int keep[BT_NCLASS];
        for (int c = 0; c < BT_NCLASS; ++c) {
            keep[c] = B[c];
            B[c] = cand;
        }
        const float t = run();
        if (t > 0.f && t < base * (1.f - BT_TUNE_GAIN)) base = t;
        else
            for (int c = 0; c < BT_NCLASS; ++c) B[c] = keep[c];
    }
    for (int sweep = 0; sweep < 2 && base > 0.f; ++sweep) {
        bool changed = false;
        for (int c : classes) {
            for (int cand : {1, 2, 4, 8}) {
                if (cand > max_tile(pl->variant) || cand == B[c]) continue;
                const int old = B[c];
                B[c] = cand;
                const float t = run();
                if (t > 0.f && t < base * (1.f - BT_TUNE_GAIN)) {
                    base = t;
                    changed = true;
                } else {
                    B[c] = old;
                }
            }
        }
        if (!changed) break;
    }
    for (int c = 0; c < BT_NCLASS; ++c) pl->class_B[c] = B[c];
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    (void)hipStreamDestroy(s);
}

} // namespace

extern "C" {

amgs_status_t amgs_batch_plan_create(amgs_handle_t h, int32_t batch, const int64_t *m_host,
                                     const int64_t *n_host, amgs_variant_t v,
                                     amgs_precision_t p, const amgs_opts_t *o,
                                     int32_t autotune_on, amgs_batch_plan_t *plan)
{
    if (!plan) return AMGS_ERR_ARG;
    *plan = nullptr;
    if (!h || batch < 0 || (batch > 0 && (!m_host || !n_host))) return AMGS_ERR_ARG;
    if (!(v == AMGS_NAIVE || v == AMGS_HA || v == AMGS_HP) || !(p == AMGS_FP64 || p == AMGS_FP32))
        return AMGS_ERR_ARG;
    for (int32_t k = 0; k < batch; ++k)
        if (n_host[k] < 1 || m_host[k] < n_host[k] || m_host[k] > BT_MAX_M || n_host[k] > BT_MAX_N)
            return AMGS_ERR_ARG;
    amgs_batch_plan *pl = new (std::nothrow) amgs_batch_plan();
    if (!pl) return AMGS_ERR_HIP;
    pl->h = h;
    pl->batch = batch;
    pl->variant = (int)v;
    pl->precision = (int)p;
    pl->reorth = o ? (o->reorth != 0) : 0;
    pl->m.assign(m_host, m_host + batch);
    pl->n.assign(n_host, n_host + batch);
    for (int c = 0; c < BT_NCLASS; ++c) pl->class_B[c] = default_B(c, pl->variant);
    pl->d_items = nullptr;
    pl->d_counter = nullptr;
    pl->cap_stream = nullptr;
    pl->done = nullptr;
    pl->launched = 0;
    pl->graph = nullptr;
    pl->exec = nullptr;
    pl->g_desc = nullptr;
    pl->g_work = nullptr;
    pl->g_info = nullptr;
    DevGuard dg(h->device);
    if (autotune_on && batch > 0) {
        if (p == AMGS_FP64) autotune<double>(pl);
        else autotune<float>(pl);
    }
    build_items(pl);
    pl->grid = std::min(batched_resident_wgs(h->device, pl->precision, pl->variant, pl->bmax),
                        std::max(batch, 1));
    if (hipMalloc((void **)&pl->d_items, std::max<size_t>(pl->items.size(), 1) * sizeof(BatchItem)) != hipSuccess ||
        hipMalloc((void **)&pl->d_counter, 4) != hipSuccess ||
        (batch > 0 && hipMemcpy(pl->d_items, pl->items.data(), pl->items.size() * sizeof(BatchItem),
                                hipMemcpyHostToDevice) != hipSuccess) ||
        hipStreamCreateWithFlags(&pl->cap_stream, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&pl->done, hipEventDisableTiming) != hipSuccess) {
        amgs_batch_plan_destroy(pl);
        return AMGS_ERR_HIP;
    }
    *plan = pl;
    return AMGS_OK;
}

amgs_status_t amgs_batch_plan_destroy(amgs_batch_plan_t pl)
{
    if (!pl) return AMGS_ERR_ARG;
    DevGuard dg(pl->h->device);
    release_graph(pl);
    if (pl->d_items) (void)hipFree(pl->d_items);
    if (pl->d_counter) (void)hipFree(pl->d_counter);
    if (pl->cap_stream) (void)hipStreamDestroy(pl->cap_stream);
    if (pl->done) (void)hipEventDestroy(pl->done);
    delete pl;
    return AMGS_OK;
}

size_t amgs_batch_workspace_bytes(amgs_batch_plan_t pl) { return pl ? pl->ws_bytes : 0; }

int32_t amgs_batch_plan_tiles(amgs_batch_plan_t pl, int32_t *out, int32_t cap)
{
    if (!pl) return 0;
    for (int c = 0; c < BT_NCLASS && c < cap; ++c)
        if (out) out[c] = pl->class_B[c];
    return BT_NCLASS;
}

amgs_status_t amgs_qr_batched(amgs_batch_plan_t pl, const amgs_batch_desc_t *desc, void *work,
                              size_t work_bytes, int32_t *info, void *stream)
{
    if (!pl) return AMGS_ERR_ARG;
    if (pl->batch == 0) return AMGS_OK;
    if (!desc || !info) return AMGS_ERR_ARG;
    if (pl->ws_bytes > 0 && (!work || work_bytes < pl->ws_bytes)) return AMGS_ERR_WORKSPACE;
    DevGuard dg(pl->h->device);
    if (!pl->exec || pl->g_desc != desc || pl->g_work != work || pl->g_info != info) {
        release_graph(pl);
        if (hipStreamBeginCapture(pl->cap_stream, hipStreamCaptureModeThreadLocal) != hipSuccess)
            return AMGS_ERR_HIP;
        launch_batched(pl->precision, pl->variant, pl->bmax, pl->reorth, pl->grid, desc,
                       pl->d_items, pl->batch, work, info, pl->d_counter, pl->cap_stream);
        if (hipStreamEndCapture(pl->cap_stream, &pl->graph) != hipSuccess) {
            pl->graph = nullptr;
            return AMGS_ERR_HIP;
        }
        if (hipGraphInstantiate(&pl->exec, pl->graph, nullptr, nullptr, 0) != hipSuccess) {
            release_graph(pl);
            return AMGS_ERR_HIP;
        }
        pl->g_desc = desc;
        pl->g_work = work;
        pl->g_info = info;
    }
    // successive passes of one plan share its work-queue counter: a pass
    // starts only after the previous one (possibly on another stream) ended.
    // Under a caller's stream capture the caller's graph orders the passes.
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing((hipStream_t)stream, &cs) != hipSuccess) return AMGS_ERR_HIP;
    const bool capturing = cs != hipStreamCaptureStatusNone;
    if (!capturing && pl->launched && hipStreamWaitEvent((hipStream_t)stream, pl->done, 0) != hipSuccess)
        return AMGS_ERR_HIP;
    if (hipGraphLaunch(pl->exec, (hipStream_t)stream) != hipSuccess) return AMGS_ERR_HIP;
    if (!capturing) {
        if (hipEventRecord(pl->done, (hipStream_t)stream) != hipSuccess) return AMGS_ERR_HIP;
        pl->launched = 1;
    }
    pl->h->stats = amgs_stats_t{};
    pl->h->stats.kernel_launches = 2;
    return AMGS_OK;
}

} // extern "C"
