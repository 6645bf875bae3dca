// amgs_bsweep.hip -- the block sweep of the two- and three-level panel
// schedules (opts->panel = 8 and 16): after each outer panel of eight (or
// sixteen) columns, one pass over every later column applies the previous
// outer panel as a block and forms the dots with this outer panel's p
// vectors, on the matrix cores.  The three-level schedule also runs it as an
// update-only sweep over a sixteen-panel's own columns and as a dots-only
// sweep after its first eight-panel.  Kept in a file of its own so that its
// measured HBM traffic can be tied to its source.
#include <hip/hip_ext.h>

#include "amgs_device.h"
#include "amgs_internal.h"

namespace amgs {

// ------------------------------------------------ outer block sweep
// After an outer panel I = [d0, d0 + nd) is finished, one pass over every
// later column c (the columns of grid row y) applies the pending outer panel
// I-1 = [k0, k1) as a block, z_c -= Q_{I-1} r_{I-1,c} (coefficients final in
// R), and forms the partials of W_c = P_I^T z_c.  Both are small dense
// contractions and run on the matrix cores, on tiles of 16 rows x 16 later
// columns: the update is D = Z + Q_{I-1} (-R_{I-1,tile}) (BB/4 16x16x4 steps
// over the BB pending columns, Z entering as the accumulator), and the
// dots W += P_I^T D take D's registers directly as the B operand (four
// 16x16x4 steps over the tile's rows; for BB = 8 rows 8..15 of W unused).  For that the
// tile's rows are permuted so that register v of lane l holds matrix row
// 4 (l/16) + v of the tile: tile row i of the update's A operand is matrix
// row bs_act(i).  A wave owns BS_ST consecutive 16-row tiles (64 rows) and
// walks the workgroup's later columns 16 at a time.  Each column of such a
// 64 x 16 block is read and written with whole-wave contiguous accesses and
// moved between that layout and the matrix-core layout through the wave's
// own LDS tile.  Each later column is read and written once per outer
// panel.  The per-wave W tiles are added in wave order through LDS.
template <typename T>
__device__ __forceinline__ int bs_act(int i)
{
    // binary64 results: register v of lane l is tile row 4 v + l/16
    return sizeof(T) == 8 ? 4 * (i & 3) + (i >> 2) : i;
}

// The W partials of one 16-column tile starting at ct (nc columns): the
// waves' entries added in wave order, stored in XCD order (xcd_pos).
template <typename T, int BB>
__device__ __forceinline__ void bs_wpart(const T (*red)[16 * BB], int64_t ct, int nc,
                                         int nd, const BSweepArgs &a)
{
    const int tid = threadIdx.x;
    if (tid < nc * BB) {
        const int cl = tid / BB, d = tid - cl * BB;
        if (d < nd) {
            T s = red[0][tid];
#pragma unroll
            for (int w = 1; w < 256 / WAVE; ++w) s += red[w][tid];
            ((T *)a.part)[((ct + cl) * BB + d) * xcd_span(a.g) + xcd_pos(blockIdx.x, a.g)] = s;
        }
    }
}

// BB: the block width, 8 (two-level schedule) or 16 (three levels: all 16
// rows of W in use, the update four 16x16x4 steps).  DOTS = false: the
// update alone (no dot columns), without the P_I operand and the W work.
// ONE: every workgroup has a single 16-column tile, whose loads are issued
// together with those of the operands (one memory round trip, not two).
template <typename T, bool NTS, int BB, bool DOTS, bool ONE>
__global__ __launch_bounds__(256, 4) void k_bsweep(BSweepArgs a)
{
    typedef typename Mfma<T>::acc_t acc_t;
    constexpr int ST = BS_ST;
    constexpr int WR = ST * 16;         // rows per wave
    constexpr int LD = WR + 4;          // padded LDS column (16-byte aligned)
    constexpr int KS = BB / 4;          // 16x16x4 steps of the update
    static_assert(BB == 8 || BB == 16, "block widths of the panel schedules");
    static_assert(WR == WAVE, "one row per lane in the contiguous accesses");
    __shared__ T red[256 / WAVE][16 * BB];   // the waves' W of one 16-column tile
    __shared__ __attribute__((aligned(16))) T tile[256 / WAVE][16][LD];
    if (*a.info) return;
    const int tid = threadIdx.x, wave = tid / WAVE, lane = tid & (WAVE - 1);
    const int g4 = lane >> 4, jl = lane & 15;
    T *__restrict__ Q = (T *)a.Q;
    const T *__restrict__ Zs = (const T *)a.Zs;   // the later columns' current values
    const T *__restrict__ P = (const T *)a.P;
    const int64_t m = a.m, ldq = a.ldq;
    const int64_t wrow0 = ((int64_t)blockIdx.x * (256 / WAVE) + wave) * WR;
    const int64_t myrow = wrow0 + lane;
    const bool rin = myrow < m;
    const int kw = (int)(a.k1 - a.k0), nd = (int)a.nd;
    T(*tl)[LD] = tile[wave];
    // Operands that stay for every column: p_{d0+l%16} at matrix row
    // 4 (l/16) + v (A of the dots, step v) and q_{k0+4s+l/16} at tile row
    // l%16 (A of the update), both brought in with contiguous column reads
    // through the LDS tile.  Grid row 0 also forms P_I^T Q_I over the wave's
    // rows (entry [i, k] = p_{d0+i}^T q_{d0+k}, B operand q_{d0+l%16} at
    // matrix row 4 (l/16) + v), added over the waves after the columns; its
    // strictly lower part is the L of the block solve.
    const bool own_l = DOTS && blockIdx.y == 0 && nd > 1;
    T qa[ST][KS], pa[ST][4];
    acc_t lw = {0, 0, 0, 0};
    // P_I first, then (grid row 0) Q_I for L, then the pending Q_{I-1},
    // each through the wave's 16-column tile.  All three are loaded at once,
    // from clamped addresses and zeroed after the loads, so that no load
    // waits for the one before it.
    T vp[BB], vq[BB], vk[BB];
#pragma unroll
    for (int c = 0; c < BB; ++c) {
        if constexpr (DOTS) {
            vp[c] = ld_fix(P, myrow + (a.d0 + c) * a.ldp, 0, rin && c < nd);
            vq[c] = ld_fix((const T *)Q, myrow + (a.d0 + c) * ldq, 0, own_l && rin && c < nd);
        }
        vk[c] = ld_fix((const T *)Q, myrow + (a.k0 + c) * ldq, 0, rin && c < kw);
    }
    const int64_t cA = a.c0 + (int64_t)blockIdx.y * a.cpw;
    const int64_t cB = (cA + a.cpw < a.c1) ? cA + a.cpw : a.c1;
    // the wave's 64 x 16 block of the tile at ct, one contiguous column
    // access per column, and the B operand of the update,
    // -r_{k0+4s+l/16, col}, loaded beside it (clamped addresses: no load
    // waits for the one before it)
    T zl[16];
    double rd[KS];
    auto load_tile = [&](int64_t ct) {
        const int nc = (int)(cB - ct < 16 ? cB - ct : 16);
#pragma unroll
        for (int c = 0; c < 16; ++c)
            zl[c] = (c < nc && rin) ? ld_stream<NTS>(Zs + (ct + c) * a.ldzs + myrow) : (T)0;
#pragma unroll
        for (int s = 0; s < KS; ++s) {
            const int kk = 4 * s + g4;
            rd[s] = ld_fix(a.R, (a.k0 + kk) + (ct + jl) * a.ldr, 0, jl < nc && kk < kw);
        }
    };
    if (ONE && cA < cB) load_tile(cA);
    pin();
    if constexpr (DOTS) {
#pragma unroll
        for (int c = 0; c < BB; ++c) tl[c][lane] = pick(vp[c], rin && c < nd);
        __syncthreads();
#pragma unroll
        for (int st = 0; st < ST; ++st)
#pragma unroll
            for (int v = 0; v < 4; ++v) pa[st][v] = jl < BB ? tl[jl][st * 16 + 4 * g4 + v] : (T)0;
    }
    if (own_l) {
        __syncthreads();
#pragma unroll
        for (int c = 0; c < BB; ++c) tl[c][lane] = pick(vq[c], rin && c < nd);
        __syncthreads();
#pragma unroll
        for (int st = 0; st < ST; ++st)
#pragma unroll
            for (int v = 0; v < 4; ++v)
                lw = Mfma<T>::op(pa[st][v], jl < BB ? tl[jl][st * 16 + 4 * g4 + v] : (T)0, lw);
    }
    if constexpr (DOTS) __syncthreads();
#pragma unroll
    for (int c = 0; c < BB; ++c) tl[c][lane] = pick(vk[c], rin && c < kw);
    __syncthreads();
#pragma unroll
    for (int st = 0; st < ST; ++st)
#pragma unroll
        for (int s2 = 0; s2 < KS; ++s2) qa[st][s2] = tl[4 * s2 + g4][st * 16 + bs_act<T>(jl)];
    for (int64_t ct = cA; ct < cB; ct += 16) {
        const int nc = (int)(cB - ct < 16 ? cB - ct : 16);
        const bool cin = jl < nc;
        if constexpr (!ONE) {
            load_tile(ct);
            pin();
        }
        __syncthreads();   // the previous block's LDS reads and W entries are done
        if (DOTS && ct > cA) bs_wpart<T, BB>(red, ct - 16, 16, nd, a);
#pragma unroll
        for (int c = 0; c < 16; ++c) tl[c][lane] = zl[c];
        __syncthreads();
        T rb[KS];
#pragma unroll
        for (int s = 0; s < KS; ++s) rb[s] = -(T)pick(rd[s], cin && 4 * s + g4 < kw);
        acc_t w = {0, 0, 0, 0};
#pragma unroll
        for (int st = 0; st < ST; ++st) {
            acc_t z;
#pragma unroll
            for (int v = 0; v < 4; ++v) z[v] = tl[jl][st * 16 + 4 * g4 + v];
            if (kw > 0) {
#pragma unroll
                for (int s2 = 0; s2 < KS; ++s2)
                    if (kw > 4 * s2) z = Mfma<T>::op(qa[st][s2], rb[s2], z);
#pragma unroll
                for (int v = 0; v < 4; ++v) tl[jl][st * 16 + 4 * g4 + v] = (T)z[v];
            }
            if constexpr (DOTS) {
#pragma unroll
                for (int v = 0; v < 4; ++v) w = Mfma<T>::op(pa[st][v], (T)z[v], w);
            }
        }
        if (kw > 0) {
            __syncthreads();
#pragma unroll
            for (int c = 0; c < 16; ++c)
                if (c < nc && rin) st_stream<NTS>(Q + (ct + c) * ldq + myrow, tl[c][lane]);
        }
        // W[i, col] for i = Mfma<T>::row(lane, v) < BB, added over the
        // waves at the next tile (or below)
        if constexpr (DOTS) {
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int i = Mfma<T>::row(lane, v);
                if (i < BB) red[wave][jl * BB + i] = (T)w[v];
            }
        }
    }
    if (!DOTS) return;
    __syncthreads();
    if (cA < cB) {
        const int64_t last = cA + (cB - 1 - cA) / 16 * 16;
        bs_wpart<T, BB>(red, last, (int)(cB - last), nd, a);
    }
    if (own_l) {
        __syncthreads();   // the W entries have been read
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int i = Mfma<T>::row(lane, v);
            if (i < BB && jl < BB) red[wave][i * BB + jl] = (T)lw[v];
        }
        __syncthreads();
        for (int idx = tid; idx < BB * BB; idx += 256) {
            const int i = idx / BB, k = idx - i * BB;
            if (!(k < i && i < nd)) continue;
            T s = red[0][idx];
#pragma unroll
            for (int w = 1; w < 256 / WAVE; ++w) s += red[w][idx];
            ((T *)a.lpart)[(int64_t)idx * xcd_span(a.g) + xcd_pos(blockIdx.x, a.g)] = s;
        }
    }
}

// ------------------------------------------------------------- launcher
int64_t bsweep_chunks(int64_t m, size_t w)
{
    (void)w;
    const int64_t rows = (int64_t)(256 / WAVE) * BS_ST * 16;
    const int64_t g = (m + rows - 1) / rows;
    return g < 1 ? 1 : g;
}

template <typename T>
void launch_bsweep(const Ctx &c, int64_t k0, int64_t k1, int64_t d0, int64_t d1, int64_t c0,
                   int64_t c1, bool from_z, int bb)
{
    BSweepArgs a{};
    a.m = c.m; a.Q = c.Q; a.ldq = c.ldq; a.P = c.P; a.ldp = c.ldp; a.R = c.R; a.ldr = c.ldr;
    a.Zs = from_z ? c.Z : c.Q;
    a.ldzs = from_z ? c.ldz : c.ldq;
    a.info = c.info; a.k0 = k0; a.k1 = k1; a.d0 = d0; a.nd = d1 - d0;
    a.c0 = c0; a.c1 = c1 > c0 ? c1 : c0; a.part = c.wpart; a.lpart = c.lpart8; a.g = c.g_b;
    const int64_t ncols = a.c1 - a.c0;
    // column groups: multiples of 16, at most BS_MAXC, enough workgroups
    int64_t gy = 1, cpw = 16;
    if (ncols > 0) {
        gy = (SWEEP_TARGET_WG + c.g_b - 1) / c.g_b;
        const int64_t max_gy = (ncols + 15) / 16;
        if (gy > max_gy) gy = max_gy;
        if (gy < 1) gy = 1;
        cpw = (ncols + gy - 1) / gy;
        cpw = (cpw + 15) / 16 * 16;
        if (cpw > BS_MAXC) cpw = BS_MAXC;
        gy = (ncols + cpw - 1) / cpw;
    }
    a.cpw = cpw;
    const dim3 grid((unsigned)c.g_b, (unsigned)gy), block(256);
    const bool one = ncols > 0 && cpw == 16;
    const bool nts = (double)ncols * (double)c.m * sizeof(T) > SWEEP_NT_BYTES;
#define AMGS_BS1(NT_, BB_, D_, O_)                                                                \
    do {                                                                                          \
        if (c.ev_start)                                                                           \
            hipExtLaunchKernelGGL((k_bsweep<T, NT_, BB_, D_, O_>), grid, block, 0, c.stream,      \
                                  c.ev_start, c.ev_stop, 0, a);                                   \
        else                                                                                      \
            hipLaunchKernelGGL((k_bsweep<T, NT_, BB_, D_, O_>), grid, block, 0, c.stream, a);     \
    } while (0)
    // the one-tile instances serve the three-level schedule's short sweeps:
    // the update-only one (width 16) and the dots-only one (width 8)
#define AMGS_BS(NT_, BB_)                                                                         \
    do {                                                                                          \
        if (a.nd > 0) {                                                                           \
            if (BB_ == PANEL_B1 && one) AMGS_BS1(NT_, BB_, true, true);                           \
            else AMGS_BS1(NT_, BB_, true, false);                                                 \
        } else {                                                                                  \
            if (BB_ == PANEL_B2 && one) AMGS_BS1(NT_, BB_, false, true);                          \
            else AMGS_BS1(NT_, BB_, false, false);                                                \
        }                                                                                         \
    } while (0)
    if (bb == PANEL_B2) {
        if (nts) AMGS_BS(true, PANEL_B2);
        else AMGS_BS(false, PANEL_B2);
    } else {
        if (nts) AMGS_BS(true, PANEL_B1);
        else AMGS_BS(false, PANEL_B1);
    }
#undef AMGS_BS
#undef AMGS_BS1
}


template void launch_bsweep<double>(const Ctx &, int64_t, int64_t, int64_t, int64_t, int64_t, int64_t,
                                    bool, int);
template void launch_bsweep<float>(const Ctx &, int64_t, int64_t, int64_t, int64_t, int64_t, int64_t,
                                   bool, int);

} // namespace amgs
