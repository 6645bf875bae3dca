// amgs_gemm.hip -- the HP block product X = A Z for dense A on the matrix
// cores (Alg. 6: the n MV of the method issued as one
// matrix-matrix product, which Section 2.3 expects to run much faster than
// n sequential MV).
//
// A is symmetric and column-major, so X[k, c] = sum_l A[l, k] Z[l, c]: both
// operands are contiguous along the contraction index l.  MFMA 16x16 tiles
// (v_mfma_f64_16x16x4f64 in binary64, v_mfma_f32_16x16x4f32 in binary32);
// K is consumed in slabs of 16 staged through LDS (double-buffered), each
// thread loading a run of consecutive k values of one column.
#include <type_traits>

#include "amgs_device.h"
#include "amgs_internal.h"

namespace amgs {

constexpr int GB_K = 16;

// Operand layout of the 16x16x4 instructions: lane l supplies A[l%16][l/16]
// and B[l/16][l%16]; result rows follow Mfma<T>::row.  A workgroup of four
// waves (2 x 2) computes a TM x TN tile of X; each wave owns a
// (TM/2) x (TN/2) block of (TM/32) x (TN/32) MFMA tiles.  Larger tiles read
// A fewer times (once per TN columns of X) and feed more MFMAs per LDS read.
template <typename T, int TM, int TN>
__global__ __launch_bounds__(256, 2) void k_gemm_atb(int64_t m, int64_t n, const T *__restrict__ A,
                                                  int64_t lda, const T *__restrict__ Z,
                                                  int64_t ldz, T *__restrict__ X, int64_t ldx)
{
    typedef typename Mfma<T>::acc_t acc_t;
    constexpr int FM = TM / 32, FN = TN / 32;
    // staging: each thread loads a run of consecutive k values of one column
    constexpr int A_PER = TM * GB_K / 256, B_PER = TN * GB_K / 256;
    constexpr int A_TPC = GB_K / A_PER, B_TPC = GB_K / B_PER;
    static_assert(A_PER >= 1 && B_PER >= 1 && GB_K % A_PER == 0 && GB_K % B_PER == 0, "tile");
    // LDS: [buffer][k][col], padded by one element per row against bank
    // conflicts between the four k rows read by one instruction.
    __shared__ T As[2][GB_K][TM + 1];
    __shared__ T Bs[2][GB_K][TN + 1];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int64_t m0 = (int64_t)blockIdx.x * TM;   // rows of X (= columns of A)
    const int64_t n0 = (int64_t)blockIdx.y * TN;   // columns of X (= columns of Z)
    const int wm = (wave & 1) * (TM / 2), wn = (wave >> 1) * (TN / 2);

    const int ac = tid / A_TPC, ak = (tid % A_TPC) * A_PER;
    const int bc = tid / B_TPC, bk = (tid % B_TPC) * B_PER;
    const bool a_ok = m0 + ac < m, b_ok = n0 + bc < n;
    const T *__restrict__ Acol = A + (a_ok ? (m0 + ac) : 0) * lda;
    const T *__restrict__ Zcol = Z + (b_ok ? (n0 + bc) : 0) * ldz;

    acc_t acc[FM][FN];
#pragma unroll
    for (int a = 0; a < FM; ++a)
#pragma unroll
        for (int b = 0; b < FN; ++b)
#pragma unroll
            for (int v = 0; v < 4; ++v) acc[a][b][v] = 0;

    // Two register sets of staged loads: slab kt+2 is requested while slab
    // kt is multiplied and slab kt+1 waits in registers, so the loads have
    // two slabs of MFMA work to arrive.  Every load is issued on every path
    // (a slab past the end re-reads the last one, whose values are never
    // used), so the wait before each LDS store covers only the older set.
    // Interior tiles (every row, column and slab inside the matrix) load
    // without any test; edge tiles clamp the index to a valid element and
    // zero the value.
    const int64_t nk = (m + GB_K - 1) / GB_K;
    const int64_t klast = (nk - 1) * GB_K;
    auto run = [&](auto edge_tag) {
        constexpr bool EDGE = decltype(edge_tag)::value;
        T ra[2][A_PER], rb[2][B_PER];
        auto gload = [&](int set, int64_t k0) {
            k0 = k0 < klast ? k0 : klast;
#pragma unroll
            for (int t = 0; t < A_PER; ++t) {
                const int64_t k = k0 + ak + t;
                if (EDGE) {
                    const bool ok = a_ok && k < m;
                    const T v = Acol[ok ? k : 0];
                    ra[set][t] = ok ? v : (T)0;
                } else {
                    ra[set][t] = Acol[k];
                }
            }
#pragma unroll
            for (int t = 0; t < B_PER; ++t) {
                const int64_t k = k0 + bk + t;
                if (EDGE) {
                    const bool ok = b_ok && k < m;
                    const T v = Zcol[ok ? k : 0];
                    rb[set][t] = ok ? v : (T)0;
                } else {
                    rb[set][t] = Zcol[k];
                }
            }
        };
        auto lstore = [&](int set, int buf) {
#pragma unroll
            for (int t = 0; t < A_PER; ++t) As[buf][ak + t][ac] = ra[set][t];
#pragma unroll
            for (int t = 0; t < B_PER; ++t) Bs[buf][bk + t][bc] = rb[set][t];
        };
        auto compute = [&](int buf) {
#pragma unroll
            for (int ks = 0; ks < GB_K; ks += 4) {
                const int kk = ks + (lane >> 4);
                T av[FM], bv[FN];
#pragma unroll
                for (int a = 0; a < FM; ++a) av[a] = As[buf][kk][wm + a * 16 + (lane & 15)];
#pragma unroll
                for (int b = 0; b < FN; ++b) bv[b] = Bs[buf][kk][wn + b * 16 + (lane & 15)];
#pragma unroll
                for (int a = 0; a < FM; ++a)
#pragma unroll
                    for (int b = 0; b < FN; ++b) acc[a][b] = Mfma<T>::op(av[a], bv[b], acc[a][b]);
            }
        };
        gload(0, 0);
        lstore(0, 0);
        gload(1, GB_K);
        __syncthreads();
        // LDS buffer 0 holds even slabs, buffer 1 odd ones; register set 0
        // stages even slabs, set 1 odd ones
        for (int64_t kt = 0; kt < nk; kt += 2) {
            gload(0, (kt + 2) * GB_K);
            compute(0);
            if (kt + 1 >= nk) break;
            lstore(1, 1);
            __syncthreads();
            gload(1, (kt + 3) * GB_K);
            compute(1);
            lstore(0, 0);
            __syncthreads();
        }
    };
    const bool interior = m % GB_K == 0 && m0 + TM <= m && n0 + TN <= n;
    if (interior) run(std::integral_constant<bool, false>{});
    else run(std::integral_constant<bool, true>{});
    // store each 16x16 tile
#pragma unroll
    for (int a = 0; a < FM; ++a)
#pragma unroll
        for (int b = 0; b < FN; ++b)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int64_t row = m0 + wm + a * 16 + Mfma<T>::row(lane, v);
                const int64_t col = n0 + wn + b * 16 + (lane & 15);
                if (row < m && col < n) X[row + col * ldx] = acc[a][b][v];
            }
}

// Large products: 128 x 64 tiles in binary64 and 128 x 128 in binary32 (the
// faster of the two on MI355X for the 16384 x 16384 x 256 product), when the
// grid still has a workgroup per compute unit; otherwise 64 x 64.
template <typename T>
void launch_dense_gemm(const Ctx &c)
{
    // the new columns [first, n) only
    constexpr int TN = sizeof(T) == 8 ? 64 : 128;
    const int64_t nn = c.n - c.first;
    const T *Zn = (const T *)c.Z + c.first * c.ldz;   // read from Z (see launch_csr_spmm)
    T *Xn = (T *)c.X + c.first * c.m;
    const int64_t big = ((c.m + 127) / 128) * ((nn + TN - 1) / TN);
    if (big >= 256) {
        const dim3 grid((unsigned)((c.m + 127) / 128), (unsigned)((nn + TN - 1) / TN));
        hipLaunchKernelGGL((k_gemm_atb<T, 128, TN>), grid, dim3(256), 0, c.stream, c.m, nn,
                           (const T *)c.A, c.lda, Zn, c.ldz, Xn, c.m);
    } else {
        const dim3 grid((unsigned)((c.m + 63) / 64), (unsigned)((nn + 63) / 64));
        hipLaunchKernelGGL((k_gemm_atb<T, 64, 64>), grid, dim3(256), 0, c.stream, c.m, nn,
                           (const T *)c.A, c.lda, Zn, c.ldz, Xn, c.m);
    }
}

template void launch_dense_gemm<double>(const Ctx &);
template void launch_dense_gemm<float>(const Ctx &);

} // namespace amgs
