// amgs_device.h -- device helpers shared by the library's HIP kernels.
//
// Reductions are deterministic: every sum is taken in a fixed order that does
// not depend on timing, so repeated runs return identical bits and every
// workgroup that re-reduces the same partials obtains the same value.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace amgs {

constexpr int WAVE = 64;

// z - r*q with one rounding (the projection update z_j -= r_ij q_i,
// eq. (9)).  Every kernel applies the update through this function, so a
// value recomputed on the fly equals the stored one bit for bit.
__device__ __forceinline__ double upd(double z, double r, double q) { return __builtin_fma(-r, q, z); }
__device__ __forceinline__ float upd(float z, float r, float q) { return __builtin_fmaf(-r, q, z); }

// Scaling q = z / r_jj (eq. (10)) in binary64, rounded once to storage.
template <typename T>
__device__ __forceinline__ T scale_div(T z, double r) { return (T)((double)z / r); }

// Data-parallel-primitive (DPP) move of a 32-bit lane value; lanes whose
// source is outside the pattern, or whose row is masked off, receive 0.
template <int CTRL, int ROWS>
__device__ __forceinline__ uint32_t dpp32(uint32_t v)
{
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, CTRL, ROWS, 0xf, false);
}
template <int CTRL, int ROWS>
__device__ __forceinline__ float dpp_mov(float v)
{
    return __builtin_bit_cast(float, dpp32<CTRL, ROWS>(__builtin_bit_cast(uint32_t, v)));
}
template <int CTRL, int ROWS>
__device__ __forceinline__ double dpp_mov(double v)
{
    const uint64_t b = __builtin_bit_cast(uint64_t, v);
    const uint64_t lo = dpp32<CTRL, ROWS>((uint32_t)b), hi = dpp32<CTRL, ROWS>((uint32_t)(b >> 32));
    return __builtin_bit_cast(double, (hi << 32) | lo);
}
__device__ __forceinline__ float lane63(float v)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), 63));
}
__device__ __forceinline__ double lane63(double v)
{
    const uint64_t b = __builtin_bit_cast(uint64_t, v);
    const uint64_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)b, 63);
    const uint64_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(b >> 32), 63);
    return __builtin_bit_cast(double, (hi << 32) | lo);
}

// Sum over a wave with DPP moves: pairs and quads (quad_perm), the four
// quads of each 16-lane row (row_ror 4, 8), then rows 0..3 folded into lane
// 63 (row_bcast 15 and 31), whose value is broadcast to every lane.  The
// order is fixed, so the bits are the same on every run and in every wave
// given the same per-lane inputs.
template <typename A>
__device__ __forceinline__ A wave_sum(A v)
{
    v += dpp_mov<0xb1, 0xf>(v);   // quad_perm [1,0,3,2]
    v += dpp_mov<0x4e, 0xf>(v);   // quad_perm [2,3,0,1]
    v += dpp_mov<0x124, 0xf>(v);  // row_ror 4
    v += dpp_mov<0x128, 0xf>(v);  // row_ror 8
    v += dpp_mov<0x142, 0xa>(v);  // row_bcast 15 into rows 1 and 3
    v += dpp_mov<0x143, 0xc>(v);  // row_bcast 31 into rows 2 and 3
    return lane63(v);
}

// Sums of four per-lane values over a whole wave, transposed: on return
// lane l holds the wave's total of value (l & 3).  Half of the values are
// exchanged with lane l^1, then half of the rest with lane l^2 (quad_perm),
// the row is closed with rotations by 4 and 8, and the four rows of the wave
// are added with lane exchanges l^16 and l^32.  Each lane does the work of
// about one reduction instead of four; the order is fixed, so the bits do
// not depend on timing.
template <typename A>
__device__ __forceinline__ A wave_sum4(A v0, A v1, A v2, A v3)
{
    const int lane = threadIdx.x & (WAVE - 1);
    const bool b0 = lane & 1, b1 = lane & 2;
    const A s0 = b0 ? v0 : v1, s1 = b0 ? v2 : v3;
    const A k0 = b0 ? v1 : v0, k1 = b0 ? v3 : v2;
    const A t0 = k0 + dpp_mov<0xb1, 0xf>(s0);   // value b0 of the pair
    const A t1 = k1 + dpp_mov<0xb1, 0xf>(s1);   // value b0 + 2 of the pair
    const A s2 = b1 ? t0 : t1, k2 = b1 ? t1 : t0;
    A r = k2 + dpp_mov<0x4e, 0xf>(s2);          // value (l & 3) of the quad
    r += dpp_mov<0x124, 0xf>(r);                // row_ror 4
    r += dpp_mov<0x128, 0xf>(r);                // row_ror 8
    r += __shfl_xor(r, 16);
    r += __shfl_xor(r, 32);
    return r;
}

// Canonical reduction of v[0..N): lane l adds v[l], v[l+64], v[l+128], ...
// in ascending order into one accumulator, then the butterfly.  The loads
// are issued eight at a time, so N <= 512 costs one memory round trip.  Any
// wave of any workgroup calling it on the same data gets the same bits.
template <typename A>
__device__ __forceinline__ A wave_reduce_seq(const A *__restrict__ v, int64_t N)
{
    const int lane = threadIdx.x & (WAVE - 1);
    A s = 0;
    for (int64_t i = lane; i < N; i += 8 * WAVE) {
        A t[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) t[k] = i + k * WAVE < N ? v[i + k * WAVE] : (A)0;
#pragma unroll
        for (int k = 0; k < 8; ++k) s += t[k];
    }
    return wave_sum(s);
}

// wave_reduce_seq with D loads in flight per lane instead of eight: the same
// additions in the same order (identical bits), in fewer memory round trips,
// for a wave that has the registers to spare.
template <int D, typename A>
__device__ __forceinline__ A wave_reduce_seq_deep(const A *__restrict__ v, int64_t N)
{
    const int lane = threadIdx.x & (WAVE - 1);
    A s = 0;
    for (int64_t i = lane; i < N; i += D * WAVE) {
        A t[D];
#pragma unroll
        for (int k = 0; k < D; ++k) t[k] = i + k * WAVE < N ? v[i + k * WAVE] : (A)0;
#pragma unroll
        for (int k = 0; k < D; ++k) s += t[k];
    }
    return wave_sum(s);
}

// The coefficient a sweep's partials v[0..g) form, in one fixed order that
// one wave and eight waves of a workgroup both reach bit for bit: the
// partials are eight contiguous segments of ceil(g / 8); within a segment
// each lane adds its entries in ascending order and the butterfly adds the
// lanes (wave_reduce_seq); the eight segment sums are added in segment order.
// One wave: the eight segments side by side, one load of each in flight.
template <typename A>
__device__ __forceinline__ A coef_reduce_wave(const A *__restrict__ v, int64_t g)
{
    const int lane = threadIdx.x & (WAVE - 1);
    const int64_t g8 = (g + 7) / 8;
    A acc[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) acc[k] = 0;
    for (int64_t i = lane; i < g8; i += WAVE) {
        A t[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) t[k] = k * g8 + i < g ? v[k * g8 + i] : (A)0;
#pragma unroll
        for (int k = 0; k < 8; ++k) acc[k] += t[k];
    }
    A s = wave_sum(acc[0]);
#pragma unroll
    for (int k = 1; k < 8; ++k) s += wave_sum(acc[k]);
    return s;
}

// Eight waves: wave k < 8 reduces segment k (sixteen loads in flight per
// lane) into seg[k] (LDS); the caller adds seg[0..8) in order after a
// barrier.  Waves from 8 on do nothing.
template <typename A>
__device__ __forceinline__ void coef_reduce_segments(const A *__restrict__ v, int64_t g, A *seg)
{
    const int wave = threadIdx.x / WAVE;
    if (wave < 8) {
        const int64_t g8 = (g + 7) / 8;
        const int64_t rest = g - wave * g8;
        const int64_t len = rest < 0 ? 0 : rest < g8 ? rest : g8;
        const A s = wave_reduce_seq_deep<16>(v + wave * g8, len);
        if ((threadIdx.x & (WAVE - 1)) == 0) seg[wave] = s;
    }
}

// coef_reduce_wave computed once per workgroup (by wave 0) and broadcast
// through one LDS slot; every thread must call it.
template <typename A>
__device__ __forceinline__ A coef_reduce_bcast(const A *__restrict__ v, int64_t g, A *slot)
{
    if (threadIdx.x < WAVE) {
        const A s = coef_reduce_wave(v, g);
        if (threadIdx.x == 0) *slot = s;
    }
    __syncthreads();
    return *slot;
}

// Partials of g workgroups stored in XCD order: workgroups are dispatched
// to the 8 XCDs in turn, so workgroup x is stored at xcd_pos(x) = (x % 8) g8
// + x / 8 (g8 = ceil(g / 8)), and the partials that share a cache line come
// from one XCD's L2 (written there as whole sectors, not as words from
// eight caches).  An array of such partials spans 8 g8 entries.
__host__ __device__ __forceinline__ int64_t xcd_span(int64_t g) { return 8 * ((g + 7) / 8); }
__device__ __forceinline__ int64_t xcd_pos(int64_t x, int64_t g)
{
    return (x & 7) * ((g + 7) / 8) + (x >> 3);
}

// The reduction of g such partials: XCD segment by segment, each as in
// wave_reduce_seq (the unused tail entries of a segment are skipped).
template <typename A>
__device__ __forceinline__ A wave_reduce_xcd(const A *__restrict__ v, int64_t g)
{
    const int lane = threadIdx.x & (WAVE - 1);
    const int64_t g8 = (g + 7) / 8;
    A s = 0;
    for (int x = 0; x < 8; ++x) {
        const A *__restrict__ seg = v + x * g8;
        const int64_t n = (g - x + 7) / 8;   // workgroups x, x + 8, ... below g
        for (int64_t i = lane; i < n; i += 8 * WAVE) {
            A t[8];
#pragma unroll
            for (int k = 0; k < 8; ++k) t[k] = i + k * WAVE < n ? seg[i + k * WAVE] : (A)0;
#pragma unroll
            for (int k = 0; k < 8; ++k) s += t[k];
        }
    }
    return wave_sum(s);
}

// wave_reduce_seq computed once per workgroup (by wave 0) and broadcast
// through one LDS slot; every thread must call it.
template <typename A>
__device__ __forceinline__ A block_reduce_bcast(const A *__restrict__ v, int64_t N, A *slot)
{
    if (threadIdx.x < WAVE) {
        const A s = wave_reduce_seq(v, N);
        if (threadIdx.x == 0) *slot = s;
    }
    __syncthreads();
    return *slot;
}

// Sum over a workgroup of NT threads: wave butterflies, then the NT/64 wave
// results added in wave order by every thread.  `lds` holds NT/64 entries.
template <typename A, int NT>
__device__ __forceinline__ A block_sum(A v, A *lds)
{
    v = wave_sum(v);
    if ((threadIdx.x & (WAVE - 1)) == 0) lds[threadIdx.x / WAVE] = v;
    __syncthreads();
    A t = lds[0];
#pragma unroll
    for (int w = 1; w < NT / WAVE; ++w) t += lds[w];
    __syncthreads();
    return t;
}

// Loads and stores of streamed columns; NT selects the non-temporal
// (streaming) cache policy.
template <bool NT, typename T>
__device__ __forceinline__ T ld_stream(const T *p)
{
    if constexpr (NT) return __builtin_nontemporal_load(p);
    else return *p;
}
// Guarded loads that stay in flight together.  A load under a test that is
// the same in every lane (a column count) is otherwise compiled as a branch
// that waits for the load at its join.  ld_fix issues the load from an
// index that is always valid (f when !ok), pin() keeps the compiler from
// moving the issued loads below it, and pick() then drops the values of the
// failed tests: v = ld_fix(p, i, f, ok); ...; pin(); v = pick(v, ok).
template <bool NT = false, typename T>
__device__ __forceinline__ T ld_fix(const T *__restrict__ p, int64_t i, int64_t f, bool ok)
{
    return ld_stream<NT>(p + (ok ? i : f));
}
__device__ __forceinline__ void pin() { asm volatile("" ::: "memory"); }
template <typename T>
__device__ __forceinline__ T pick(T v, bool ok) { return ok ? v : (T)0; }

template <bool NT, typename T>
__device__ __forceinline__ void st_stream(T *p, T v)
{
    if constexpr (NT) __builtin_nontemporal_store(v, p);
    else *p = v;
}

// Matrix-core 16x16x4 instructions (v_mfma_f64_16x16x4f64 in binary64,
// v_mfma_f32_16x16x4f32 in binary32): D = C + A B with lane l supplying
// A[l%16][l/16] and B[l/16][l%16].  Result rows: register v of lane l holds
// row 4*v + l/16 for the binary64 instruction and row 4*(l/16) + v for the
// binary32 one (column l%16 in both), as measured on gfx950.
typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

template <typename T> struct Mfma;
template <> struct Mfma<double> {
    typedef d4 acc_t;
    static __device__ __forceinline__ acc_t op(double a, double b, acc_t c)
    {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int row(int lane, int v) { return 4 * v + (lane >> 4); }
};
template <> struct Mfma<float> {
    typedef f4 acc_t;
    static __device__ __forceinline__ acc_t op(float a, float b, acc_t c)
    {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int row(int lane, int v) { return 4 * (lane >> 4) + v; }
};

__device__ __forceinline__ bool norm_ok(double rr) { return rr > 0.0 && rr <= 1.7976931348623157e308; }

} // namespace amgs
