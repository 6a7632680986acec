// Internal: MFMA 16x16x4 operand helpers shared by the dense block and SpMM kernels,
// and an LDS-only work-group barrier.
//
// MFMA 16x16x4 layout (gfx950, FP32 and FP64): lane l supplies A[l%16][l/16] and
// B[l/16][l%16]; result register r of lane l holds D[4(l/16)+r][l%16] (FP32) or
// D[(l/16)+4r][l%16] (FP64).
//
// Column runs: a wave that covers NT tiles of 16 columns may give lane column lc of
// tile a any W column, as long as every tile's 16 columns are distinct. Splitting
// the NT tiles into segments of VW tiles (then 2, then 1) and giving lane lc of the
// e-th tile of a segment starting at tile t the column 16 t + q lc + e (q = segment
// width) lets each lane read q adjacent elements with one vector access, aligned to
// q elements.
#pragma once

#include <hip/hip_runtime.h>

#include <type_traits>
#include <utility>

namespace css {

typedef double mf_d4 __attribute__((ext_vector_type(4)));
typedef float mf_f4 __attribute__((ext_vector_type(4)));

template <typename T>
struct Mfma;
template <>
struct Mfma<double> {
    typedef mf_d4 acc;
    static constexpr int VW = 2;      // elements per 16-byte access
    __device__ static acc zero() { return acc{0.0, 0.0, 0.0, 0.0}; }
    __device__ static acc mma(double a, double b, acc c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }
    __device__ static int row(int l, int r) { return (l >> 4) + 4 * r; }
};
template <>
struct Mfma<float> {
    typedef mf_f4 acc;
    static constexpr int VW = 4;
    __device__ static acc zero() { return acc{0.f, 0.f, 0.f, 0.f}; }
    __device__ static acc mma(float a, float b, acc c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
    __device__ static int row(int l, int r) { return 4 * (l >> 4) + r; }
};

// Cross-lane moves for a 16 x 16 FP64 tile held in the D layout (row group g = lanes
// 16g .. 16g+15 holds rows g + 4r, lane 16g + c column c), all on the VALU:
//   lane_read(v, s): v of lane s in every lane (two readlanes; s uniform);
//   col_bcast<K>(v): v of lane K of the lane's own row group (DPP row_newbcast), i.e.
//     the element of column K in each of the lane's rows;
//   grp_bcast<G>(v): v of the lane in row group G with the lane's own column, i.e. a
//     row held by group G sent to every group (permlane32_swap gives groups 0,1,0,1 and
//     2,3,2,3; permlane16_swap of either gives a,a,a,a and b,b,b,b).
__device__ __forceinline__ double lane_read(double v, int src) {
    const long long u = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane(static_cast<int>(u & 0xffffffffLL), src);
    const int hi = __builtin_amdgcn_readlane(static_cast<int>(u >> 32), src);
    return __longlong_as_double((static_cast<long long>(hi) << 32) | static_cast<unsigned int>(lo));
}
template <int K>
__device__ __forceinline__ double col_bcast(double v) {     // one 64-bit DPP move
    static_assert(K >= 0 && K < 16, "lane within a row group");
    return __longlong_as_double(__builtin_amdgcn_mov_dpp(__double_as_longlong(v), 0x150 + K, 0xf, 0xf, true));
}
template <int G>
__device__ __forceinline__ int grp_bcast32(int x) {
    static_assert(G >= 0 && G < 4, "row group");
    const auto h = __builtin_amdgcn_permlane32_swap(x, x, false, false);
    const int y = static_cast<int>(h[G >> 1]);
    const auto q = __builtin_amdgcn_permlane16_swap(y, y, false, false);
    return static_cast<int>(q[G & 1]);
}
template <int G>
__device__ __forceinline__ double grp_bcast(double v) {
    const long long u = __double_as_longlong(v);
    const int lo = grp_bcast32<G>(static_cast<int>(u & 0xffffffffLL));
    const int hi = grp_bcast32<G>(static_cast<int>(u >> 32));
    return __longlong_as_double((static_cast<long long>(hi) << 32) | static_cast<unsigned int>(lo));
}
// f(std::integral_constant<int, K>) for K = 0 .. N-1 in order (compile-time step index)
template <typename F, int... K>
__device__ __forceinline__ void static_steps(F&& f, std::integer_sequence<int, K...>) {
    (f(std::integral_constant<int, K>{}), ...);
}
// 1/x and 1/sqrt(x) for positive normal x: the hardware estimate refined by two Newton
// steps, r <- r + r (1 - x r) and r <- r + (r/2)(1 - x r^2); each step squares the
// relative error, so the result is within a few units in the last place.
__device__ __forceinline__ double recip_newton(double x) {
    double r = __builtin_amdgcn_rcp(x);
    double e = __builtin_fma(-x, r, 1.0);
    r = __builtin_fma(r, e, r);
    e = __builtin_fma(-x, r, 1.0);
    return __builtin_fma(r, e, r);
}
__device__ __forceinline__ double rsqrt_newton(double x) {
    double r = __builtin_amdgcn_rsq(x);
    double e = __builtin_fma(-x * r, r, 1.0);
    r = __builtin_fma(0.5 * r, e, r);
    e = __builtin_fma(-x * r, r, 1.0);
    return __builtin_fma(0.5 * r, e, r);
}

// Work-group barrier that orders LDS accesses only: the LDS writes before it are
// complete (release at work-group scope, LDS only) when the waves meet, and the
// empty asm keeps the compiler from moving memory accesses across it. Global loads
// in flight (the prefetched X chunks) stay in flight.
__device__ __forceinline__ void lds_barrier() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    asm volatile("" ::: "memory");
}

template <typename T, int Q>
__device__ inline void load_q(const T* p, T (&o)[Q]) {
    if constexpr (Q == 1) {
        o[0] = *p;
    } else {
        typedef T vt __attribute__((ext_vector_type(Q)));
        const vt v = *reinterpret_cast<const vt*>(p);
#pragma unroll
        for (int e = 0; e < Q; ++e) o[e] = v[e];
    }
}

template <typename T, int Q>
__device__ inline void store_q(T* p, const T (&o)[Q]) {
    if constexpr (Q == 1) {
        *p = o[0];
    } else {
        typedef T vt __attribute__((ext_vector_type(Q)));
        vt v;
#pragma unroll
        for (int e = 0; e < Q; ++e) v[e] = o[e];
        *reinterpret_cast<vt*>(p) = v;
    }
}

// Segments of a run of NT tiles: `full` tiles in runs of VW, then `two`, then `one`.
template <int NT, int VW>
struct Seg {
    static constexpr int full = NT / VW * VW;
    static constexpr int two = (VW > 2 && NT - full >= 2) ? 2 : 0;
    static constexpr int one = NT - full - two;
};

// Column (within the NT*16 run) that lane column lc of tile a stands for.
template <int NT, int VW>
__device__ constexpr int seg_col(int a, int lc) {
    typedef Seg<NT, VW> S;
    if (a < S::full) return 16 * (a / VW * VW) + VW * lc + a % VW;
    if (a < S::full + S::two) return 16 * S::full + 2 * lc + (a - S::full);
    return 16 * a + lc;
}

// Loads this lane's NT values of a row run starting at p (16 NT elements, aligned to
// VW elements): x[a] = p[seg_col(a, lc)].
template <typename T, int NT>
__device__ inline void load_run(const T* __restrict__ p, int lc, T (&x)[NT]) {
    constexpr int VW = Mfma<T>::VW;
    typedef Seg<NT, VW> S;
#pragma unroll
    for (int t = 0; t < S::full; t += VW) {
        T y[VW];
        load_q<T, VW>(p + 16 * t + VW * lc, y);
#pragma unroll
        for (int e = 0; e < VW; ++e) x[t + e] = y[e];
    }
    if constexpr (S::two) {
        T y[2];
        load_q<T, 2>(p + 16 * S::full + 2 * lc, y);
        x[S::full] = y[0];
        x[S::full + 1] = y[1];
    }
    if constexpr (S::one) x[NT - 1] = p[16 * (NT - 1) + lc];
}

// Stores this lane's NT values of a row run: p[seg_col(a, lc)] = x[a].
template <typename T, int NT>
__device__ inline void store_run(T* __restrict__ p, int lc, const T (&x)[NT]) {
    constexpr int VW = Mfma<T>::VW;
    typedef Seg<NT, VW> S;
#pragma unroll
    for (int t = 0; t < S::full; t += VW) {
        T y[VW];
#pragma unroll
        for (int e = 0; e < VW; ++e) y[e] = x[t + e];
        store_q<T, VW>(p + 16 * t + VW * lc, y);
    }
    if constexpr (S::two) {
        const T y[2] = {x[S::full], x[S::full + 1]};
        store_q<T, 2>(p + 16 * S::full + 2 * lc, y);
    }
    if constexpr (S::one) p[16 * (NT - 1) + lc] = x[NT - 1];
}

}  // namespace css
