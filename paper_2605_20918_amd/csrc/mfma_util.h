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
