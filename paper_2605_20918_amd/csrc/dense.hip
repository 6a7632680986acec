// Dense block kernels of the block Lanczos process (text after Eq.(4)).
//
// * Gram products X^T Y of tall n x b blocks on MFMA (16x16x4, FP64 or FP32
//   inputs), split over row chunks; the chunk partials are summed by a second
//   kernel in a fixed order, so results are deterministic.
// * Block updates OUT = alpha IN + sum_p X_p op(S_p) with small FP64 b x b S_p,
//   on MFMA; operands are read straight from global memory (the small matrix
//   stays in L1/L2 and the MFMA time dominates).
// * b x b FP64 Cholesky and triangular inverse in one workgroup.
//
// MFMA 16x16x4 operand layout (gfx950): lane l supplies A[l%16][l/16] and
// B[l/16][l%16]. Result register r of lane l holds D[(l/16) + 4r][l%16] for
// the FP64 instruction and D[4(l/16) + r][l%16] for the FP32 one.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <type_traits>
#include <atomic>
#include <cmath>

#include "css_common.h"
#include "dense.h"
#include "mfma_util.h"

namespace css {
namespace {

template <typename T>
using MF = Mfma<T>;

// ------------------------------------------------------------------ Gram

// One workgroup computes a TILE x TILE tile of X_p^T Y over a chunk of rows for
// product p = blockIdx.z, writing one partial per (p, chunk). The workgroup has
// KS groups of WPG waves; group g takes the 4-row steps g, g+KS, ... of the chunk,
// and the group tiles are added into one LDS tile in group order. WPG = 1: one
// wave owns the whole (16 TW)^2 tile; WPG = 4: 2 x 2 waves of (16 TW)^2 each.
// With sym, wave tiles strictly below the diagonal are skipped (the reduction
// mirrors them). The operands of each step are fetched gram_depth() steps ahead of
// their use. RUN: every wave tile lies inside ld, and each lane reads runs of
// adjacent columns (seg_col order); otherwise one column per lane and tile,
// masked beyond ld.
// operand steps in flight: 8 for the single-wave FP32 tiles (one wave per SIMD),
// 4 for the 2 x 2-wave tiles
template <typename T, int WPG>
constexpr int gram_depth() { return (WPG == 1 && sizeof(T) == 4) ? 8 : 4; }

template <typename T, int TW, bool RUN>
__device__ inline void gram_load(const T* __restrict__ p, int lc, const bool (&valid)[TW], T (&x)[TW]) {
    if constexpr (RUN) {
        load_run<T, TW>(p, lc, x);
    } else {
#pragma unroll
        for (int a = 0; a < TW; ++a) x[a] = valid[a] ? p[16 * a + lc] : T(0);
    }
}

template <typename T, int TW, bool RUN>
__device__ constexpr int gram_col(int a, int x) {
    if constexpr (RUN) return seg_col<TW, MF<T>::VW>(a, x);
    return 16 * a + x;
}

template <typename T, typename PT, int TW, int KS, int WPG, bool RUN>
__global__ __launch_bounds__(64 * WPG * KS) void k_gram(const T* __restrict__ X, int64_t xstride,
                                                        const T* __restrict__ Y, int64_t Np, int64_t rpc, int ld,
                                                        int ntw, int sym, PT* __restrict__ partial, int nchunk,
                                                        const int* __restrict__ state) {
    if (state && state[0]) return;
    typedef MF<T> M;
    constexpr int D = gram_depth<T, WPG>();
    extern __shared__ char gram_lds[];
    PT* buf = reinterpret_cast<PT*>(gram_lds);            // one TILE^2 tile
    constexpr int TILE = (WPG == 1 ? 16 : 32) * TW;
    const int l = threadIdx.x & 63, w = threadIdx.x >> 6, lr = l >> 4, lc = l & 15;
    const int grp = w / WPG, wl = w % WPG;
    const int wi = (WPG == 1) ? 0 : (wl & 1), wj = (WPG == 1) ? 0 : (wl >> 1);
    const int I0 = (blockIdx.y / ntw) * TILE, J0 = (blockIdx.y % ntw) * TILE;
    const int i0 = I0 + wi * 16 * TW, j0 = J0 + wj * 16 * TW;
    const bool skip = (i0 >= ld || j0 >= ld) || (sym && i0 > j0 + 16 * TW - 16);
    const int chunk = blockIdx.x, p = blockIdx.z;
    const int64_t r0 = (int64_t)chunk * rpc;
    const int64_t r1 = r0 + rpc < Np ? r0 + rpc : Np;
    // r1 - r0 is a multiple of 128, so nst is a multiple of D (4 KS D divides 128)
    static_assert((128 % (4 * KS * D)) == 0, "chunks must hold whole rounds of D steps");
    const int nst = (int)((r1 - r0) / (4 * KS));
    bool vi[TW], vj[TW];
#pragma unroll
    for (int a = 0; a < TW; ++a) { vi[a] = i0 + 16 * a < ld; vj[a] = j0 + 16 * a < ld; }
    typename M::acc c[TW][TW];
#pragma unroll
    for (int a = 0; a < TW; ++a)
#pragma unroll
        for (int b = 0; b < TW; ++b) c[a][b] = M::zero();
    // WPG = 1: the single wave tile always lies inside ld and chunks hold rows, so
    // there is no branch (keeps the accumulators in one register class)
    if (WPG == 1 || (!skip && nst > 0)) {
        const int64_t step = 4 * (int64_t)KS * ld;
        const T* xa = X + (int64_t)p * xstride + (r0 + 4 * grp + lr) * ld + i0;
        const T* ya = Y + (r0 + 4 * grp + lr) * ld + j0;
        T xr[D][TW], yr[D][TW];
#pragma unroll
        for (int d = 0; d < D; ++d) {
            const int64_t o = (int64_t)min(d, nst - 1) * step;
            gram_load<T, TW, RUN>(xa + o, lc, vi, xr[d]);
            gram_load<T, TW, RUN>(ya + o, lc, vj, yr[d]);
        }
        for (int s0 = 0; s0 < nst; s0 += D) {
#pragma unroll
            for (int d = 0; d < D; ++d) {
#pragma unroll
                for (int a = 0; a < TW; ++a)
#pragma unroll
                    for (int b = 0; b < TW; ++b) c[a][b] = M::mma(xr[d][a], yr[d][b], c[a][b]);
                const int64_t o = (int64_t)min(s0 + d + D, nst - 1) * step;
                gram_load<T, TW, RUN>(xa + o, lc, vi, xr[d]);
                gram_load<T, TW, RUN>(ya + o, lc, vj, yr[d]);
                __builtin_amdgcn_sched_barrier(0);       // keep each step's loads D steps ahead of their use
            }
        }
    }
    // group tiles added into LDS in group order (tile-local coordinates)
#pragma unroll
    for (int g = 0; g < KS; ++g) {
        if (grp == g) {
#pragma unroll
            for (int a = 0; a < TW; ++a)
#pragma unroll
                for (int b = 0; b < TW; ++b)
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const int row = wi * 16 * TW + gram_col<T, TW, RUN>(a, M::row(l, r));
                        const int col = wj * 16 * TW + gram_col<T, TW, RUN>(b, lc);
                        const PT v = PT(c[a][b][r]);
                        PT& e = buf[row * TILE + col];
                        e = (g == 0) ? v : e + v;
                        if (r == 3) __builtin_amdgcn_sched_barrier(0);   // one tile's values live at a time
                    }
        }
        __syncthreads();
    }
    PT* out = partial + ((int64_t)p * nchunk + chunk) * ld * ld;
    for (int e = threadIdx.x; e < TILE * TILE; e += 64 * WPG * KS) {
        const int row = e / TILE, col = e % TILE;
        const int gi = I0 + row, gj = J0 + col;
        if (gi < ld && gj < ld) out[(int64_t)gi * ld + gj] = buf[e];
    }
}

// Sum of the chunk partials in a fixed order: thread group g (of 16) adds chunks
// g, g+16, ... for 64 entries, then the group sums are added in order. mode 0: plain,
// 64 consecutive entries per work-group; 1: (S + S^T)/2; 2: out += (S + S^T)/2. The
// symmetrised outputs take an 8 x 8 tile (bi, bj) per work-group: lane e = 8r + c adds
// entry (r, c) of tile (bi, bj) and entry (r, c) of tile (bj, bi), both read as rows
// of 8, and S^T's entry comes from the lane 8c + r through LDS. copy: mode 1's result
// also written there; product sym_p (tiled in any mode): sym_to += (S + S^T)/2.
constexpr int kRedGroups = 16;
static unsigned reduce_blocks(int ld, bool tiled) {
    const int64_t lin = grid_for((int64_t)ld * ld, 64), til = (int64_t)((ld + 7) / 8) * ((ld + 7) / 8);
    return static_cast<unsigned>(tiled ? std::max(lin, til) : lin);
}

template <typename PT>
__global__ __launch_bounds__(64 * kRedGroups) void k_gram_reduce(const PT* __restrict__ partial, int nchunk, int ld,
                                                                int sym, int mode, double* __restrict__ out,
                                                                int64_t out_stride, const int* __restrict__ state,
                                                                double* __restrict__ copy, double* __restrict__ sym_to,
                                                                int sym_p) {
    if (state && state[0]) return;
    __shared__ double s1s[kRedGroups][64], s2s[kRedGroups][64];
    const int p = blockIdx.y;
    const int g = threadIdx.x >> 6, e = threadIdx.x & 63;
    const int64_t mat = (int64_t)ld * ld;
    const bool tiled = mode != 0 || p == sym_p;           // uniform in the work-group
    int i, j, i2 = 0, j2 = 0;
    bool valid, valid2 = false;
    if (!tiled) {
        const int idx = blockIdx.x * 64 + e;
        valid = idx < ld * ld;
        i = valid ? idx / ld : 0;
        j = valid ? idx % ld : 0;
    } else {
        const int nt = (ld + 7) / 8;
        const int bi = (int)blockIdx.x / nt, bj = (int)blockIdx.x % nt, r = e >> 3, c = e & 7;
        i = 8 * bi + r;
        j = 8 * bj + c;
        i2 = 8 * bj + r;                                       // entry (r, c) of tile (bj, bi)
        j2 = 8 * bi + c;
        valid = i < ld && j < ld;
        valid2 = i2 < ld && j2 < ld;
    }
    const int64_t sij = (sym && i > j) ? (int64_t)j * ld + i : (int64_t)i * ld + j;
    const int64_t s2ij = (sym && i2 > j2) ? (int64_t)j2 * ld + i2 : (int64_t)i2 * ld + j2;
    const PT* base = partial + (int64_t)p * nchunk * mat;
    double s1 = 0.0, s2 = 0.0;
    // chunks g, g+16, ... added in that order; unrolled so the loads are issued together
    if (tiled) {
#pragma unroll 8
        for (int c = g; c < nchunk; c += kRedGroups) {
            if (valid) s1 += (double)base[c * mat + sij];
            if (valid2) s2 += (double)base[c * mat + s2ij];
        }
    } else if (valid) {
#pragma unroll 8
        for (int c = g; c < nchunk; c += kRedGroups) s1 += (double)base[c * mat + sij];
    }
    s1s[g][e] = s1;
    s2s[g][e] = s2;
    __syncthreads();
    if (g == 0 && valid) {
        double t1 = 0.0, t2 = 0.0;
        for (int q = 0; q < kRedGroups; ++q) t1 += s1s[q][e];
        if (tiled) {
            const int et = 8 * (e & 7) + (e >> 3);             // S_ji: lane (c, r) of the mirror tile
            for (int q = 0; q < kRedGroups; ++q) t2 += s2s[q][et];
        }
        const double sv = 0.5 * (t1 + t2);
        const int64_t at = (int64_t)i * ld + j;
        double* o = out + p * out_stride + at;
        if (mode == 2)
            *o += sv;
        else if (mode == 1)
            *o = sv;
        else
            *o = t1;
        if (mode == 1 && copy) copy[at] = sv;
        if (p == sym_p) sym_to[at] += sv;
    }
}

// ------------------------------------------------------------------ update

// OUT = alpha IN + sum_p X_p S'_p with S'_p already in the block precision (and
// transposed / scaled by the caller's staging kernel). A workgroup owns 64*MT
// rows (4 waves x 16*MT) and up to 16*NTW columns. K (the ld columns of every
// X_p) is walked in chunks of 32: S'_p's chunk rows are staged in LDS (double
// buffered) and each lane reads its X row's chunk as vector runs. K is permuted
// inside a chunk: lane row lr of MFMA step (j, e) stands for k = 4 VW j + VW lr + e
// (VW = elements per 16 bytes), so a lane's VW values of one run feed VW steps.
// The next chunk's X runs and S' rows are fetched while the current one is used.
constexpr int kKC = 32;

template <typename T, int MT, int NTW>
__global__ __launch_bounds__(256) void k_update(T* OUT, const T* IN, double alpha, const T* __restrict__ X,
                                                int64_t xstride, int nprod, const T* __restrict__ S,
                                                int64_t Np, int ld, const int* __restrict__ state) {
    if (state && state[0]) return;
    typedef MF<T> M;
    constexpr int VW = M::VW;
    constexpr int NJ = kKC / (4 * VW);                        // runs per lane and row tile in a chunk
    constexpr int NC = 16 * NTW;                              // columns per workgroup
    constexpr int SP = NC + (sizeof(T) == 8 ? 8 : 16);        // padded LDS row
    constexpr int PER = (kKC * NC + 255) / 256;               // staged elements per thread
    __shared__ T sS[2][kKC * SP];
    const int l = threadIdx.x & 63, w = threadIdx.x >> 6, lr = l >> 4, lc = l & 15;
    const int64_t m0 = ((int64_t)blockIdx.x * 4 + w) * (16 * MT);
    const int jc0 = blockIdx.y * NC;
    const int ntw = min(NTW, (ld - jc0) / 16);
    const bool active = m0 < Np;
    const int64_t mat = (int64_t)ld * ld;
    const int nkc = (ld + kKC - 1) / kKC;
    const int total = nprod * nkc;
    typename M::acc c[MT][NTW];
#pragma unroll
    for (int a = 0; a < MT; ++a)
#pragma unroll
        for (int b = 0; b < NTW; ++b) c[a][b] = M::zero();

    auto fetch_s = [&](int it, T (&reg)[PER]) {
        const int p = it / nkc, kc = (it % nkc) * kKC;
        const T* Sp = S + (int64_t)p * mat;
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const int t = threadIdx.x + 256 * q;
            const int kk = t / NC, jj = t % NC;
            const int k = kc + kk, j = jc0 + jj;
            reg[q] = (t < kKC * NC && k < ld && j < ld) ? Sp[(int64_t)k * ld + j] : T(0);
        }
    };
    auto store_s = [&](int buf, const T (&reg)[PER]) {
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const int t = threadIdx.x + 256 * q;
            if (t < kKC * NC) sS[buf][(t / NC) * SP + t % NC] = reg[q];
        }
    };
    // this lane's runs of chunk it: x[mt][j][e] = X_p[m0 + 16 mt + lc][kc + 4 VW j + VW lr + e]
    auto fetch_x = [&](int it, T (&x)[MT][NJ][VW]) {
        const int p = it / nkc, kc = (it % nkc) * kKC;
        const int kend = min(kKC, ld - kc);
        const T* Xp = X + (int64_t)p * xstride + (m0 + lc) * ld + kc + VW * lr;
#pragma unroll
        for (int mt = 0; mt < MT; ++mt)
#pragma unroll
            for (int j = 0; j < NJ; ++j) {
                if (active && 4 * VW * j < kend) {
                    load_q<T, VW>(Xp + (int64_t)16 * mt * ld + 4 * VW * j, x[mt][j]);
                } else {
#pragma unroll
                    for (int e = 0; e < VW; ++e) x[mt][j][e] = T(0);
                }
            }
    };
    auto compute = [&](int buf, const T (&x)[MT][NJ][VW]) {
#pragma unroll
        for (int j = 0; j < NJ; ++j)
#pragma unroll
            for (int e = 0; e < VW; ++e) {
                const int k = 4 * VW * j + VW * lr + e;
#pragma unroll
                for (int nt = 0; nt < NTW; ++nt) {
                    if (nt < ntw) {
                        const T bv = sS[buf][k * SP + nt * 16 + lc];
#pragma unroll
                        for (int mt = 0; mt < MT; ++mt) c[mt][nt] = M::mma(x[mt][j][e], bv, c[mt][nt]);
                    }
                }
            }
    };
    T sreg[PER];
    T xa[MT][NJ][VW], xb[MT][NJ][VW];
    fetch_x(0, xa);
    fetch_s(0, sreg);
    store_s(0, sreg);
    // chunk `it` lives in sS[it & 1] and in xa (even it) / xb (odd it)
    for (int it = 0; it < total; it += 2) {
        if (it + 1 < total) {
            fetch_x(it + 1, xb);
            fetch_s(it + 1, sreg);
        }
        __syncthreads();                                  // sS[0] holds chunk it
        compute(0, xa);
        if (it + 1 < total) store_s(1, sreg);
        if (it + 1 >= total) break;
        if (it + 2 < total) {
            fetch_x(it + 2, xa);
            fetch_s(it + 2, sreg);
        }
        __syncthreads();                                  // sS[1] holds chunk it + 1
        compute(1, xb);
        if (it + 2 < total) store_s(0, sreg);
    }
    if (!active) return;
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
        for (int nt = 0; nt < NTW; ++nt) {
            if (nt < ntw) {
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int64_t row = m0 + 16 * mt + M::row(l, r);
                    const int col = jc0 + nt * 16 + lc;
                    const int64_t idx = row * ld + col;
                    double v = (double)c[mt][nt][r];
                    if (IN != nullptr && alpha != 0.0) v += alpha * (double)IN[idx];
                    OUT[idx] = T(v);
                }
            }
        }
}

// ------------------------------------------------------------------ BF16 correction
//
// W -= sum_p Q_p C_p where the coefficients C_p are corrections of the size of the
// basis' loss of orthogonality (full reorthogonalisation after the three-term
// update): each FP32 factor is split into two BF16 parts, x = hi + lo with
// hi = RNE(x), lo = RNE(x - hi), |x - hi - lo| <= 2^-17 |x|, and the product
// is hi*hi + hi*lo + lo*hi on the 16x16x32 BF16 MFMA (FP32 accumulation). The
// dropped and rounded parts are below 2^-15 |Q| |C| in each term, far under the
// FP32 rounding of W when C is as small as such corrections are.
//
// MFMA 16x16x32 BF16 layout (gfx950): lane l supplies A[l%16][k] and B[k][l%16]
// for the 8 K slots k of lane group l/16 (any assignment of K slots shared by A
// and B gives the same product); D[4(l/16)+r][l%16] in result register r.
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
constexpr int kSplitK = 32;


// Splits of 8 floats into NPL BF16 parts, x = x_0 + .. + x_{NPL-1},
// x_i = RNE(x - x_0 - .. - x_{i-1}), two elements at a time: one packed conversion,
// the parts back to FP32 by shifts (exact), one subtraction each.
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));

// Bits of the BF16 value nearest to x (ties to even).
__device__ __forceinline__ unsigned short bf16_bits(float x) {
    return __builtin_bit_cast(unsigned short, static_cast<__bf16>(x));
}
typedef unsigned u32x4 __attribute__((ext_vector_type(4)));

template <int NPL>
__device__ __forceinline__ void split_planes(const float (&x)[8], bf16x8 (&pl)[NPL]) {
    unsigned w[NPL][4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        f32x2 r = {x[2 * i], x[2 * i + 1]};
#pragma unroll
        for (int k = 0; k < NPL; ++k) {
            const unsigned bits = __builtin_bit_cast(unsigned, __builtin_convertvector(r, bf16x2));
            w[k][i] = bits;
            if (k + 1 < NPL) {
                const f32x2 back = {__uint_as_float(bits << 16), __uint_as_float(bits & 0xffff0000u)};
                r = r - back;
            }
        }
    }
#pragma unroll
    for (int k = 0; k < NPL; ++k) pl[k] = __builtin_bit_cast(bf16x8, u32x4{w[k][0], w[k][1], w[k][2], w[k][3]});
}

__device__ __forceinline__ void split_bf16(const float (&x)[8], bf16x8& hi, bf16x8& lo) {
    bf16x8 pl[2];
    split_planes<2>(x, pl);
    hi = pl[0];
    lo = pl[1];
}

// FP16 two-part split of s x (s a power of two, so s x is exact): s x = hi + lo + r with
// hi = RNE(s x), lo = RNE(s x - hi), |r| <= 2^-22 |s x| while lo is a normal FP16 number
// and <= 2^-25 below that (FP16 subnormals, which the MFMA honours). The residual
// s x - hi is exact in FP32; the compiler forms it with one mixed-precision FMA.
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ void split_f16(const float (&x)[8], float sc, f16x8 (&pl)[2]) {
    unsigned w[2][4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const f32x2 y = f32x2{x[2 * i], x[2 * i + 1]} * sc;
        const f16x2 h = __builtin_convertvector(y, f16x2);
        const f16x2 lo = __builtin_convertvector(y - __builtin_convertvector(h, f32x2), f16x2);
        w[0][i] = __builtin_bit_cast(unsigned, h);
        w[1][i] = __builtin_bit_cast(unsigned, lo);
    }
#pragma unroll
    for (int k = 0; k < 2; ++k) pl[k] = __builtin_bit_cast(f16x8, u32x4{w[k][0], w[k][1], w[k][2], w[k][3]});
}

// Power-of-two scales for the FP16 split of Krylov blocks (unit-norm columns, entries
// of about Np^-1/2) and of W (entries bounded by ||H||_2 <= ||H||_inf): the typical
// entry lands near 1, the largest at most 2^12 (Np < 2^24), far from FP16 overflow.
__device__ __forceinline__ float q_split_scale(int64_t Np) {
    const int e = (63 - __builtin_clzll((unsigned long long)(Np > 1 ? Np : 1))) / 2;
    return __builtin_ldexpf(1.f, e);
}
__device__ __forceinline__ float w_split_scale(int64_t Np, const double* hinf) {
    int e = 0;
    const double h = hinf ? *hinf : 1.0;
    if (h > 0.0 && isfinite(h)) frexp(h, &e);               // 2^(e-1) <= h < 2^e
    return __builtin_ldexpf(q_split_scale(Np), -e);
}

// B fragments of S'_p = scale * (trans ? S_p^T : S_p), rounded to FP32 and split in
// NPL parts: frag[((pk * NPL + plane) * NT + nt) * 64 + l][e] = plane of
// S'_p[32 kc + 8 (l/16) + e][16 nt + l%16] (pk = p nkc + kc, zero for rows beyond
// ld), followed by one all-zero chunk (pk = nprod nkc) that the update reads past
// the last chunk. With S1 set, products p >= 1 take S1 + (p - 1) sstride and trans1.
template <int NPL>
__global__ void k_frag_s(const double* __restrict__ S, int64_t sstride, int nprod, int ld, int trans, double scale,
                         const double* __restrict__ S1, int trans1, bf16x8* __restrict__ frag) {
    const int NT = ld / 16, nkc = (ld + kSplitK - 1) / kSplitK;
    const int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (idx >= ((int64_t)nprod * nkc + 1) * NT * 64) return;
    const int l = (int)(idx % 64), nt = (int)((idx / 64) % NT);
    const int64_t pk = idx / (64 * NT);
    const bool pad = pk == (int64_t)nprod * nkc;
    const int kc = (int)(pk % nkc);
    const int64_t p = pad ? 0 : pk / nkc;
    const double* Sp = (S1 && p >= 1) ? S1 + (p - 1) * sstride : S + p * sstride;
    if (S1 && p >= 1) trans = trans1;
    const int j = 16 * nt + (l & 15);
    float v[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) {
        const int k = kSplitK * kc + 8 * (l >> 4) + e;
        v[e] = (!pad && k < ld) ? static_cast<float>(scale * (trans ? Sp[(int64_t)j * ld + k] : Sp[(int64_t)k * ld + j]))
                                : 0.f;
    }
    bf16x8 pl[NPL];
    split_planes<NPL>(v, pl);
#pragma unroll
    for (int q = 0; q < NPL; ++q) frag[((pk * NPL + q) * NT + nt) * 64 + l] = pl[q];
}

// OUT = alpha IN + sum_p X_p S'_p for FP32 blocks with ld = 16 NT. A wave owns 16 MT
// rows and all ld columns; the X runs of a K chunk (8 consecutive elements per lane
// and row tile) are fetched D chunks ahead, the chunk's B fragments go through LDS
// (double buffered, shared by the four waves). The loop body has no branch: it runs
// whole rounds of D chunks, chunks past the end take the zero fragments, and X
// addresses are clamped into the block (a clamped value always meets a zero
// coefficient), so that every wait for a load can leave the later loads in flight.
template <int MT, int NT, int D, int NPL>
__global__ __launch_bounds__(256, 3) void k_update_split(float* OUT, const float* IN, double alpha,
                                                      const float* __restrict__ X, int64_t xstride, int nprod,
                                                      const bf16x8* __restrict__ frag, int64_t Np, int ld_arg,
                                                      const int* __restrict__ state,
                                                      unsigned short* __restrict__ OUT16) {
    constexpr int ld = 16 * NT;                           // the launcher passes ld = 16 NT
    (void)ld_arg;
    if (state && state[0]) return;
    constexpr int FR = NPL * NT * 64;                     // fragments of one K chunk
    constexpr int PER = (FR + 255) / 256;
    __shared__ bf16x8 sB[2][PER * 256];
    const int l = threadIdx.x & 63, w = threadIdx.x >> 6, lr = l >> 4, lc = l & 15;
    const int64_t m0 = ((int64_t)blockIdx.x * 4 + w) * (16 * MT);
    const bool active = m0 < Np;
    const int64_t mrow = active ? m0 : 0;                 // inactive waves read (and discard) rows 0..
    const int nkc = (ld + kSplitK - 1) / kSplitK;
    const int total = nprod * nkc;
    mf_f4 c[MT][NT];
#pragma unroll
    for (int a = 0; a < MT; ++a)
#pragma unroll
        for (int b = 0; b < NT; ++b) c[a][b] = mf_f4{0.f, 0.f, 0.f, 0.f};

    auto fetch_x = [&](int it, float (&x)[MT][8]) {
        const int p = it / nkc, k = min((it % nkc) * kSplitK + 8 * lr, ld - 8);
        const float* Xp = X + (int64_t)p * xstride + (mrow + lc) * ld + k;
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) {
            float a4[4], b4[4];
            load_q<float, 4>(Xp + (int64_t)16 * mt * ld, a4);
            load_q<float, 4>(Xp + (int64_t)16 * mt * ld + 4, b4);
#pragma unroll
            for (int e = 0; e < 4; ++e) { x[mt][e] = a4[e]; x[mt][4 + e] = b4[e]; }
        }
    };
    auto fetch_s = [&](int it, bf16x8 (&reg)[PER]) {
        const bf16x8* src = frag + (int64_t)it * FR;
#pragma unroll
        for (int q = 0; q < PER; ++q) reg[q] = src[min(threadIdx.x + 256 * q, (unsigned)FR - 1)];
    };
    auto store_s = [&](int buf, const bf16x8 (&reg)[PER]) {
#pragma unroll
        for (int q = 0; q < PER; ++q) sB[buf][threadIdx.x + 256 * q] = reg[q];
    };
    auto compute = [&](int buf, const float (&x)[MT][8]) {
        bf16x8 ap[MT][NPL];
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) split_planes<NPL>(x[mt], ap[mt]);
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) {
            bf16x8 bp[NPL];
#pragma unroll
            for (int q = 0; q < NPL; ++q) bp[q] = sB[buf][(q * NT + nt) * 64 + l];
#pragma unroll
            for (int mt = 0; mt < MT; ++mt) {
                // the terms of order >= 2^-16 (NPL = 3) or >= 2^-8 (NPL = 2), smallest first
                if constexpr (NPL == 3) {
                    c[mt][nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ap[mt][2], bp[0], c[mt][nt], 0, 0, 0);
                    c[mt][nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ap[mt][1], bp[1], c[mt][nt], 0, 0, 0);
                    c[mt][nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ap[mt][0], bp[2], c[mt][nt], 0, 0, 0);
                }
                c[mt][nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ap[mt][1], bp[0], c[mt][nt], 0, 0, 0);
                c[mt][nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ap[mt][0], bp[1], c[mt][nt], 0, 0, 0);
                c[mt][nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ap[mt][0], bp[0], c[mt][nt], 0, 0, 0);
            }
        }
    };
    float xr[D][MT][8];
#pragma unroll
    for (int d = 0; d < D; ++d) fetch_x(min(d, total - 1), xr[d]);
    // loads are issued in the order they are needed (vmcnt counts in order): the
    // coefficients of chunk it + 1 (stored after chunk it) one chunk ahead, then X
    // D chunks ahead
    bf16x8 sreg[PER];
    fetch_s(0, sreg);
    store_s(0, sreg);
    fetch_s(min(1, total), sreg);
    for (int it0 = 0; it0 < total; it0 += D) {
#pragma unroll
        for (int d = 0; d < D; ++d) {
            const int it = it0 + d;
            lds_barrier();                                // sB[it & 1] holds chunk it; chunk it - 1 done
            compute(it & 1, xr[d]);
            store_s((it + 1) & 1, sreg);
            fetch_s(min(it + 2, total), sreg);
            fetch_x(min(it + D, total - 1), xr[d]);       // D chunks ahead (clamped at the end)
            __builtin_amdgcn_sched_barrier(0);
        }
    }
    if (!active) return;
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
        for (int nt = 0; nt < NT; ++nt)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int64_t row = m0 + 16 * mt + 4 * lr + r;
                const int64_t idx = row * ld + nt * 16 + lc;
                double v = (double)c[mt][nt][r];
                if (IN != nullptr && alpha != 0.0) v += alpha * (double)IN[idx];
                const float o = static_cast<float>(v);
                OUT[idx] = o;
                if (OUT16) OUT16[idx] = bf16_bits(o);
            }
}

// OUT = alpha IN + sum_p X_p S'_p with X_p given as BF16 values (a rounded copy of an
// FP32 block) and S'_p as one BF16 part: one 16x16x32 BF16 MFMA per tile and K chunk.
// For coefficient blocks of the size of a loss of orthogonality (the correction of
// the re-orthogonalisation), each term is within 2^-8 |X||S| of the exact one, far
// under FP32 rounding of OUT. Structure as k_update_split (X runs fetched D chunks
// ahead, fragments double buffered in LDS, branch-free loop), with two K chunks per
// stage, so one work-group barrier per two chunks.
template <int MT, int NT, int D>
__global__ __launch_bounds__(256) void k_update_bf16x(float* OUT, const float* IN, double alpha,
                                                      const unsigned short* __restrict__ X, int64_t xstride, int nprod,
                                                      const bf16x8* __restrict__ frag, int64_t Np, int ld_arg,
                                                      const int* __restrict__ state) {
    constexpr int ld = 16 * NT;                           // the launcher passes ld = 16 NT
    (void)ld_arg;
    if (state && state[0]) return;
    constexpr int FR = NT * 64;                           // fragments of one K chunk
    constexpr int PER = (FR + 255) / 256;
    constexpr int CPS = 2;                                // K chunks per stage (one barrier per stage)
    __shared__ bf16x8 sB[2][CPS][PER * 256];
    const int l = threadIdx.x & 63, w = threadIdx.x >> 6, lr = l >> 4, lc = l & 15;
    const int64_t m0 = ((int64_t)blockIdx.x * 4 + w) * (16 * MT);
    const bool active = m0 < Np;
    const int64_t mrow = active ? m0 : 0;
    const int nkc = (ld + kSplitK - 1) / kSplitK;
    const int total = nprod * nkc;
    const int nstage = (total + CPS - 1) / CPS;
    mf_f4 c[MT][NT];
#pragma unroll
    for (int a = 0; a < MT; ++a)
#pragma unroll
        for (int b = 0; b < NT; ++b) c[a][b] = mf_f4{0.f, 0.f, 0.f, 0.f};
    // chunk it: X runs clamped to the last chunk (past the end they meet the zero
    // fragments), fragments clamped to the zero chunk `total`
    auto fetch_x = [&](int st, bf16x8 (&x)[CPS][MT]) {
#pragma unroll
        for (int q = 0; q < CPS; ++q) {
            const int it = min(CPS * st + q, total - 1);
            const int p = it / nkc, k = min((it % nkc) * kSplitK + 8 * lr, ld - 8);
            const unsigned short* Xp = X + (int64_t)p * xstride + (mrow + lc) * ld + k;
#pragma unroll
            for (int mt = 0; mt < MT; ++mt) x[q][mt] = *reinterpret_cast<const bf16x8*>(Xp + (int64_t)16 * mt * ld);
        }
    };
    auto fetch_s = [&](int st, bf16x8 (&reg)[CPS][PER]) {
#pragma unroll
        for (int q = 0; q < CPS; ++q) {
            const bf16x8* src = frag + (int64_t)min(CPS * st + q, total) * FR;
#pragma unroll
            for (int e = 0; e < PER; ++e) reg[q][e] = src[min(threadIdx.x + 256 * e, (unsigned)FR - 1)];
        }
    };
    auto store_s = [&](int buf, const bf16x8 (&reg)[CPS][PER]) {
#pragma unroll
        for (int q = 0; q < CPS; ++q)
#pragma unroll
            for (int e = 0; e < PER; ++e) sB[buf][q][threadIdx.x + 256 * e] = reg[q][e];
    };
    auto compute = [&](int buf, const bf16x8 (&x)[CPS][MT]) {
#pragma unroll
        for (int q = 0; q < CPS; ++q)
#pragma unroll
            for (int nt = 0; nt < NT; ++nt) {
                const bf16x8 bp = sB[buf][q][nt * 64 + l];
#pragma unroll
                for (int mt = 0; mt < MT; ++mt)
                    c[mt][nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(x[q][mt], bp, c[mt][nt], 0, 0, 0);
            }
    };
    // D K chunks in flight: D / CPS stages of X runs ahead, fragments one stage ahead
    constexpr int DS = D / CPS > 0 ? D / CPS : 1;
    bf16x8 xr[DS][CPS][MT];
#pragma unroll
    for (int d = 0; d < DS; ++d) fetch_x(d, xr[d]);
    bf16x8 sreg[CPS][PER];
    fetch_s(0, sreg);
    store_s(0, sreg);
    fetch_s(1, sreg);
    for (int st0 = 0; st0 < nstage; st0 += DS) {
#pragma unroll
        for (int d = 0; d < DS; ++d) {
            const int st = st0 + d;
            lds_barrier();                                // sB[st & 1] holds stage st; stage st - 1 done
            compute(st & 1, xr[d]);
            store_s((st + 1) & 1, sreg);
            fetch_s(st + 2, sreg);
            fetch_x(st + DS, xr[d]);
            __builtin_amdgcn_sched_barrier(0);
        }
    }
    if (!active) return;
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
        for (int nt = 0; nt < NT; ++nt)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int64_t row = m0 + 16 * mt + 4 * lr + r;
                const int64_t idx = row * ld + nt * 16 + lc;
                double v = (double)c[mt][nt][r];
                if (IN != nullptr && alpha != 0.0) v += alpha * (double)IN[idx];
                OUT[idx] = static_cast<float>(v);
            }
}

// BF16 (round to nearest even) copy of an FP32 array.
__global__ void k_to_bf16(const float* __restrict__ in, unsigned short* __restrict__ out, int64_t n) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < n) out[i] = bf16_bits(in[i]);
}

// Y (Np x ld FP32, Np a multiple of 8) split into NPL BF16 planes in the operand
// layout of the 16x16x32 MFMA: plane q, 8-row group r8, column c holds the 8 parts
// of Y[8 r8 .. 8 r8 + 7][c] (16 bytes) at q (Np / 8) ld + r8 ld + c. One thread per
// (r8, c); the parts are those of split_planes.
// F16: the two FP16 parts of w_split_scale(Np, hinf) Y instead (same layout).
template <int NPL, bool F16>
__global__ __launch_bounds__(256) void k_split_rows8(const float* __restrict__ Y, int64_t Np, int ld,
                                                     bf16x8* __restrict__ P, const int* __restrict__ state,
                                                     const double* __restrict__ hinf) {
    if (state && state[0]) return;
    const int64_t cnt = (Np / 8) * ld;
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= cnt) return;
    const int64_t r8 = i / ld;
    const int c = (int)(i % ld);
    float v[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) v[e] = Y[(8 * r8 + e) * ld + c];
    if constexpr (F16) {
        static_assert(NPL == 2, "two FP16 parts");
        f16x8 pl[2];
        split_f16(v, w_split_scale(Np, hinf), pl);
#pragma unroll
        for (int q = 0; q < 2; ++q) P[q * cnt + i] = __builtin_bit_cast(bf16x8, pl[q]);
    } else {
        bf16x8 pl[NPL];
        split_planes<NPL>(v, pl);
#pragma unroll
        for (int q = 0; q < NPL; ++q) P[q * cnt + i] = pl[q];
    }
}

// ------------------------------------------------------------------ BF16 Gram
//
// X_p^T Y for FP32 blocks on the 16x16x32 BF16 MFMA, with every factor split
// into NPL BF16 parts x = x0 + x1 (+ x2), x_i = RNE(x - x_0 - .. - x_{i-1}):
// NPL = 3 keeps the six products of order >= 2^-16 (x0y0, x0y1, x1y0, x0y2, x1y1,
// x2y0), each term then carries a relative error of a few 2^-24, no more than the
// rounding of the FP32 product it replaces; NPL = 2 keeps x0y0 + x0y1 + x1y0
// (a few 2^-17 per term). Accumulation is FP32 in the MFMA, at most kGramFp32Rows
// rows per wave before the FP64 reduction, as in k_gram.
// One workgroup of four waves per (chunk, p): NH column parts x 4/NH row groups.
// Wave (grp, h) owns the ld x (ld/NH) tile of Y columns [h ld/NH, (h+1) ld/NH) and
// takes the 32-row steps grp, grp + 4/NH, ... of the chunk; a lane holds the 8 rows
// 8 (l/16) .. + 7 of a step (its K slots), for X the columns seg_col(a, l%16) of
// each tile a, for Y the column 16 b + l%16 of each of its tiles b. Operands are
// fetched one step ahead (the chunk's steps per wave are even, see
// gram_plan_split). The row groups' tiles are added in LDS in group order and
// written as one partial, as in k_gram. The products of a chunk run together on one
// XCD, so the workgroups that read the same Y rows share that XCD's L2.
// YP: Y given as its NPL BF16 planes (k_split_rows8), loaded as ready operands.
// F16 (with YP, NPL = 2): two FP16 parts of q_split_scale X and w_split_scale Y, the
// three products lo*hi + hi*lo + hi*hi on the FP16 MFMA (dropped and rounded parts
// below 3 2^-22 of each term), the partial scaled back exactly.
template <int NT, int NH, int NPL, bool YP, bool F16>
__global__ __launch_bounds__(256, F16 ? 2 : 1) void k_gram_split(const float* __restrict__ X, int64_t xstride,
                                                    const float* __restrict__ Y, const bf16x8* __restrict__ Yp,
                                                    int64_t Np, int64_t rpc, int ld_arg, float* __restrict__ partial,
                                                    int nchunk, const int* __restrict__ state,
                                                    const double* __restrict__ hinf) {
    constexpr int ld = 16 * NT;                           // the launcher passes ld = 16 NT: row offsets fold into immediates
    (void)ld_arg;
    static_assert(!F16 || (YP && NPL == 2), "FP16 parts come with the pre-split Y");
    if (state && state[0]) return;
    constexpr int TILE = 16 * NT, NB = NT / NH, KG = 4 / NH;
    static_assert(NT % NH == 0 && (NH == 1 || NH == 2), "column parts");
    extern __shared__ char gram_lds[];
    float* buf = reinterpret_cast<float*>(gram_lds);
    const int l = threadIdx.x & 63, w = threadIdx.x >> 6, lr = l >> 4, lc = l & 15;
    const int grp = w / NH, h = w % NH;
    // Workgroups are dealt round-robin to the 8 XCDs: XCD x takes chunks x, x + 8, ...
    // with all their products, so the products of a chunk share its Y rows in one L2.
    const int nprod = (int)(gridDim.x / (8 * ((nchunk + 7) / 8)));
    const int xcd = (int)(blockIdx.x % 8), k = (int)(blockIdx.x / 8);
    const int p = k % nprod, chunk = (k / nprod) * 8 + xcd;
    if (chunk >= nchunk) return;
    const int64_t r0 = (int64_t)chunk * rpc;
    const int64_t r1 = r0 + rpc < Np ? r0 + rpc : Np;
    const int nst = (int)((r1 - r0) / (32 * KG));         // steps of this wave (even)
    mf_f4 c[NT][NB];
#pragma unroll
    for (int a = 0; a < NT; ++a)
#pragma unroll
        for (int b = 0; b < NB; ++b) c[a][b] = mf_f4{0.f, 0.f, 0.f, 0.f};
    const int64_t step = 32 * KG * (int64_t)ld;
    const float* xa = X + (int64_t)p * xstride + (r0 + 32 * grp + 8 * lr) * ld;
    const float* ya = Y + (r0 + 32 * grp + 8 * lr) * ld + 16 * NB * h + lc;
    // plane layout: plane q, 8-row group r8, column c at q (Np / 8) ld + r8 ld + c
    const int64_t pstride = (Np / 8) * ld;
    const bf16x8* ypa = Yp + ((r0 + 32 * grp + 8 * lr) / 8) * ld + 16 * NB * h + lc;
    typedef typename std::conditional<YP, bf16x8[NB][NPL], float[8][NB]>::type YBuf;
    auto fetch = [&](int st, float (&x)[8][NT], YBuf& y) {
        const int64_t o = (int64_t)st * step;
#pragma unroll
        for (int e = 0; e < 8; ++e) load_run<float, NT>(xa + o + (int64_t)e * ld, lc, x[e]);
        if constexpr (YP) {
            const int64_t o8 = (int64_t)st * (4 * KG) * ld;
#pragma unroll
            for (int b = 0; b < NB; ++b)
#pragma unroll
                for (int q = 0; q < NPL; ++q) y[b][q] = ypa[q * pstride + o8 + 16 * b];
        } else {
#pragma unroll
            for (int e = 0; e < 8; ++e)
#pragma unroll
                for (int b = 0; b < NB; ++b) y[e][b] = ya[o + (int64_t)e * ld + 16 * b];
        }
    };
    // The split of tile a + 1 is issued between the MFMAs of tile a: with one wave
    // per SIMD the VALU work then runs while the matrix core is busy instead of
    // after it (an MFMA blocks the wave's next MFMA, not its VALU instructions).
    const float xsc = F16 ? q_split_scale(Np) : 1.f;
    auto compute = [&](const float (&x)[8][NT], const YBuf& y) {
        bf16x8 yb[NB][NPL];
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            if constexpr (YP) {
#pragma unroll
                for (int q = 0; q < NPL; ++q) yb[b][q] = y[b][q];
            } else {
                float v[8];
#pragma unroll
                for (int e = 0; e < 8; ++e) v[e] = y[e][b];
                split_planes<NPL>(v, yb[b]);
            }
        }
        bf16x8 xb[2][NPL];
        auto split_x = [&](const float (&v)[8], bf16x8 (&o)[NPL]) {
            if constexpr (F16) {
                f16x8 t[2];
                split_f16(v, xsc, t);
#pragma unroll
                for (int q = 0; q < 2; ++q) o[q] = __builtin_bit_cast(bf16x8, t[q]);
            } else {
                split_planes<NPL>(v, o);
            }
        };
        {
            float v[8];
#pragma unroll
            for (int e = 0; e < 8; ++e) v[e] = x[e][0];
            split_x(v, xb[0]);
        }
#pragma unroll
        for (int a = 0; a < NT; ++a) {
            const bf16x8 (&xc)[NPL] = xb[a & 1];
            if (a + 1 < NT) {
                float v[8];
#pragma unroll
                for (int e = 0; e < 8; ++e) v[e] = x[e][a + 1];
                split_x(v, xb[(a + 1) & 1]);
            }
            // the product terms in the outer loop: an accumulator's next MFMA comes NB
            // instructions later, not right after its previous one (same order of terms)
            if constexpr (F16) {
                const f16x8 x0 = __builtin_bit_cast(f16x8, xc[0]), x1 = __builtin_bit_cast(f16x8, xc[1]);
#pragma unroll
                for (int b = 0; b < NB; ++b)
                    c[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_f16(x1, __builtin_bit_cast(f16x8, yb[b][0]), c[a][b],
                                                                     0, 0, 0);
#pragma unroll
                for (int b = 0; b < NB; ++b)
                    c[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_f16(x0, __builtin_bit_cast(f16x8, yb[b][1]), c[a][b],
                                                                     0, 0, 0);
#pragma unroll
                for (int b = 0; b < NB; ++b)
                    c[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_f16(x0, __builtin_bit_cast(f16x8, yb[b][0]), c[a][b],
                                                                     0, 0, 0);
            } else {
                if constexpr (NPL == 3) {
#pragma unroll
                    for (int b = 0; b < NB; ++b)
                        c[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xc[2], yb[b][0], c[a][b], 0, 0, 0);
#pragma unroll
                    for (int b = 0; b < NB; ++b)
                        c[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xc[1], yb[b][1], c[a][b], 0, 0, 0);
#pragma unroll
                    for (int b = 0; b < NB; ++b)
                        c[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xc[0], yb[b][2], c[a][b], 0, 0, 0);
                }
#pragma unroll
                for (int b = 0; b < NB; ++b)
                    c[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xc[1], yb[b][0], c[a][b], 0, 0, 0);
#pragma unroll
                for (int b = 0; b < NB; ++b)
                    c[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xc[0], yb[b][1], c[a][b], 0, 0, 0);
#pragma unroll
                for (int b = 0; b < NB; ++b)
                    c[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xc[0], yb[b][0], c[a][b], 0, 0, 0);
            }
            if (a + 1 < NT) {
#pragma unroll
                for (int q = 0; q < NB * (F16 ? 3 : 2 * NPL); ++q) {
                    __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);    // one MFMA
                    __builtin_amdgcn_sched_group_barrier(0x002, 3, 0);    // then up to three VALU
                }
            }
        }
    };
    float x0[8][NT], x1[8][NT];
    YBuf y0, y1;
    if (nst > 0) fetch(0, x0, y0);
    for (int st = 0; st < nst; st += 2) {
        fetch(st + 1, x1, y1);                            // nst is even
        __builtin_amdgcn_sched_barrier(0);
        compute(x0, y0);
        fetch(min(st + 2, nst - 1), x0, y0);              // the last step again at the end (not used)
        __builtin_amdgcn_sched_barrier(0);
        compute(x1, y1);
    }
    // row groups' tiles added into LDS in group order (tile-local coordinates)
#pragma unroll
    for (int g = 0; g < KG; ++g) {
        if (grp == g) {
#pragma unroll
            for (int a = 0; a < NT; ++a)
#pragma unroll
                for (int b = 0; b < NB; ++b)
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const int row = seg_col<NT, 4>(a, 4 * lr + r);
                        const int col = 16 * (NB * h + b) + lc;
                        float& e = buf[row * TILE + col];
                        e = (g == 0) ? c[a][b][r] : e + c[a][b][r];
                        if (r == 3) __builtin_amdgcn_sched_barrier(0);
                    }
        }
        __syncthreads();
    }
    float* out = partial + ((int64_t)p * nchunk + chunk) * ld * ld;
    if constexpr (F16) {
        const float unscale = 1.f / (xsc * w_split_scale(Np, hinf));   // a power of two
        for (int e = threadIdx.x; e < TILE * TILE; e += 256) out[e] = buf[e] * unscale;
    } else {
        for (int e = threadIdx.x; e < TILE * TILE; e += 256) out[e] = buf[e];
    }
}

// S'_p = scale * (trans ? S_p^T : S_p) in the block precision.
template <typename T>
__global__ void k_stage_s(const double* __restrict__ S, int64_t sstride, int nprod, int ld, int trans,
                          double scale, T* __restrict__ out) {
    const int64_t mat = (int64_t)ld * ld;
    const int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (idx >= nprod * mat) return;
    const int64_t p = idx / mat;
    const int k = (int)((idx % mat) / ld), j = (int)(idx % ld);
    const double* Sp = S + p * sstride;
    out[idx] = T(scale * (trans ? Sp[(int64_t)j * ld + k] : Sp[(int64_t)k * ld + j]));
}

// ------------------------------------------------------------------ small FP64

// Cholesky G = R^T R (R upper) and R^-1 for b <= 16*NB with a 16 x 16 thread grid;
// thread (ty, tx) keeps entries (ty + 16a, tx + 16c) in registers.
template <int NB>
__global__ __launch_bounds__(256) void k_chol_inv_reg(const double* __restrict__ G, int b, int ld,
                                                      const double* __restrict__ tau_p, double* __restrict__ R,
                                                      double* __restrict__ Rinv, int* state, int step,
                                                      double* __restrict__ min_diag) {
    __shared__ double rowk[16 * NB];
    __shared__ double colk[16 * NB];
    __shared__ double rdiag[16 * NB];
    __shared__ double rinvd[16 * NB];
    __shared__ int fail;
    __shared__ double dmin;
    if (state[0]) return;
    const double tau = tau_p ? *tau_p : 0.0;
    const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
    double m[NB][NB];
#pragma unroll
    for (int a = 0; a < NB; ++a)
#pragma unroll
        for (int c = 0; c < NB; ++c) {
            const int i = ty + 16 * a, j = tx + 16 * c;
            m[a][c] = (i < b && j < b && j >= i) ? G[(int64_t)i * ld + j] : 0.0;
        }
    if (threadIdx.x == 0) { fail = 0; dmin = INFINITY; }
    __syncthreads();
    for (int k = 0; k < b; ++k) {
        const int ka = k >> 4, kt = k & 15;
        if (ty == kt && tx == kt) {                 // owner of (k, k) takes the pivot
#pragma unroll
            for (int a = 0; a < NB; ++a)
                if (a == ka) {
                    const double piv = m[a][a];
                    if (!(piv > 0.0) || !isfinite(piv)) {
                        fail = 1;
                    } else {
                        const double d = sqrt(piv);
                        dmin = fmin(dmin, d);
                        if (!(d > tau)) fail = 1;
                        rdiag[k] = d;
                        rinvd[k] = 1.0 / d;
                    }
                }
        }
        __syncthreads();
        if (fail) break;
        const double d = rdiag[k], dinv = rinvd[k];
        if (ty == kt) {                             // owners of row k scale it and publish it
#pragma unroll
            for (int a = 0; a < NB; ++a)
                if (a == ka) {
#pragma unroll
                    for (int c = 0; c < NB; ++c) {
                        const int j = tx + 16 * c;
                        if (j > k && j < b) {
                            m[a][c] *= dinv;
                            rowk[j] = m[a][c];
                        } else if (j == k) {
                            m[a][c] = d;
                        }
                    }
                }
        }
        __syncthreads();
#pragma unroll
        for (int a = 0; a < NB; ++a) {              // trailing update of the upper triangle
            const int i = ty + 16 * a;
            if (i > k && i < b) {
                const double rki = rowk[i];
#pragma unroll
                for (int c = 0; c < NB; ++c) {
                    const int j = tx + 16 * c;
                    if (j >= i && j < b) m[a][c] -= rki * rowk[j];
                }
            }
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) min_diag[step] = dmin;
    if (fail) {
        for (int idx = threadIdx.x; idx < ld * ld; idx += 256) { Rinv[idx] = 0.0; R[idx] = 0.0; }
        __syncthreads();
        if (threadIdx.x == 0) { state[2] = step; state[0] = 1; }
        return;
    }
    // R to global (zero outside the upper b x b triangle)
    for (int idx = threadIdx.x; idx < ld * ld; idx += 256) {
        const int i = idx / ld, j = idx % ld;
        if (i >= 16 * NB || j >= 16 * NB || i >= b || j >= b || j < i) R[idx] = 0.0;
    }
#pragma unroll
    for (int a = 0; a < NB; ++a)
#pragma unroll
        for (int c = 0; c < NB; ++c) {
            const int i = ty + 16 * a, j = tx + 16 * c;
            if (i < b && j < b && j >= i) R[(int64_t)i * ld + j] = m[a][c];
        }
    // R^-1 = X by back substitution, X initialised to the identity: row i of X is
    // final once divided by R[i][i]; then X[i'][:] -= R[i'][i] X[i][:] for i' < i
    double x[NB][NB];
#pragma unroll
    for (int a = 0; a < NB; ++a)
#pragma unroll
        for (int c = 0; c < NB; ++c) x[a][c] = ((ty + 16 * a) == (tx + 16 * c)) ? 1.0 : 0.0;
    for (int i = b - 1; i >= 0; --i) {
        const int ia = i >> 4, it = i & 15;
        if (ty == it) {
            const double rii = rinvd[i];
#pragma unroll
            for (int a = 0; a < NB; ++a)
                if (a == ia) {
#pragma unroll
                    for (int c = 0; c < NB; ++c) {
                        const int j = tx + 16 * c;
                        if (j < b) {
                            x[a][c] *= rii;
                            rowk[j] = x[a][c];
                        }
                    }
                }
        }
        if (tx == it) {
#pragma unroll
            for (int c = 0; c < NB; ++c)
                if (c == ia) {
#pragma unroll
                    for (int a = 0; a < NB; ++a) {
                        const int ip = ty + 16 * a;
                        if (ip < i) colk[ip] = m[a][c];
                    }
                }
        }
        __syncthreads();
#pragma unroll
        for (int a = 0; a < NB; ++a) {
            const int ip = ty + 16 * a;
            if (ip < i) {
                const double r = colk[ip];
#pragma unroll
                for (int c = 0; c < NB; ++c) {
                    const int j = tx + 16 * c;
                    if (j >= i && j < b) x[a][c] -= r * rowk[j];
                }
            }
        }
        __syncthreads();
    }
    for (int idx = threadIdx.x; idx < ld * ld; idx += 256) {
        const int i = idx / ld, j = idx % ld;
        if (i >= 16 * NB || j >= 16 * NB || i >= b || j >= b || j < i) Rinv[idx] = 0.0;
    }
#pragma unroll
    for (int a = 0; a < NB; ++a)
#pragma unroll
        for (int c = 0; c < NB; ++c) {
            const int i = ty + 16 * a, j = tx + 16 * c;
            if (i < b && j < b && j >= i) Rinv[(int64_t)i * ld + j] = x[a][c];
        }
}

// Blocks of 16 (NB blocks, b <= 16 NB): Cholesky G = R^T R of the leading b x b
// block and X = R^-1.
// LDS holds the 16NB x 16NB matrix M (row stride W): G (mirrored from its upper
// triangle), then R in the upper triangle;
// rows/columns b..16NB-1 are padded with the identity. Diagonal blocks are factored
// and inverted in registers (MFMA D layout: lane l holds rows (l>>4)+4r, column l&15)
// with cross-lane broadcasts; panel solves R_kj = R_kk^-T A_kj, trailing updates
// A_ij -= R_ki^T R_kj and the blocked inverse X_ij = -X_ii sum_{k=i+1..j} R_ik X_kj
// run on FP64 MFMA. The X_jj are kept in XD (D layout); the X_ij (i < j) are stored
// transposed in the strictly lower block triangle of M. Four waves: wave 0 factors
// and inverts the diagonal blocks, the next one during the trailing update of the
// current step (look-ahead), which waves 1..3 do for the other tiles; the panel
// tiles are dealt to all four; two work-group barriers per block step; the block
// columns of the inverse are independent and dealt to the waves.
template <int NB>
__device__ __forceinline__ void chol_inv_blk(const double* __restrict__ G, int b, int ld, const double* __restrict__ tau_p,
                             double* __restrict__ R, double* __restrict__ Rinv, int* state, int step,
                             double* __restrict__ min_diag, double* chol_lds) {
    constexpr int N = 16 * NB, W = N + 1;
    double* M = chol_lds;                 // N x W
    double* XD = chol_lds + N * W;        // NB x 256 (D layout)
    __shared__ int sfail;
    typedef MF<double> Mf;
    const int t = threadIdx.x, l = t & 63, wv = t >> 6, lr = l >> 4, lc = l & 15;
    const double tau = tau_p ? *tau_p : 0.0;
    {
        // G from its upper triangle, mirrored (the diagonal tiles stay symmetric through
        // the trailing updates, so their factorisation reads a pivot column in-row); all
        // loads issued before the LDS stores
        constexpr int PER = (N * N + 255) / 256;
        double v[PER];
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const int e = t + 256 * q;
            const int i = e / N, j = e % N;
            v[q] = (e < N * N && i < b && j < b) ? G[(int64_t)min(i, j) * ld + max(i, j)] : 0.0;
        }
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const int e = t + 256 * q;
            const int i = e / N, j = e % N;
            if (e < N * N) M[i * W + j] = (i >= b && i == j) ? 1.0 : v[q];
        }
    }
    if (t == 0) sfail = 0;
    __syncthreads();
    double dmin = INFINITY;
    // (a)-(c) of block kb by wave 0: unblocked Cholesky of the symmetric 16 x 16 diagonal
    // block in registers (pivot by readlane, the pivot row to every row group by lane
    // swaps, the pivot column within each row group by DPP broadcast: VALU moves only),
    // R_kk into M, X_kk = R_kk^-1 by backward substitution into XD; a failure sets sfail
    auto diag_block = [&](int kb) {
        const int o = 16 * kb;
        bool fail = false;
        double a[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) a[r] = M[(o + lr + 4 * r) * W + o + lc];
        double dinv[16];
        static_steps([&](auto kc) {
            constexpr int k = decltype(kc)::value, rk = k >> 2, g = k & 3;
            const double piv = lane_read(a[rk], 16 * g + k);
            double d = 1.0, di = 1.0;
            if (o + k < b && !fail) {                   // uniform: piv is the same in every lane
                if (!(piv > 0.0) || !isfinite(piv)) {
                    fail = true;
                } else {
                    di = rsqrt_newton(piv);
                    d = piv * di;
                    dmin = fmin(dmin, d);
                    if (!(d > tau)) fail = true;
                }
            }
            dinv[k] = di;                               // after a failure the block is discarded
            double c[4];
#pragma unroll
            for (int r = 0; r < 4; ++r) c[r] = col_bcast<k>(a[r]);      // column k of my rows
            const double rk_row = lc > k ? a[rk] * di : (lc == k ? d : 0.0);   // R_k,lc
            a[rk] = lr == g ? rk_row : a[rk];
            const double vj = grp_bcast<g>(rk_row);
#pragma unroll
            for (int r = 0; r < 4; ++r) {                               // both triangles, branch-free
                const double upd = __builtin_fma(-(c[r] * di), vj, a[r]);
                a[r] = (lr + 4 * r > k && lc > k) ? upd : a[r];
            }
        }, std::make_integer_sequence<int, 16>{});
        if (fail) {
            if (l == 0) sfail = 1;
            return;
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) M[(o + lr + 4 * r) * W + o + lc] = a[r];
        double x[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) x[r] = (lr + 4 * r == lc) ? 1.0 : 0.0;
        static_steps([&](auto ic) {
            constexpr int i = 15 - decltype(ic)::value, ri = i >> 2, g = i & 3;
            const double xrow = x[ri] * dinv[i];                        // X row i, column lc
            x[ri] = lr == g ? xrow : x[ri];
            const double xij = grp_bcast<g>(xrow);
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const double rii = col_bcast<i>(a[r]);                 // R_kk[lr + 4r][i]
                const double upd = __builtin_fma(-rii, xij, x[r]);
                x[r] = lr + 4 * r < i ? upd : x[r];
            }
        }, std::make_integer_sequence<int, 16>{});
#pragma unroll
        for (int r = 0; r < 4; ++r) XD[kb * 256 + r * 64 + l] = x[r];
    };
    // A_ij -= R_ki^T R_kj for one tile
    auto trailing = [&](int ib, int jb, int o) {
        Mf::acc c;
#pragma unroll
        for (int r = 0; r < 4; ++r) c[r] = M[(16 * ib + lr + 4 * r) * W + 16 * jb + lc];
#pragma unroll
        for (int s4 = 0; s4 < 4; ++s4)
            c = Mf::mma(-M[(o + 4 * s4 + lr) * W + 16 * ib + lc], M[(o + 4 * s4 + lr) * W + 16 * jb + lc], c);
#pragma unroll
        for (int r = 0; r < 4; ++r) M[(16 * ib + lr + 4 * r) * W + 16 * jb + lc] = c[r];
    };
    // block column jb of X = R^-1, tiles upwards: X_ij = -X_ii sum_{k=i+1..j} R_ik X_kj,
    // X_ij^T stored in the strictly lower block triangle of M (which the factorisation
    // no longer reads); needs R's block columns <= jb and the X_kk
    auto inv_column = [&](int jb) {
        for (int ib = jb - 1; ib >= 0; --ib) {
            Mf::acc tv = Mf::zero();
            for (int kb = ib + 1; kb <= jb; ++kb) {
#pragma unroll
                for (int s4 = 0; s4 < 4; ++s4) {
                    const double av = M[(16 * ib + lc) * W + 16 * kb + 4 * s4 + lr];          // R_ik[lc][4s+lr]
                    const double bv = kb == jb ? XD[jb * 256 + s4 * 64 + l]                    // X_jj[4s+lr][lc]
                                               : M[(16 * jb + lc) * W + 16 * kb + 4 * s4 + lr];  // X_kj^T
                    tv = Mf::mma(av, bv, tv);
                }
            }
            Mf::acc c = Mf::zero();
#pragma unroll
            for (int s4 = 0; s4 < 4; ++s4) {
                const int li = lc, lj = 4 * s4 + lr;                   // X_ii[lc][4s+lr]
                const double av = XD[ib * 256 + (li >> 2) * 64 + 16 * (li & 3) + lj];
                c = Mf::mma(-av, tv[s4], c);
            }
#pragma unroll
            for (int r = 0; r < 4; ++r) M[(16 * jb + lc) * W + 16 * ib + lr + 4 * r] = c[r];
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        }
    };
    if (wv == 0) diag_block(0);
    __syncthreads();
    // Look-ahead: in block step kb, after the panel, wave 0 updates the next diagonal
    // tile and factors it while waves 1..3 update the other trailing tiles; then one of
    // them forms block column kb of the inverse (R's block columns <= kb and X_kk are
    // final by then), so that only the last column is left after the factorisation.
    for (int kb = 0; kb < NB && !sfail; ++kb) {
        const int o = 16 * kb;
        // (d) panel R_kj = X_kk^T A_kj, tiles dealt to the waves
        for (int jb = kb + 1 + wv; jb < NB; jb += 4) {
            Mf::acc c = Mf::zero();
#pragma unroll
            for (int s4 = 0; s4 < 4; ++s4)
                c = Mf::mma(XD[kb * 256 + s4 * 64 + l], M[(o + 4 * s4 + lr) * W + 16 * jb + lc], c);
#pragma unroll
            for (int r = 0; r < 4; ++r) M[(o + lr + 4 * r) * W + 16 * jb + lc] = c[r];
        }
        __syncthreads();
        if (kb + 1 < NB) {
            const int k1 = kb + 1;
            if (wv == 0) {
                trailing(k1, k1, o);
                __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");   // the tile's LDS writes before its reads
                diag_block(k1);
            } else {
                // (e) the other trailing tiles kb < i <= j, dealt to waves 1..3
                int tile = 0;
                for (int ib = k1; ib < NB; ++ib)
                    for (int jb = ib; jb < NB; ++jb) {
                        if (ib == k1 && jb == k1) continue;
                        if (tile++ % 3 != wv - 1) continue;
                        trailing(ib, jb, o);
                    }
                if (kb >= 1 && wv == 1 + kb % 3) inv_column(kb);
            }
            __syncthreads();
        }
    }
    if (t == 0) min_diag[step] = dmin;
    if (sfail) {
        for (int idx = t; idx < ld * ld; idx += 256) { Rinv[idx] = 0.0; R[idx] = 0.0; }
        if (t == 0) { state[2] = step; state[0] = 1; }
        return;
    }
    // the last block column of the inverse (the others were formed during the factorisation)
    if (NB > 1 && wv == 0) inv_column(NB - 1);
    __syncthreads();
    // ld == N (checked by the launcher): constant index arithmetic; two adjacent
    // elements per thread (one 16-byte store each to R and R^-1), branch-free
    for (int e2 = t; e2 < N * N / 2; e2 += 256) {
        const int idx = 2 * e2, i = idx / N, j = idx % N;    // j even: j, j + 1 in one block column
        const int bi = i >> 4, bj = j >> 4, li = i & 15, lj = j & 15;
        double rv[2], xv[2];
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            const int jj = j + q;
            const double r = M[i * W + jj];
            const double xd = XD[bi * 256 + (li >> 2) * 64 + 16 * (li & 3) + lj + q];
            const double xm = M[jj * W + i];
            const bool in = i < b && jj < b && jj >= i;
            rv[q] = in ? r : 0.0;
            xv[q] = in ? (bi == bj ? xd : xm) : 0.0;
        }
        *reinterpret_cast<double2*>(R + idx) = make_double2(rv[0], rv[1]);
        *reinterpret_cast<double2*>(Rinv + idx) = make_double2(xv[0], xv[1]);
    }
}

template <int NB>
__global__ __launch_bounds__(256) void k_chol_inv_blk(const double* __restrict__ G, int b, int ld,
                                                      const double* __restrict__ tau_p, double* __restrict__ R,
                                                      double* __restrict__ Rinv, int* state, int step,
                                                      double* __restrict__ min_diag) {
    extern __shared__ double chol_lds[];
    if (state[0]) return;
    chol_inv_blk<NB>(G, b, ld, tau_p, R, Rinv, state, step, min_diag, chol_lds);
}

// Cholesky G = R^T R and X = R^-1 for G = I + E near the identity (the second pass of
// CholQR2, where E is of the order of the first pass's loss of orthogonality). With
// U1 = up(E) and U = U1 + up(-U1^T U1), up(S) = strict upper part of S plus half its
// diagonal, R = I + U is upper triangular and R^T R = G + O(|E|^3); X = I - U + U^2
// has X R = I + O(|E|^3). Used when max |E_ij| <= thresh (a bound that keeps |E|^3
// below the rounding of the working precision); otherwise, and for a non-finite E, the
// blocked factorisation above runs. The two products are on FP64 MFMA, U in LDS.
template <int NB>
__global__ __launch_bounds__(256) void k_chol_inv_near_id(const double* __restrict__ G, int b, int ld,
                                                          double thresh, double* __restrict__ R,
                                                          double* __restrict__ Rinv, int* state, int step,
                                                          double* __restrict__ min_diag) {
    constexpr int N = 16 * NB, W = N + 1, NT = NB * (NB + 1) / 2, TPW = (NT + 3) / 4;
    extern __shared__ double chol_lds[];
    double* M = chol_lds;                 // N x W: U1, then U
    __shared__ double red[256];
    if (state[0]) return;
    typedef MF<double> Mf;
    const int t = threadIdx.x, l = t & 63, wv = t >> 6, lr = l >> 4, lc = l & 15;
    // U1 = up(E) over the upper triangle (zero beyond b) and max |E|; every load is
    // issued before the first use
    constexpr int PER = (N * N + 255) / 256;
    double g[PER];
#pragma unroll
    for (int q = 0; q < PER; ++q) {
        const int e = t + 256 * q;
        const int i = e / N, j = e % N;
        g[q] = (e < N * N && i < b && j < b && j >= i) ? G[(int64_t)i * ld + j] : 0.0;
    }
    double emax = 0.0;
#pragma unroll
    for (int q = 0; q < PER; ++q) {
        const int e = t + 256 * q;
        const int i = e / N, j = e % N;
        if (e >= N * N) continue;
        double u = 0.0;
        if (i < b && j < b && j >= i) {
            const double ev = g[q] - (i == j ? 1.0 : 0.0);
            const double a = fabs(ev);
            if (!(a <= emax)) emax = (emax != emax) ? emax : a;
            u = i == j ? 0.5 * ev : ev;
        }
        M[i * W + j] = u;
    }
    // max over the work-group: within each wave by shuffles, then the four wave maxima
    for (int off = 32; off > 0; off >>= 1) {
        const double o = __shfl_xor(emax, off);
        if (!(o <= emax) && emax == emax) emax = o;
    }
    if (l == 0) red[wv] = emax;
    __syncthreads();
    double gmax = red[0];
    for (int w2 = 1; w2 < 4; ++w2) {
        const double o = red[w2];
        if (!(o <= gmax) && gmax == gmax) gmax = o;
    }
    if (!(gmax <= thresh)) {              // uniform: every thread reads the same values
        __syncthreads();
        chol_inv_blk<NB>(G, b, ld, nullptr, R, Rinv, state, step, min_diag, chol_lds);
        return;
    }
    // upper tiles (ib <= jb) dealt to the waves: tile q of wave wv is number wv + 4 q
    int tib[TPW], tjb[TPW];
#pragma unroll
    for (int q = 0; q < TPW; ++q) {
        int n = wv + 4 * q < NT ? wv + 4 * q : NT - 1;          // past the end: not used
        int ib = 0;
        while (n >= NB - ib) { n -= NB - ib; ++ib; }
        tib[q] = ib;
        tjb[q] = ib + n;
    }
    // P = U1^T U1 on the upper tiles, kept in registers across the barrier. A wave's
    // tiles are independent chains, interleaved over the whole K range so that the LDS
    // reads of a step are in flight together (terms outside a tile's nonzero range are
    // zeros of the triangular factor).
    Mf::acc pt[TPW];
#pragma unroll
    for (int q = 0; q < TPW; ++q) pt[q] = Mf::zero();
    for (int k4 = 0; k4 < N; k4 += 4)
#pragma unroll
        for (int q = 0; q < TPW; ++q)
            pt[q] = Mf::mma(M[(k4 + lr) * W + 16 * tib[q] + lc], M[(k4 + lr) * W + 16 * tjb[q] + lc], pt[q]);
    __syncthreads();
    // U = U1 + up(-P) in place
#pragma unroll
    for (int q = 0; q < TPW; ++q) {
        if (wv + 4 * q >= NT) continue;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int i = 16 * tib[q] + lr + 4 * r, j = 16 * tjb[q] + lc;
            if (j > i) M[i * W + j] -= pt[q][r];
            else if (j == i) M[i * W + j] -= 0.5 * pt[q][r];
        }
    }
    __syncthreads();
    // U U on the same tiles, interleaved as above (U[i][k] = 0 for k < i, U[k][j] = 0 for k > j)
#pragma unroll
    for (int q = 0; q < TPW; ++q) pt[q] = Mf::zero();
    for (int k4 = 0; k4 < N; k4 += 4)
#pragma unroll
        for (int q = 0; q < TPW; ++q)
            pt[q] = Mf::mma(M[(16 * tib[q] + lc) * W + k4 + lr], M[(k4 + lr) * W + 16 * tjb[q] + lc], pt[q]);
    // R = I + U and X = I - U + U U: the upper tiles from the registers, everything else
    // zero (ld == N); two adjacent entries per store
#pragma unroll 2
    for (int e = 2 * t; e < N * N; e += 512) {
        const int i = e / N, j = e % N;                   // j even, j + 1 in the same row
        double2 rv, xv;
        rv.x = (i < b && j < b && j >= i) ? (i == j ? 1.0 : 0.0) + M[i * W + j] : 0.0;
        rv.y = (i < b && j + 1 < b && j + 1 >= i) ? (i == j + 1 ? 1.0 : 0.0) + M[i * W + j + 1] : 0.0;
        *reinterpret_cast<double2*>(R + e) = rv;
        // X entries outside the upper tiles (the strict lower block triangle and
        // rows/columns beyond b inside the tiles are written by the tile owners)
        if ((i >> 4) > (j >> 4)) {
            xv.x = 0.0;
            xv.y = 0.0;
            *reinterpret_cast<double2*>(Rinv + e) = xv;
        }
    }
#pragma unroll
    for (int q = 0; q < TPW; ++q) {
        if (wv + 4 * q >= NT) continue;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int i = 16 * tib[q] + lr + 4 * r, j = 16 * tjb[q] + lc;
            const bool in = i < b && j < b && j >= i;
            Rinv[i * N + j] = in ? (i == j ? 1.0 : 0.0) - M[i * W + j] + pt[q][r] : 0.0;
        }
    }
    if (wv == 0) {
        double d = INFINITY;
        for (int i = l; i < b; i += 64) d = fmin(d, 1.0 + M[i * W + i]);
        for (int off = 32; off > 0; off >>= 1) d = fmin(d, __shfl_xor(d, off));
        if (l == 0) min_diag[step] = d;
    }
}

// General-size fallback (global-memory working set).
__global__ __launch_bounds__(256) void k_chol_inv(const double* __restrict__ G, int b, int ld,
                                                  const double* __restrict__ tau_p,
                                                  double* __restrict__ R, double* __restrict__ Rinv,
                                                  double* gscratch, int* state, int step,
                                                  double* __restrict__ min_diag, int use_lds) {
    extern __shared__ double smem[];
    __shared__ int fail;
    __shared__ double dmin;
    if (state[0]) return;
    const double tau = tau_p ? *tau_p : 0.0;
    double* Mx = use_lds ? smem : gscratch;
    const int st = b + 1;
    double* dinv = Mx + (int64_t)b * st;
    const int tid = threadIdx.x, nth = blockDim.x;
    for (int idx = tid; idx < b * b; idx += nth) {
        const int i = idx / b, j = idx % b;
        Mx[i * st + j] = (j >= i) ? G[(int64_t)i * ld + j] : 0.0;
    }
    if (tid == 0) { fail = 0; dmin = INFINITY; }
    __syncthreads();
    for (int k = 0; k < b; ++k) {
        if (tid == 0) {
            const double piv = Mx[k * st + k];
            if (!(piv > 0.0) || !isfinite(piv)) {
                fail = 1;
            } else {
                const double d = sqrt(piv);
                Mx[k * st + k] = d;
                dmin = fmin(dmin, d);
                if (!(d > tau)) fail = 1;
            }
        }
        __syncthreads();
        if (fail) break;
        const double d = Mx[k * st + k];
        for (int j = k + 1 + tid; j < b; j += nth) Mx[k * st + j] /= d;
        __syncthreads();
        const int m = b - k - 1;
        for (int idx = tid; idx < m * m; idx += nth) {
            const int i = k + 1 + idx / m, j = k + 1 + idx % m;
            if (j >= i) Mx[i * st + j] -= Mx[k * st + i] * Mx[k * st + j];
        }
        __syncthreads();
    }
    if (tid == 0) min_diag[step] = dmin;
    if (fail) {
        for (int idx = tid; idx < ld * ld; idx += nth) { Rinv[idx] = 0.0; R[idx] = 0.0; }
        __syncthreads();
        if (tid == 0) { state[2] = step; state[0] = 1; }
        return;
    }
    // R^-1 by back substitution, row i from the bottom; X[i][j] (j > i) kept at Mx[j][i]
    for (int i = b - 1; i >= 0; --i) {
        if (tid == 0) dinv[i] = 1.0 / Mx[i * st + i];
        __syncthreads();
        const double di = dinv[i];
        for (int j = i + 1 + tid; j < b; j += nth) {
            double s = 0.0;
            for (int k = i + 1; k < j; ++k) s += Mx[i * st + k] * Mx[j * st + k];
            s += Mx[i * st + j] * dinv[j];
            Mx[j * st + i] = -s * di;
        }
        __syncthreads();
    }
    for (int idx = tid; idx < ld * ld; idx += nth) {
        const int i = idx / ld, j = idx % ld;
        double r = 0.0, x = 0.0;
        if (i < b && j < b && j >= i) {
            r = Mx[i * st + j];
            x = (j == i) ? dinv[i] : Mx[j * st + i];
        }
        R[idx] = r;
        Rinv[idx] = x;
    }
}

// R = R2 R1 for upper triangular ld x ld R1, R2 (zero below the diagonal), ld = 16 NB,
// on FP64 MFMA: workgroup ib, wave jb forms tile (ib, jb) from k in [16 ib, 16 jb + 16),
// the only k where R2[i][k] R1[k][j] can be nonzero; tiles below the diagonal are zero.
// All operands of a wave are loaded before its first MFMA.
template <int NB>
__global__ __launch_bounds__(64 * NB) void k_trmm_upper_mfma(const double* __restrict__ R2,
                                                             const double* __restrict__ R1, double* __restrict__ R,
                                                             const int* __restrict__ state) {
    if (state && state[0]) return;
    constexpr int ld = 16 * NB, MAXS = 4 * NB;
    typedef MF<double> M;
    const int ib = blockIdx.x, jb = threadIdx.x >> 6, l = threadIdx.x & 63, lr = l >> 4, lc = l & 15;
    typename M::acc c = M::zero();
    if (jb >= ib) {
        const int nst = 4 * (jb - ib + 1);
        double a[MAXS], bv[MAXS];
#pragma unroll
        for (int s4 = 0; s4 < MAXS; ++s4) {
            const int k = 16 * ib + 4 * s4 + lr;
            a[s4] = s4 < nst ? R2[(16 * ib + lc) * ld + k] : 0.0;
            bv[s4] = s4 < nst ? R1[k * ld + 16 * jb + lc] : 0.0;
        }
#pragma unroll
        for (int s4 = 0; s4 < MAXS; ++s4)
            if (s4 < nst) c = M::mma(a[s4], bv[s4], c);
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) R[(16 * ib + M::row(l, r)) * ld + 16 * jb + lc] = c[r];
}

__global__ void k_trmm_upper(const double* __restrict__ R2, const double* __restrict__ R1, double* __restrict__ R,
                             int ld, const int* __restrict__ state) {
    if (state && state[0]) return;
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= ld * ld) return;
    const int i = idx / ld, j = idx % ld;
    double s = 0.0;
    for (int k = i; k <= j; ++k) s += R2[i * ld + k] * R1[k * ld + j];
    R[idx] = (j >= i) ? s : 0.0;
}


__global__ void k_copy_small(const double* __restrict__ M, int ld, int b, double* __restrict__ out) {
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= b * b) return;
    out[idx] = M[(idx / b) * ld + idx % b];
}

// ------------------------------------------------------------------ generic FP64 GEMM

__global__ __launch_bounds__(64) void k_gemm_f64(int Mr, int Nc, int K, const double* __restrict__ A, int64_t a_rs,
                                                 int64_t a_cs, const double* __restrict__ B, int64_t b_rs,
                                                 int64_t b_cs, double* __restrict__ C, int64_t c_rs, int64_t c_cs) {
    typedef MF<double> M;
    const int l = threadIdx.x, lr = l >> 4, lc = l & 15;
    const int i0 = blockIdx.x * 32, j0 = blockIdx.y * 32;
    M::acc c00 = M::zero(), c01 = M::zero(), c10 = M::zero(), c11 = M::zero();
    const int ia = i0 + lc, ib = ia + 16, ja = j0 + lc, jb = ja + 16;
    for (int k0 = 0; k0 < K; k0 += 4) {
        const int k = k0 + lr;
        const bool kv = k < K;
        const double a0 = (kv && ia < Mr) ? A[ia * a_rs + k * a_cs] : 0.0;
        const double a1 = (kv && ib < Mr) ? A[ib * a_rs + k * a_cs] : 0.0;
        const double b0 = (kv && ja < Nc) ? B[k * b_rs + ja * b_cs] : 0.0;
        const double b1 = (kv && jb < Nc) ? B[k * b_rs + jb * b_cs] : 0.0;
        c00 = M::mma(a0, b0, c00);
        c01 = M::mma(a0, b1, c01);
        c10 = M::mma(a1, b0, c10);
        c11 = M::mma(a1, b1, c11);
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int ra = i0 + M::row(l, r), rb = ra + 16;
        if (ra < Mr && ja < Nc) C[ra * c_rs + ja * c_cs] = c00[r];
        if (ra < Mr && jb < Nc) C[ra * c_rs + jb * c_cs] = c01[r];
        if (rb < Mr && ja < Nc) C[rb * c_rs + ja * c_cs] = c10[r];
        if (rb < Mr && jb < Nc) C[rb * c_rs + jb * c_cs] = c11[r];
    }
}

int max_lds_bytes() {
    static std::atomic<int> cached{-1};        // same value from any thread
    int c = cached.load(std::memory_order_relaxed);
    if (c < 0) {
        int dev = 0, v = 65536;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess)
            v = 65536;
        cached.store(v, std::memory_order_relaxed);
        c = v;
    }
    return c;
}

}  // namespace

// ------------------------------------------------------------------ launchers

int64_t gram_partial_mats(int ld) {
    int64_t m = (int64_t(1) << 26) / ((int64_t)ld * ld);
    return std::min<int64_t>(1024, std::max<int64_t>(64, m));
}

namespace {
// Gram layout: FP32 with ld <= 96 -> one wave per 96-wide tile (TW = 6, WPG = 1:
// 36 accumulators of 4 floats); FP64 with ld <= 96 -> 2 x 2 waves of TW = 3;
// ld > 96 -> 2 x 2 waves of TW = 4 (128-wide tiles).
// Wave tiles: FP32 with ld <= 96 -> one wave per ld x ld tile (TW = ld/16, up to
// 36 accumulators of 4 floats); otherwise 2 x 2 waves of TW = 3 (FP64, ld <= 96)
// or TW = 4 (ld > 96).
int gram_tw(int ld, int elem) { return (ld <= 96 && elem == 4) ? ld / 16 : (ld <= 96 ? 3 : 4); }
int gram_wpg(int ld, int elem) { return (ld <= 96 && elem == 4) ? 1 : 4; }
int gram_tile(int ld, int elem) { return (gram_wpg(ld, elem) == 1 ? 16 : 32) * gram_tw(ld, elem); }
int gram_ks(int ld, int elem) { return gram_wpg(ld, elem) == 1 ? 4 : 2; }
}

// FP32 Grams: a wave adds at most this many rows in FP32 before its partial is
// summed in FP64 (rounding of an FP32 running sum grows with its length).
constexpr int64_t kGramFp32Rows = 512;

int64_t gram_min_chunks(int64_t Np, int ld, int elem) {
    if (elem != 4) return 1;
    const int64_t rows = (int64_t)gram_ks(ld, elem) * kGramFp32Rows;     // rows of one chunk
    return (Np + rows - 1) / rows;
}

GramPlan gram_plan(int64_t Np, int ld, int nprod, bool sym, int64_t cap_mats, int elem) {
    GramPlan g;
    g.ld = ld;
    g.nprod = nprod;
    g.Np = Np;
    g.sym = sym;
    const int tile = gram_tile(ld, elem);
    const int ntw = (ld + tile - 1) / tile;
    g.ntiles = ntw * ntw;
    // about 1024 waves in flight; a workgroup holds WPG*KS waves
    const int ks = gram_ks(ld, elem);
    const int64_t target_wg =
        std::max<int64_t>(16, 1024 / (gram_wpg(ld, elem) * ks * std::max(1, g.ntiles)));
    int64_t nchunk = (target_wg + nprod - 1) / nprod;
    nchunk = std::min<int64_t>(nchunk, std::max<int64_t>(1, Np / 256));
    nchunk = std::max<int64_t>(nchunk, gram_min_chunks(Np, ld, elem));
    nchunk = std::min<int64_t>(nchunk, std::max<int64_t>(1, cap_mats / std::max(1, nprod)));
    int64_t rpc = (Np + nchunk - 1) / nchunk;
    rpc = (rpc + 127) / 128 * 128;                // whole prefetch rounds per chunk (Np is a multiple of 256)
    g.rows_per_chunk = rpc;
    g.nchunk = static_cast<int>((Np + rpc - 1) / rpc);
    return g;
}

template <typename T, int TW, int WPG, bool RUN>
void gram_tw_launch(const GramPlan& g, const T* X, int64_t xstride, const T* Y, T* part, int ntw, const int* state,
                    hipStream_t s) {
    constexpr int TILE = (WPG == 1 ? 16 : 32) * TW;
    constexpr int KS = WPG == 1 ? 4 : 2;
    dim3 grid(g.nchunk, g.ntiles, g.nprod);
    const size_t lds = (size_t)TILE * TILE * sizeof(T);
    k_gram<T, T, TW, KS, WPG, RUN><<<grid, 64 * WPG * KS, lds, s>>>(X, xstride, Y, g.Np, g.rows_per_chunk, g.ld,
                                                                     ntw, g.sym ? 1 : 0, part, g.nchunk, state);
}

template <typename T>
void gram_launch(const GramPlan& g, const T* X, int64_t xstride, const T* Y, double* partial, double* out,
                 int64_t out_stride, int mode, const int* state, hipStream_t s, const GramExtra& ex) {
    const int elem = (int)sizeof(T);
    const int tile = gram_tile(g.ld, elem);
    const int ntw = (g.ld + tile - 1) / tile;
    T* part = reinterpret_cast<T*>(partial);      // partials in the block precision
    if constexpr (sizeof(T) == 4) {
        if (g.ld <= 96) {
            switch (g.ld / 16) {
                case 1: gram_tw_launch<T, 1, 1, true>(g, X, xstride, Y, part, ntw, state, s); break;
                case 2: gram_tw_launch<T, 2, 1, true>(g, X, xstride, Y, part, ntw, state, s); break;
                case 3: gram_tw_launch<T, 3, 1, true>(g, X, xstride, Y, part, ntw, state, s); break;
                case 4: gram_tw_launch<T, 4, 1, true>(g, X, xstride, Y, part, ntw, state, s); break;
                case 5: gram_tw_launch<T, 5, 1, true>(g, X, xstride, Y, part, ntw, state, s); break;
                default: gram_tw_launch<T, 6, 1, true>(g, X, xstride, Y, part, ntw, state, s); break;
            }
        } else if (g.ld % 64 == 0) {
            gram_tw_launch<T, 4, 4, true>(g, X, xstride, Y, part, ntw, state, s);
        } else {
            gram_tw_launch<T, 4, 4, false>(g, X, xstride, Y, part, ntw, state, s);
        }
    } else if (g.ld <= 96) {
        if (g.ld % 48 == 0)
            gram_tw_launch<T, 3, 4, true>(g, X, xstride, Y, part, ntw, state, s);
        else
            gram_tw_launch<T, 3, 4, false>(g, X, xstride, Y, part, ntw, state, s);
    } else if (g.ld % 64 == 0) {
        gram_tw_launch<T, 4, 4, true>(g, X, xstride, Y, part, ntw, state, s);
    } else {
        gram_tw_launch<T, 4, 4, false>(g, X, xstride, Y, part, ntw, state, s);
    }
    dim3 rgrid(reduce_blocks(g.ld, mode != 0 || ex.sym_p >= 0), g.nprod);
    k_gram_reduce<T><<<rgrid, 64 * kRedGroups, 0, s>>>(part, g.nchunk, g.ld, g.sym ? 1 : 0, mode, out, out_stride,
                                                        state, ex.copy, ex.sym_to, ex.sym_p);
}

template <typename T, int NTW>
void update_one(T* OUT, const T* IN, double alpha, const T* X, int64_t xstride, int nprod, const T* S, int64_t Np,
                int ld, const int* state, hipStream_t s) {
    constexpr int MT = sizeof(T) == 4 ? 2 : 1;   // FP64: one row tile per wave keeps two waves per SIMD
    const int64_t rows_per_block = 4 * 16 * MT;
    dim3 grid(static_cast<unsigned>((Np + rows_per_block - 1) / rows_per_block), (ld + 16 * NTW - 1) / (16 * NTW));
    k_update<T, MT, NTW><<<grid, 256, 0, s>>>(OUT, IN, alpha, X, xstride, nprod, S, Np, ld, state);
}

template <typename T>
static void update_staged(T* OUT, const T* IN, double alpha, const T* X, int64_t xstride, int nprod, const T* st,
                          int64_t Np, int ld, const int* state, hipStream_t s);

static bool split_full_ok(int ld);
template <int NPL>
static void frag_launch(const double* S, int64_t sstride, int nprod, int ld, bool trans, double scale, void* stage,
                        hipStream_t s, const double* S1 = nullptr, bool trans1 = false);
template <int NPL>
static void update_split_any(float* OUT, const float* IN, double alpha, const float* X, int64_t xstride, int nprod,
                             const void* frag, int64_t Np, int ld, const int* state, hipStream_t s,
                             unsigned short* OUT16 = nullptr);

template <typename T>
void update_launch(T* OUT, const T* IN, double alpha, const T* X, int64_t xstride, int nprod, const double* S,
                   int64_t sstride, bool trans, double scale, int64_t Np, int ld, void* stage, const int* state,
                   hipStream_t s, void* out16) {
    if constexpr (std::is_same<T, float>::value) {
        if (split_full_ok(ld)) {
            frag_launch<3>(S, sstride, nprod, ld, trans, scale, stage, s);
            update_split_any<3>(OUT, IN, alpha, X, xstride, nprod, stage, Np, ld, state, s,
                                static_cast<unsigned short*>(out16));
            return;
        }
    }
    T* st = static_cast<T*>(stage);
    const int64_t cnt = (int64_t)nprod * ld * ld;
    k_stage_s<T><<<grid_for(cnt, 256), 256, 0, s>>>(S, sstride, nprod, ld, trans ? 1 : 0, scale, st);
    update_staged<T>(OUT, IN, alpha, X, xstride, nprod, st, Np, ld, state, s);
    if constexpr (std::is_same<T, float>::value) {
        if (out16) bf16_copy_launch(OUT, out16, Np * ld, s);
    }
}

template <typename T>
void update2_launch(T* OUT, const T* IN, double alpha, const T* X0, const double* S0, bool trans0, const T* X1,
                    const double* S1, bool trans1, double scale, int64_t Np, int ld, void* stage, const int* state,
                    hipStream_t s) {
    if constexpr (std::is_same<T, float>::value) {
        if (split_full_ok(ld)) {
            frag_launch<3>(S0, 0, 2, ld, trans0, scale, stage, s, S1, trans1);
            update_split_any<3>(OUT, IN, alpha, X0, X1 - X0, 2, stage, Np, ld, state, s);
            return;
        }
    }
    T* st = static_cast<T*>(stage);
    const int64_t mat = (int64_t)ld * ld;
    k_stage_s<T><<<grid_for(mat, 256), 256, 0, s>>>(S0, 0, 1, ld, trans0 ? 1 : 0, scale, st);
    k_stage_s<T><<<grid_for(mat, 256), 256, 0, s>>>(S1, 0, 1, ld, trans1 ? 1 : 0, scale, st + mat);
    update_staged<T>(OUT, IN, alpha, X0, X1 - X0, 2, st, Np, ld, state, s);
}

template <typename T>
static void update_staged(T* OUT, const T* IN, double alpha, const T* X, int64_t xstride, int nprod, const T* st,
                          int64_t Np, int ld, const int* state, hipStream_t s) {
    const int nt = ld / 16;
    // fewer than ~4 row workgroups per CU: split the columns in two blocks for parallelism
    const bool few = Np / (sizeof(T) == 4 ? 128 : 64) < 1024;
    if (nt <= 2)
        update_one<T, 2>(OUT, IN, alpha, X, xstride, nprod, st, Np, ld, state, s);
    else if (nt <= 4)
        update_one<T, 4>(OUT, IN, alpha, X, xstride, nprod, st, Np, ld, state, s);
    else if (nt <= 6 && few)
        update_one<T, 3>(OUT, IN, alpha, X, xstride, nprod, st, Np, ld, state, s);
    else if (nt <= 6)
        update_one<T, 6>(OUT, IN, alpha, X, xstride, nprod, st, Np, ld, state, s);
    else
        update_one<T, 8>(OUT, IN, alpha, X, xstride, nprod, st, Np, ld, state, s);
}

template <int NT, int NPL>
static void update_split_one(float* OUT, const float* IN, double alpha, const float* X, int64_t xstride, int nprod,
                             const void* frag, int64_t Np, int ld, const int* state, hipStream_t s,
                             unsigned short* OUT16) {
    constexpr int D = 4;
    // rows per work-group: 128 (MT = 2) by default, 64 (MT = 1) by the tuning
    if (tuning().update_rows == 64) {
        const unsigned grid = static_cast<unsigned>((Np + 63) / 64);
        k_update_split<1, NT, D, NPL><<<grid, 256, 0, s>>>(OUT, IN, alpha, X, xstride, nprod,
                                                            static_cast<const bf16x8*>(frag), Np, ld, state, OUT16);
    } else {
        const unsigned grid = static_cast<unsigned>((Np + 127) / 128);
        k_update_split<2, NT, D, NPL><<<grid, 256, 0, s>>>(OUT, IN, alpha, X, xstride, nprod,
                                                            static_cast<const bf16x8*>(frag), Np, ld, state, OUT16);
    }
}

template <int NPL>
static void update_split_any(float* OUT, const float* IN, double alpha, const float* X, int64_t xstride, int nprod,
                             const void* frag, int64_t Np, int ld, const int* state, hipStream_t s,
                             unsigned short* OUT16) {
    switch (ld / 16) {
        case 1: update_split_one<1, NPL>(OUT, IN, alpha, X, xstride, nprod, frag, Np, ld, state, s, OUT16); break;
        case 2: update_split_one<2, NPL>(OUT, IN, alpha, X, xstride, nprod, frag, Np, ld, state, s, OUT16); break;
        case 3: update_split_one<3, NPL>(OUT, IN, alpha, X, xstride, nprod, frag, Np, ld, state, s, OUT16); break;
        case 4: update_split_one<4, NPL>(OUT, IN, alpha, X, xstride, nprod, frag, Np, ld, state, s, OUT16); break;
        case 5: update_split_one<5, NPL>(OUT, IN, alpha, X, xstride, nprod, frag, Np, ld, state, s, OUT16); break;
        case 6: update_split_one<6, NPL>(OUT, IN, alpha, X, xstride, nprod, frag, Np, ld, state, s, OUT16); break;
        case 7: update_split_one<7, NPL>(OUT, IN, alpha, X, xstride, nprod, frag, Np, ld, state, s, OUT16); break;
        default: update_split_one<8, NPL>(OUT, IN, alpha, X, xstride, nprod, frag, Np, ld, state, s, OUT16); break;
    }
}

template <int NT>
static void update_bf16x_one(float* OUT, const float* IN, double alpha, const unsigned short* X, int64_t xstride,
                             int nprod, const void* frag, int64_t Np, int ld, const int* state, hipStream_t s) {
    constexpr int D = 4;
    if (tuning().update_rows == 64) {
        const unsigned grid = static_cast<unsigned>((Np + 63) / 64);
        k_update_bf16x<1, NT, D><<<grid, 256, 0, s>>>(OUT, IN, alpha, X, xstride, nprod,
                                                       static_cast<const bf16x8*>(frag), Np, ld, state);
    } else {
        const unsigned grid = static_cast<unsigned>((Np + 127) / 128);
        k_update_bf16x<2, NT, D><<<grid, 256, 0, s>>>(OUT, IN, alpha, X, xstride, nprod,
                                                       static_cast<const bf16x8*>(frag), Np, ld, state);
    }
}

// Fragments of scale * op(S_p), p < nprod (S_p = S1 and op1 for p = 1 when S1 is set).
template <int NPL>
static void frag_launch(const double* S, int64_t sstride, int nprod, int ld, bool trans, double scale, void* stage,
                        hipStream_t s, const double* S1, bool trans1) {
    const int nt = ld / 16, nkc = (ld + kSplitK - 1) / kSplitK;
    const int64_t cnt = ((int64_t)nprod * nkc + 1) * nt * 64;
    k_frag_s<NPL><<<grid_for(cnt, 256), 256, 0, s>>>(S, sstride, nprod, ld, trans ? 1 : 0, scale, S1, trans1 ? 1 : 0,
                                                     static_cast<bf16x8*>(stage));
}

// Full-accuracy FP32 block updates on split BF16 (three parts, six products) when
// ld = 16 NT with 3 <= NT <= 8: the fragments of nprod coefficient blocks, plus the
// zero chunk, then fit the staging area of nprod + 1 ld x ld FP64 matrices.
static bool split_full_ok(int ld) { return ld % 16 == 0 && ld / 16 >= 3 && ld / 16 <= 8; }

void bf16_copy_launch(const float* in, void* out, int64_t n, hipStream_t s) {
    k_to_bf16<<<grid_for(n, 256), 256, 0, s>>>(in, static_cast<unsigned short*>(out), n);
}

bool update_correction_bf16_launch(float* OUT, const float* IN, double alpha, const void* X16, int64_t xstride,
                                   int nprod, const double* S, int64_t sstride, bool trans, double scale, int64_t Np,
                                   int ld, void* stage, const int* state, hipStream_t s) {
    if (ld % 16 != 0 || ld / 16 < 1 || ld / 16 > 8) return false;
    frag_launch<1>(S, sstride, nprod, ld, trans, scale, stage, s);
    const unsigned short* X = static_cast<const unsigned short*>(X16);
    switch (ld / 16) {
        case 1: update_bf16x_one<1>(OUT, IN, alpha, X, xstride, nprod, stage, Np, ld, state, s); break;
        case 2: update_bf16x_one<2>(OUT, IN, alpha, X, xstride, nprod, stage, Np, ld, state, s); break;
        case 3: update_bf16x_one<3>(OUT, IN, alpha, X, xstride, nprod, stage, Np, ld, state, s); break;
        case 4: update_bf16x_one<4>(OUT, IN, alpha, X, xstride, nprod, stage, Np, ld, state, s); break;
        case 5: update_bf16x_one<5>(OUT, IN, alpha, X, xstride, nprod, stage, Np, ld, state, s); break;
        case 6: update_bf16x_one<6>(OUT, IN, alpha, X, xstride, nprod, stage, Np, ld, state, s); break;
        case 7: update_bf16x_one<7>(OUT, IN, alpha, X, xstride, nprod, stage, Np, ld, state, s); break;
        default: update_bf16x_one<8>(OUT, IN, alpha, X, xstride, nprod, stage, Np, ld, state, s); break;
    }
    return true;
}

template <>
void update_correction_launch<float>(float* OUT, const float* IN, double alpha, const float* X, int64_t xstride,
                                     int nprod, const double* S, int64_t sstride, bool trans, double scale,
                                     int64_t Np, int ld, void* stage, const int* state, hipStream_t s) {
    const int nt = ld / 16;
    if (ld % 16 != 0 || nt > 8) {
        update_launch<float>(OUT, IN, alpha, X, xstride, nprod, S, sstride, trans, scale, Np, ld, stage, state, s);
        return;
    }
    frag_launch<2>(S, sstride, nprod, ld, trans, scale, stage, s);
    update_split_any<2>(OUT, IN, alpha, X, xstride, nprod, stage, Np, ld, state, s);
}

template <>
void update_correction_launch<double>(double* OUT, const double* IN, double alpha, const double* X, int64_t xstride,
                                      int nprod, const double* S, int64_t sstride, bool trans, double scale,
                                      int64_t Np, int ld, void* stage, const int* state, hipStream_t s) {
    update_launch<double>(OUT, IN, alpha, X, xstride, nprod, S, sstride, trans, scale, Np, ld, stage, state, s);
}

// Column parts and row groups of k_gram_split for ld (two column parts, hence two
// row groups, for the widest blocks).
static int gram_split_parts(int ld) { return (ld / 16) % 2 == 0 && ld / 16 >= 4 ? 2 : 1; }
static int gram_split_groups(int ld) { return 4 / gram_split_parts(ld); }

// Plan for k_gram_split: chunks of a multiple of 256 rows (an even number of steps
// per wave), at most kGramFp32Rows rows per wave.
GramPlan gram_plan_split(int64_t Np, int ld, int nprod, int64_t cap_mats) {
    GramPlan g;
    g.ld = ld;
    g.nprod = nprod;
    g.Np = Np;
    g.sym = false;
    g.ntiles = 1;
    const int per_cu = std::max(1, tuning().gram_chunks);
    int64_t nchunk = (256 * per_cu + nprod - 1) / nprod;  // about per_cu workgroups per compute unit
    nchunk = std::min<int64_t>(nchunk, std::max<int64_t>(1, Np / 256));
    const int kg = gram_split_groups(ld);
    nchunk = std::max<int64_t>(nchunk, (Np + kg * kGramFp32Rows - 1) / (kg * kGramFp32Rows));
    nchunk = std::min<int64_t>(nchunk, std::max<int64_t>(1, cap_mats / std::max(1, nprod)));
    int64_t rpc = (Np + nchunk - 1) / nchunk;
    rpc = (rpc + 255) / 256 * 256;                // Np is a multiple of 256
    g.rows_per_chunk = rpc;
    g.nchunk = static_cast<int>((Np + rpc - 1) / rpc);
    return g;
}

template <int NT>
static void gram_split_one(const GramPlan& g, const float* X, int64_t xstride, const float* Y, const bf16x8* Yp,
                           const double* hinf, float* part, const int* state, hipStream_t s) {
    constexpr int NH = (NT % 2 == 0 && NT >= 4) ? 2 : 1;
    const unsigned grid = static_cast<unsigned>(8 * ((g.nchunk + 7) / 8) * g.nprod);   // see k_gram_split
    const size_t lds = sizeof(float) * 256 * NT * NT;
    if (Yp && hinf)
        k_gram_split<NT, NH, 2, true, true><<<grid, 256, lds, s>>>(X, xstride, Y, Yp, g.Np, g.rows_per_chunk, g.ld,
                                                                   part, g.nchunk, state, hinf);
    else if (Yp)
        k_gram_split<NT, NH, 3, true, false><<<grid, 256, lds, s>>>(X, xstride, Y, Yp, g.Np, g.rows_per_chunk, g.ld,
                                                                    part, g.nchunk, state, hinf);
    else
        k_gram_split<NT, NH, 3, false, false><<<grid, 256, lds, s>>>(X, xstride, Y, Yp, g.Np, g.rows_per_chunk, g.ld,
                                                                     part, g.nchunk, state, hinf);
}

template <>
void gram_blocks_launch<float>(const float* X, int64_t xstride, int nprod, const float* Y, int64_t Np, int ld, bool sym,
                               int64_t cap_mats, double* partial, double* out, int64_t out_stride, int mode,
                               const int* state, hipStream_t s, void* yplanes, const double* hinf,
                               const GramExtra& ex) {
    if (ld % 16 != 0 || ld > 96 || Np % 256 != 0) {
        const GramPlan g = gram_plan(Np, ld, nprod, sym, cap_mats, 4);
        gram_launch<float>(g, X, xstride, Y, partial, out, out_stride, mode, state, s, ex);
        return;
    }
    // the partials are FP32: the buffer (cap_mats FP64 matrices) holds twice as many
    const GramPlan g = gram_plan_split(Np, ld, nprod, 2 * cap_mats);
    float* part = reinterpret_cast<float*>(partial);
    // several products share Y: split it once into planes instead of once per product
    bf16x8* Yp = nullptr;
    if (yplanes && nprod > 1) {
        Yp = static_cast<bf16x8*>(yplanes);
        if (hinf)
            k_split_rows8<2, true><<<grid_for((Np / 8) * ld, 256), 256, 0, s>>>(Y, Np, ld, Yp, state, hinf);
        else
            k_split_rows8<3, false><<<grid_for((Np / 8) * ld, 256), 256, 0, s>>>(Y, Np, ld, Yp, state, hinf);
    } else {
        hinf = nullptr;
    }
    switch (ld / 16) {
        case 1: gram_split_one<1>(g, X, xstride, Y, Yp, hinf, part, state, s); break;
        case 2: gram_split_one<2>(g, X, xstride, Y, Yp, hinf, part, state, s); break;
        case 3: gram_split_one<3>(g, X, xstride, Y, Yp, hinf, part, state, s); break;
        case 4: gram_split_one<4>(g, X, xstride, Y, Yp, hinf, part, state, s); break;
        case 5: gram_split_one<5>(g, X, xstride, Y, Yp, hinf, part, state, s); break;
        default: gram_split_one<6>(g, X, xstride, Y, Yp, hinf, part, state, s); break;
    }
    dim3 rgrid(reduce_blocks(ld, mode != 0 || ex.sym_p >= 0), nprod);
    k_gram_reduce<float><<<rgrid, 64 * kRedGroups, 0, s>>>(part, g.nchunk, ld, 0, mode, out, out_stride, state,
                                                           ex.copy, ex.sym_to, ex.sym_p);
}

template <>
void gram_blocks_launch<double>(const double* X, int64_t xstride, int nprod, const double* Y, int64_t Np, int ld,
                                bool sym, int64_t cap_mats, double* partial, double* out, int64_t out_stride, int mode,
                                const int* state, hipStream_t s, void*, const double*, const GramExtra& ex) {
    const GramPlan g = gram_plan(Np, ld, nprod, sym, cap_mats, 8);
    gram_launch<double>(g, X, xstride, Y, partial, out, out_stride, mode, state, s, ex);
}

size_t chol_scratch_bytes(int b) { return sizeof(double) * ((size_t)b * (b + 1) + b + 8); }

void chol_inv_near_identity_launch(const double* G, int b, int ld, double thresh, double* R, double* Rinv,
                                   double* scratch, int* state, int step, double* min_diag, hipStream_t s) {
    if (b <= 128 && ld == 16 * ((b + 15) / 16)) {
        const int nb = (b + 15) / 16;
        const size_t lds = sizeof(double) * ((size_t)16 * nb * (16 * nb + 1) + 256 * (size_t)nb);
        switch (nb) {
#define CSS_CHOL(NB) case NB: k_chol_inv_near_id<NB><<<1, 256, lds, s>>>(G, b, ld, thresh, R, Rinv, state, step, \
                                                                         min_diag); return;
            CSS_CHOL(1) CSS_CHOL(2) CSS_CHOL(3) CSS_CHOL(4) CSS_CHOL(5) CSS_CHOL(6) CSS_CHOL(7) CSS_CHOL(8)
#undef CSS_CHOL
            default: break;
        }
    }
    chol_inv_launch(G, b, ld, nullptr, R, Rinv, scratch, state, step, min_diag, s);
}

void chol_inv_launch(const double* G, int b, int ld, const double* tau, double* R, double* Rinv, double* scratch,
                     int* state, int step, double* min_diag, hipStream_t s) {
    if (b <= 128 && ld == 16 * ((b + 15) / 16)) {
        const int nb = (b + 15) / 16;
        const size_t lds = sizeof(double) * ((size_t)16 * nb * (16 * nb + 1) + 256 * (size_t)nb);
        switch (nb) {
#define CSS_CHOL(NB) case NB: k_chol_inv_blk<NB><<<1, 256, lds, s>>>(G, b, ld, tau, R, Rinv, state, step, min_diag); return;
            CSS_CHOL(1) CSS_CHOL(2) CSS_CHOL(3) CSS_CHOL(4) CSS_CHOL(5) CSS_CHOL(6) CSS_CHOL(7) CSS_CHOL(8)
#undef CSS_CHOL
            default: break;
        }
    }
    const size_t bytes = chol_scratch_bytes(b);
    const bool lds = bytes + 64 <= (size_t)max_lds_bytes();
    k_chol_inv<<<1, 256, lds ? bytes : 0, s>>>(G, b, ld, tau, R, Rinv, scratch, state, step, min_diag, lds ? 1 : 0);
}

void trmm_upper_launch(const double* R2, const double* R1, double* R, int ld, const int* state, hipStream_t s) {
    if (ld % 16 == 0 && ld <= 128) {
        switch (ld / 16) {
#define CSS_TRMM(NB) case NB: k_trmm_upper_mfma<NB><<<NB, 64 * NB, 0, s>>>(R2, R1, R, state); return;
            CSS_TRMM(1) CSS_TRMM(2) CSS_TRMM(3) CSS_TRMM(4) CSS_TRMM(5) CSS_TRMM(6) CSS_TRMM(7) CSS_TRMM(8)
#undef CSS_TRMM
            default: break;
        }
    }
    k_trmm_upper<<<grid_for((int64_t)ld * ld, 256), 256, 0, s>>>(R2, R1, R, ld, state);
}

void copy_small_launch(const double* M, int ld, int b, double* out, hipStream_t s) {
    k_copy_small<<<grid_for((int64_t)b * b, 256), 256, 0, s>>>(M, ld, b, out);
}

void gemm_f64_launch(int M, int N, int K, const double* A, int64_t a_rs, int64_t a_cs, const double* B,
                     int64_t b_rs, int64_t b_cs, double* C, int64_t c_rs, int64_t c_cs, hipStream_t s) {
    dim3 grid((M + 31) / 32, (N + 31) / 32);
    k_gemm_f64<<<grid, 64, 0, s>>>(M, N, K, A, a_rs, a_cs, B, b_rs, b_cs, C, c_rs, c_cs);
}

template void gram_launch<double>(const GramPlan&, const double*, int64_t, const double*, double*, double*,
                                  int64_t, int, const int*, hipStream_t, const GramExtra&);
template void gram_launch<float>(const GramPlan&, const float*, int64_t, const float*, double*, double*, int64_t,
                                 int, const int*, hipStream_t, const GramExtra&);
template void update_launch<double>(double*, const double*, double, const double*, int64_t, int, const double*,
                                    int64_t, bool, double, int64_t, int, void*, const int*, hipStream_t, void*);
template void update_launch<float>(float*, const float*, double, const float*, int64_t, int, const double*,
                                   int64_t, bool, double, int64_t, int, void*, const int*, hipStream_t, void*);
template void update2_launch<double>(double*, const double*, double, const double*, const double*, bool,
                                     const double*, const double*, bool, double, int64_t, int, void*, const int*,
                                     hipStream_t);
template void update2_launch<float>(float*, const float*, double, const float*, const double*, bool, const float*,
                                    const double*, bool, double, int64_t, int, void*, const int*, hipStream_t);

}  // namespace css
