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
#include <cmath>

#include "css_common.h"
#include "dense.h"

namespace css {
namespace {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

template <typename T>
struct MF;
template <>
struct MF<double> {
    typedef d4 acc;
    __device__ static acc zero() { return acc{0.0, 0.0, 0.0, 0.0}; }
    __device__ static acc mma(double a, double b, acc c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    __device__ static int row(int l, int r) { return (l >> 4) + 4 * r; }
};
template <>
struct MF<float> {
    typedef f4 acc;
    __device__ static acc zero() { return acc{0.f, 0.f, 0.f, 0.f}; }
    __device__ static acc mma(float a, float b, acc c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    __device__ static int row(int l, int r) { return 4 * (l >> 4) + r; }
};

// ------------------------------------------------------------------ Gram

template <typename T>
__global__ __launch_bounds__(64) void k_gram(const T* __restrict__ X, int64_t xstride,
                                             const T* __restrict__ Y, int64_t Np, int64_t rpc, int ld,
                                             int tpd, int sym, double* __restrict__ partial, int nchunk,
                                             const int* __restrict__ state) {
    if (state && state[0]) return;
    typedef MF<T> M;
    const int l = threadIdx.x, lr = l >> 4, lc = l & 15;
    const int chunk = blockIdx.x, p = blockIdx.z;
    int ti, tj;
    if (sym) {
        int rem = blockIdx.y, cnt = tpd;
        ti = 0;
        while (rem >= cnt) { rem -= cnt; ++ti; --cnt; }
        tj = ti + rem;
    } else {
        ti = blockIdx.y / tpd;
        tj = blockIdx.y % tpd;
    }
    const int i0 = ti * 32, j0 = tj * 32;
    const bool vi1 = i0 + 16 < ld, vj1 = j0 + 16 < ld;
    typename M::acc c00 = M::zero(), c01 = M::zero(), c10 = M::zero(), c11 = M::zero();
    const int64_t r0 = (int64_t)chunk * rpc;
    const int64_t r1 = r0 + rpc < Np ? r0 + rpc : Np;
    const T* xa = X + (int64_t)p * xstride + (r0 + lr) * ld + i0 + lc;
    const T* ya = Y + (r0 + lr) * ld + j0 + lc;
    const int64_t step = 4 * (int64_t)ld;
#pragma unroll 4
    for (int64_t r = r0; r < r1; r += 4, xa += step, ya += step) {
        const T a0 = xa[0], b0 = ya[0];
        const T a1 = vi1 ? xa[16] : T(0);
        const T b1 = vj1 ? ya[16] : T(0);
        c00 = M::mma(a0, b0, c00);
        c01 = M::mma(a0, b1, c01);
        c10 = M::mma(a1, b0, c10);
        c11 = M::mma(a1, b1, c11);
    }
    double* out = partial + ((int64_t)p * nchunk + chunk) * ld * ld;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int ra = i0 + M::row(l, r), rb = ra + 16, ca = j0 + lc, cb = ca + 16;
        out[(int64_t)ra * ld + ca] = c00[r];
        if (vj1) out[(int64_t)ra * ld + cb] = c01[r];
        if (vi1) out[(int64_t)rb * ld + ca] = c10[r];
        if (vi1 && vj1) out[(int64_t)rb * ld + cb] = c11[r];
    }
}

__global__ void k_gram_reduce(const double* __restrict__ partial, int nchunk, int ld, int sym, int mode,
                              double* __restrict__ out, int64_t out_stride, const int* __restrict__ state) {
    if (state && state[0]) return;
    const int p = blockIdx.y;
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= ld * ld) return;
    const int i = idx / ld, j = idx % ld;
    const int64_t mat = (int64_t)ld * ld;
    const double* base = partial + (int64_t)p * nchunk * mat;
    const int64_t sij = (sym && (i >> 5) > (j >> 5)) ? (int64_t)j * ld + i : (int64_t)i * ld + j;
    double s1 = 0.0;
    for (int c = 0; c < nchunk; ++c) s1 += base[c * mat + sij];
    double v = s1;
    if (mode != 0) {
        const int64_t sji = (sym && (j >> 5) > (i >> 5)) ? (int64_t)i * ld + j : (int64_t)j * ld + i;
        double s2 = 0.0;
        for (int c = 0; c < nchunk; ++c) s2 += base[c * mat + sji];
        v = 0.5 * (s1 + s2);
    }
    double* o = out + p * out_stride + idx;
    if (mode == 2)
        *o += v;
    else
        *o = v;
}

// ------------------------------------------------------------------ update

template <typename T, int MT, int NTW>
__global__ __launch_bounds__(256) void k_update(T* OUT, const T* IN, double alpha, const T* __restrict__ X,
                                                int64_t xstride, int nprod, const double* __restrict__ S,
                                                int64_t sstride, int trans, double scale, int64_t Np, int ld,
                                                const int* __restrict__ state) {
    if (state && state[0]) return;
    typedef MF<T> M;
    const int l = threadIdx.x & 63, w = threadIdx.x >> 6, lr = l >> 4, lc = l & 15;
    const int64_t m0 = ((int64_t)blockIdx.x * 4 + w) * (16 * MT);
    if (m0 >= Np) return;
    const int jt0 = blockIdx.y * NTW;
    const int ntw = min(NTW, ld / 16 - jt0);
    typename M::acc c[MT][NTW];
#pragma unroll
    for (int a = 0; a < MT; ++a)
#pragma unroll
        for (int b = 0; b < NTW; ++b) c[a][b] = M::zero();
    for (int p = 0; p < nprod; ++p) {
        const T* __restrict__ Xp = X + (int64_t)p * xstride + (m0 + lc) * ld + lr;
        const double* __restrict__ Sp = S + (int64_t)p * sstride;
        for (int k0 = 0; k0 < ld; k0 += 4) {
            T a[MT];
#pragma unroll
            for (int mt = 0; mt < MT; ++mt) a[mt] = Xp[(int64_t)16 * mt * ld + k0];
            const int k = k0 + lr;
#pragma unroll
            for (int nt = 0; nt < NTW; ++nt) {
                if (nt < ntw) {
                    const int j = (jt0 + nt) * 16 + lc;
                    const double sv = trans ? Sp[(int64_t)j * ld + k] : Sp[(int64_t)k * ld + j];
                    const T bv = T(scale * sv);
#pragma unroll
                    for (int mt = 0; mt < MT; ++mt) c[mt][nt] = M::mma(a[mt], bv, c[mt][nt]);
                }
            }
        }
    }
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
        for (int nt = 0; nt < NTW; ++nt) {
            if (nt < ntw) {
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int64_t row = m0 + 16 * mt + M::row(l, r);
                    const int col = (jt0 + nt) * 16 + lc;
                    const int64_t idx = row * ld + col;
                    double v = (double)c[mt][nt][r];
                    if (IN != nullptr && alpha != 0.0) v += alpha * (double)IN[idx];
                    OUT[idx] = T(v);
                }
            }
        }
}

// ------------------------------------------------------------------ small FP64

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

__global__ void k_sym_add(const double* __restrict__ C, double* __restrict__ A, int ld,
                          const int* __restrict__ state) {
    if (state && state[0]) return;
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= ld * ld) return;
    const int i = idx / ld, j = idx % ld;
    A[idx] += 0.5 * (C[idx] + C[j * ld + i]);
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
    static int cached = -1;
    if (cached < 0) {
        int dev = 0, v = 65536;
        if (hipGetDevice(&dev) == hipSuccess &&
            hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) == hipSuccess)
            cached = v;
        else
            cached = 65536;
    }
    return cached;
}

}  // namespace

// ------------------------------------------------------------------ launchers

int64_t gram_partial_mats(int ld) {
    int64_t m = (int64_t(1) << 26) / ((int64_t)ld * ld);
    return std::min<int64_t>(1024, std::max<int64_t>(64, m));
}

GramPlan gram_plan(int64_t Np, int ld, int nprod, bool sym, int64_t cap_mats) {
    GramPlan g;
    g.ld = ld;
    g.nprod = nprod;
    g.Np = Np;
    g.sym = sym;
    const int tpd = (ld + 31) / 32;
    g.ntiles = sym ? tpd * (tpd + 1) / 2 : tpd * tpd;
    int64_t want = (4096 + (int64_t)g.ntiles * nprod - 1) / ((int64_t)g.ntiles * nprod);
    int64_t nchunk = std::max<int64_t>(1, std::min<int64_t>(want, cap_mats / std::max(1, nprod)));
    nchunk = std::min<int64_t>(nchunk, std::max<int64_t>(1, Np / 64));
    int64_t rpc = (Np + nchunk - 1) / nchunk;
    rpc = (rpc + 3) / 4 * 4;
    g.rows_per_chunk = rpc;
    g.nchunk = static_cast<int>((Np + rpc - 1) / rpc);
    return g;
}

template <typename T>
void gram_launch(const GramPlan& g, const T* X, int64_t xstride, const T* Y, double* partial, double* out,
                 int64_t out_stride, int mode, const int* state, hipStream_t s) {
    const int tpd = (g.ld + 31) / 32;
    dim3 grid(g.nchunk, g.ntiles, g.nprod);
    k_gram<T><<<grid, 64, 0, s>>>(X, xstride, Y, g.Np, g.rows_per_chunk, g.ld, tpd, g.sym ? 1 : 0, partial,
                                  g.nchunk, state);
    dim3 rgrid(grid_for((int64_t)g.ld * g.ld, 256), g.nprod);
    k_gram_reduce<<<rgrid, 256, 0, s>>>(partial, g.nchunk, g.ld, g.sym ? 1 : 0, mode, out, out_stride, state);
}

template <typename T>
void update_launch(T* OUT, const T* IN, double alpha, const T* X, int64_t xstride, int nprod, const double* S,
                   int64_t sstride, bool trans, double scale, int64_t Np, int ld, const int* state,
                   hipStream_t s) {
    constexpr int MT = 2, NTW = 8;
    const int64_t rows_per_block = 4 * 16 * MT;
    dim3 grid(static_cast<unsigned>((Np + rows_per_block - 1) / rows_per_block), (ld / 16 + NTW - 1) / NTW);
    k_update<T, MT, NTW><<<grid, 256, 0, s>>>(OUT, IN, alpha, X, xstride, nprod, S, sstride, trans ? 1 : 0, scale,
                                               Np, ld, state);
}

size_t chol_scratch_bytes(int b) { return sizeof(double) * ((size_t)b * (b + 1) + b + 8); }

void chol_inv_launch(const double* G, int b, int ld, const double* tau, double* R, double* Rinv,
                     double* scratch, int* state, int step, double* min_diag, hipStream_t s) {
    const size_t bytes = chol_scratch_bytes(b);
    const bool lds = bytes + 64 <= (size_t)max_lds_bytes();
    k_chol_inv<<<1, 256, lds ? bytes : 0, s>>>(G, b, ld, tau, R, Rinv, scratch, state, step, min_diag,
                                               lds ? 1 : 0);
}

void trmm_upper_launch(const double* R2, const double* R1, double* R, int ld, const int* state, hipStream_t s) {
    k_trmm_upper<<<grid_for((int64_t)ld * ld, 256), 256, 0, s>>>(R2, R1, R, ld, state);
}

void sym_add_launch(const double* C, double* A, int ld, const int* state, hipStream_t s) {
    k_sym_add<<<grid_for((int64_t)ld * ld, 256), 256, 0, s>>>(C, A, ld, state);
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
                                  int64_t, int, const int*, hipStream_t);
template void gram_launch<float>(const GramPlan&, const float*, int64_t, const float*, double*, double*, int64_t,
                                 int, const int*, hipStream_t);
template void update_launch<double>(double*, const double*, double, const double*, int64_t, int, const double*,
                                    int64_t, bool, double, int64_t, int, const int*, hipStream_t);
template void update_launch<float>(float*, const float*, double, const float*, int64_t, int, const double*,
                                   int64_t, bool, double, int64_t, int, const int*, hipStream_t);

}  // namespace css
