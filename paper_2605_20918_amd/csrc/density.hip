// The CSS density matrix on the cutoff pattern (Eqs.(1)-(7) with S = I).
//
// After block Lanczos (lanczos.hip):
//   T  = block tridiagonal projected H (A_j diagonal, B_j below, B_j^T above);
//   F  = [g f(T)]_{:,1} B_0, B_0 = diag(sqrt n_c), f the Fermi function of Eq.(1)
//        (Eqs.(6)-(7)): by default from a pole expansion of the contour integral
//        (subspace.hip); with CSS_SUBSPACE_EIG (and for b > 128) by exact
//        diagonalisation T = U diag(lambda) U^T (rocSOLVER dsyevd),
//        F = U diag(g f(lambda)) U[0:b,:]^T B_0, f evaluated without overflow;
//   X  = sum_j Q_j F_j  (F_j = j-th block of b rows of F)          (Eq.(6));
//   P_mn = s_n X[m, c(n)] on the pattern                           (Eq.(3)),
//        optionally (P + P^T)/2 computed from X directly;
//   trace = sum_m P_mm, e_band = sum over entries in H and the pattern of H_mn P_mn.
// Krylov quadrature: w_k = sum_c n_c U[c,k]^2, trace_K = sum_k g f_k w_k,
// E_K = sum_k lambda_k g f_k w_k. All reductions use a fixed order.

#include <hip/hip_runtime.h>
#include <rocblas/rocblas.h>
#include <rocsolver/rocsolver.h>

#include <algorithm>
#include <cmath>
#include <mutex>
#include <vector>

#include "css_common.h"
#include "dense.h"
#include "driver.h"
#include "spmm.h"
#include "subspace.h"

namespace css {

size_t color_workspace_bytes(int n);
size_t lanczos_workspace_bytes(const LzPlan& p);

namespace {

// ------------------------------------------------------------------ rocSOLVER handle

std::mutex g_mu;
rocblas_handle g_handle[64] = {};

rocblas_handle handle_for_current_device() {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return nullptr;
    if (!g_handle[dev]) {
        rocblas_handle h = nullptr;
        if (rocblas_create_handle(&h) != rocblas_status_success) return nullptr;
        g_handle[dev] = h;
    }
    return g_handle[dev];
}

size_t eig_workspace_bytes(int nT) {
    std::lock_guard<std::mutex> lock(g_mu);
    rocblas_handle h = handle_for_current_device();
    if (!h) return 0;
    size_t sz = 0;
    if (rocblas_start_device_memory_size_query(h) != rocblas_status_success) return 0;
    rocsolver_dsyevd(h, rocblas_evect_original, rocblas_fill_upper, nT, nullptr, nT, nullptr, nullptr, nullptr);
    if (rocblas_stop_device_memory_size_query(h, &sz) != rocblas_status_success) return 0;
    return sz;
}

// Row-major n x n products C = A B on rocBLAS (a plain dense GEMM): column-major
// dgemm of the transposes, C^T = B^T A^T. Workspace from the caller.
css_status gemm_rowmajor(int n, const double* A, const double* B, double* C, void* ws, size_t wsb, hipStream_t s) {
    std::lock_guard<std::mutex> lock(g_mu);
    rocblas_handle h = handle_for_current_device();
    if (!h) return CSS_E_DEVICE;
    if (rocblas_set_stream(h, s) != rocblas_status_success) return CSS_E_DEVICE;
    if (rocblas_set_workspace(h, ws, wsb) != rocblas_status_success) return CSS_E_DEVICE;
    const double one = 1.0, zero = 0.0;
    rocblas_status st = rocblas_dgemm(h, rocblas_operation_none, rocblas_operation_none, n, n, n, &one, B, n, A, n,
                                      &zero, C, n);
    rocblas_set_workspace(h, nullptr, 0);
    return st == rocblas_status_success ? CSS_OK : CSS_E_DEVICE;
}

css_status eig(double* T, int nT, double* lam, double* E, int* dinfo, void* ws, size_t wsb, hipStream_t s) {
    std::lock_guard<std::mutex> lock(g_mu);
    rocblas_handle h = handle_for_current_device();
    if (!h) return CSS_E_DEVICE;
    if (rocblas_set_stream(h, s) != rocblas_status_success) return CSS_E_DEVICE;
    if (rocblas_set_workspace(h, ws, wsb) != rocblas_status_success) return CSS_E_DEVICE;
    rocblas_status st = rocsolver_dsyevd(h, rocblas_evect_original, rocblas_fill_upper, nT, T, nT, lam, E, dinfo);
    rocblas_set_workspace(h, nullptr, 0);
    return st == rocblas_status_success ? CSS_OK : CSS_E_EIG;
}

// ------------------------------------------------------------------ kernels

// T (column-major nT x nT) from the padded A_j, B_j (ld x ld row-major).
__global__ void k_assemble_T(const double* __restrict__ A, const double* __restrict__ B, int v, int b, int ld,
                             double* __restrict__ T, int* __restrict__ bad) {
    const int64_t nT = (int64_t)v * b;
    const int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (idx >= nT * nT) return;
    const int64_t col = idx / nT, row = idx % nT;
    const int bi = (int)(row / b), bj = (int)(col / b);
    const int i = (int)(row % b), j = (int)(col % b);
    const int64_t mat = (int64_t)ld * ld;
    double x = 0.0;
    if (bi == bj)
        x = A[bi * mat + (int64_t)i * ld + j];
    else if (bi == bj + 1)
        x = B[bj * mat + (int64_t)i * ld + j];          // block below the diagonal: B_j
    else if (bj == bi + 1)
        x = B[bi * mat + (int64_t)j * ld + i];          // above: B_j^T
    if (!isfinite(x)) atomicOr(bad, 1);
    T[idx] = x;
}

__device__ __forceinline__ double fermi(double x, double mu, double kT) {
    const double t = (x - mu) / kT;
    if (t > 0.0) {
        const double e = exp(-t);
        return e / (1.0 + e);
    }
    return 1.0 / (1.0 + exp(t));
}

// The function of the projected matrix: g f(x) (Fermi, Eq.(1)) or x^(-1/2) (the
// overlap's inverse square root, 1/sqrt(x) with IEEE sqrt and division).
enum SubFn { kFnFermi = 0, kFnInvSqrt = 1 };

__device__ __forceinline__ double sub_fn(int fn, double x, double mu, double kT, double g) {
    return fn == kFnInvSqrt ? 1.0 / sqrt(x) : g * fermi(x, mu, kT);
}

// Y[k][c] = fn(lambda_k) U[c][k] sqrt(n_c)   (nT x b, row-major)
__global__ void k_occ_y(const double* __restrict__ U, const double* __restrict__ lam, const int* __restrict__ counts,
                        int nT, int b, int fn, double mu, double kT, double g, double* __restrict__ Y) {
    const int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (idx >= (int64_t)nT * b) return;
    const int k = (int)(idx / b), c = (int)(idx % b);
    const double occ = sub_fn(fn, lam[k], mu, kT, g);
    Y[idx] = occ * U[(int64_t)k * nT + c] * sqrt((double)counts[c]);
}

// Per-eigenpair quadrature terms: t0 = fn(lambda) w, t1 = lambda fn(lambda) w; with
// x^(-1/2) a Ritz value <= 0 (overlap not positive definite) sets *bad.
__global__ void k_quad_terms(const double* __restrict__ U, const double* __restrict__ lam,
                             const int* __restrict__ counts, int nT, int b, int fn, double mu, double kT, double g,
                             double* __restrict__ t0, double* __restrict__ t1, int* __restrict__ bad) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= nT) return;
    double w = 0.0;
    for (int c = 0; c < b; ++c) {
        const double u = U[(int64_t)k * nT + c];
        w += (double)counts[c] * u * u;
    }
    if (fn == kFnInvSqrt && !(lam[k] > 0.0)) atomicOr(bad, 1);
    const double occ = sub_fn(fn, lam[k], mu, kT, g);
    t0[k] = occ * w;
    t1[k] = lam[k] * occ * w;
}

// Krylov quadrature weights alone: w_k = sum_c n_c U[c,k]^2.
__global__ void k_quad_weights(const double* __restrict__ U, const int* __restrict__ counts, int nT, int b,
                               double* __restrict__ w) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= nT) return;
    double acc = 0.0;
    for (int c = 0; c < b; ++c) {
        const double u = U[(int64_t)k * nT + c];
        acc += (double)counts[c] * u * u;
    }
    w[k] = acc;
}

constexpr int kMuThreads = 256;
constexpr int kMuMaxIter = 400;

// Block-uniform sum over k of g f_mu(lambda_k) w_k in a fixed order (strided
// per-thread sums, then a fixed tree).
__device__ double krylov_count(const double* __restrict__ lam, const double* __restrict__ w, int nT, double mu,
                               double kT, double g, double* sm) {
    double acc = 0.0;
    for (int k = threadIdx.x; k < nT; k += kMuThreads) acc += g * fermi(lam[k], mu, kT) * w[k];
    sm[threadIdx.x] = acc;
    __syncthreads();
    for (int h = kMuThreads / 2; h > 0; h >>= 1) {
        if (threadIdx.x < h) sm[threadIdx.x] += sm[threadIdx.x + h];
        __syncthreads();
    }
    const double r = sm[0];
    __syncthreads();
    return r;
}

// Bisection for the mu at which the Krylov quadrature count equals n_e, on
// [min lambda - 50 kT, max lambda + 50 kT] (the count is monotone in mu).
// One workgroup; out = {mu, count at mu, iterations, count at the lower end,
// count at the upper end}.
__global__ __launch_bounds__(kMuThreads) void k_mu_bisect(const double* __restrict__ lam, const double* __restrict__ w,
                                                          int nT, double n_e, double kT, double g, double tol,
                                                          double* __restrict__ out) {
    __shared__ double sm[kMuThreads];
    __shared__ double smx[kMuThreads];
    double lo = INFINITY, hi = -INFINITY;
    for (int k = threadIdx.x; k < nT; k += kMuThreads) {
        lo = fmin(lo, lam[k]);
        hi = fmax(hi, lam[k]);
    }
    sm[threadIdx.x] = lo;
    smx[threadIdx.x] = hi;
    __syncthreads();
    for (int h = kMuThreads / 2; h > 0; h >>= 1) {
        if (threadIdx.x < h) {
            sm[threadIdx.x] = fmin(sm[threadIdx.x], sm[threadIdx.x + h]);
            smx[threadIdx.x] = fmax(smx[threadIdx.x], smx[threadIdx.x + h]);
        }
        __syncthreads();
    }
    lo = sm[0] - 50.0 * kT;
    hi = smx[0] + 50.0 * kT;
    __syncthreads();
    const double n_lo = krylov_count(lam, w, nT, lo, kT, g, sm);
    const double n_hi = krylov_count(lam, w, nT, hi, kT, g, sm);
    int it = 0;
    while (hi - lo > tol * fmax(1.0, fmax(fabs(lo), fabs(hi))) && it < kMuMaxIter) {
        const double mid = 0.5 * (lo + hi);
        if (krylov_count(lam, w, nT, mid, kT, g, sm) < n_e)
            lo = mid;
        else
            hi = mid;
        ++it;
    }
    const double mu = 0.5 * (lo + hi);
    const double n_mu = krylov_count(lam, w, nT, mu, kT, g, sm);
    if (threadIdx.x == 0) {
        out[0] = mu;
        out[1] = n_mu;
        out[2] = (double)it;
        out[3] = n_lo;
        out[4] = n_hi;
    }
}

// out[i] = (double)in[i]
template <typename T>
__global__ void k_widen(const T* __restrict__ in, double* __restrict__ out, int64_t n) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < n) out[i] = (double)in[i];
}

// int32 row pointers of a pattern whose nnz is below 2^31 (checked on the host).
__global__ void k_narrow_rp(const int64_t* __restrict__ rp, int32_t* __restrict__ out, int64_t n1) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < n1) out[i] = (int32_t)rp[i];
}

// The probe block r (Eq.(2)): out[m][c] = sign[m] if c = colour(m), else 0; zero padding.
__global__ void k_probe_block(const int32_t* __restrict__ color, const int8_t* __restrict__ sign, int n, int64_t Np,
                              int ld, double* __restrict__ out) {
    const int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (idx >= Np * ld) return;
    const int64_t m = idx / ld;
    const int c = (int)(idx % ld);
    out[idx] = (m < n && color[m] == c) ? (double)sign[m] : 0.0;
}

__global__ void k_fill0(double* __restrict__ p, int64_t n) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0.0;
}

// General first block B_0 = R0 (ld x ld row-major, upper): UB[k][c] = sum_{c' <= c}
// U[c'][k] R0[c'][c]; Y[k][c] = fn(lambda_k) UB[k][c].
__global__ void k_occ_y_r0(const double* __restrict__ U, const double* __restrict__ lam, const double* __restrict__ R0,
                           int nT, int b, int ld, double mu, double kT, double g, double* __restrict__ Y) {
    const int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (idx >= (int64_t)nT * b) return;
    const int k = (int)(idx / b), c = (int)(idx % b);
    double ub = 0.0;
    for (int cp = 0; cp <= c; ++cp) ub += U[(int64_t)k * nT + cp] * R0[(int64_t)cp * ld + c];
    Y[idx] = g * fermi(lam[k], mu, kT) * ub;
}

// Quadrature terms with B_0 = R0: w_k = |R0^T U[0:b,k]|^2, t0 = g f w, t1 = lambda g f w.
__global__ void k_quad_terms_r0(const double* __restrict__ U, const double* __restrict__ lam,
                                const double* __restrict__ R0, int nT, int b, int ld, double mu, double kT, double g,
                                double* __restrict__ t0, double* __restrict__ t1) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= nT) return;
    double w = 0.0;
    for (int c = 0; c < b; ++c) {
        double ub = 0.0;
        for (int cp = 0; cp <= c; ++cp) ub += U[(int64_t)k * nT + cp] * R0[(int64_t)cp * ld + c];
        w += ub * ub;
    }
    const double occ = g * fermi(lam[k], mu, kT);
    t0[k] = occ * w;
    t1[k] = lam[k] * occ * w;
}

__global__ void k_fill_ones(int* __restrict__ p, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 1;
}

// Krylov sums with a triangular B_0 = R0 from F = g f(T) E_1 R0 (nT x b):
// trace_K = sum R0 .* F_1, E_K = sum R0 .* (A_1 F_1 + B_1^T F_2) over the b x b
// leading blocks (elementwise products, entries with c' <= c). One workgroup,
// strided per-thread sums, then a fixed tree.
constexpr int kR0SumThreads = 1024;
__global__ __launch_bounds__(kR0SumThreads) void k_krylov_sums_r0(const double* __restrict__ A,
                                                                   const double* __restrict__ B,
                                                                   const double* __restrict__ F,
                                                                   const double* __restrict__ R0, int v, int b,
                                                                   int ld, double* __restrict__ out) {
    __shared__ double st[kR0SumThreads], se[kR0SumThreads];
    double tr = 0.0, en = 0.0;
    for (int e = threadIdx.x; e < b * b; e += kR0SumThreads) {
        const int cp = e / b, c = e % b;
        if (cp > c) continue;
        const double r = R0[(int64_t)cp * ld + c];
        double g = 0.0;
        for (int k = 0; k < b; ++k) {
            g += A[(int64_t)cp * ld + k] * F[(int64_t)k * b + c];
            if (v > 1) g += B[(int64_t)k * ld + cp] * F[(int64_t)(b + k) * b + c];
        }
        tr += r * F[(int64_t)cp * b + c];
        en += r * g;
    }
    st[threadIdx.x] = tr;
    se[threadIdx.x] = en;
    __syncthreads();
    for (int h = kR0SumThreads / 2; h > 0; h >>= 1) {
        if (threadIdx.x < h) {
            st[threadIdx.x] += st[threadIdx.x + h];
            se[threadIdx.x] += se[threadIdx.x + h];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) { out[0] = st[0]; out[1] = se[0]; }
}

// Coupled Newton-Schulz iteration for the inverse square root of the projected
// overlap (Higham, "Functions of Matrices", 2008, sec. 6.7): with Y_0 = T / c
// (c >= the largest eigenvalue, so the spectrum is in (0, 1]) and Z_0 = I,
//   M = (3 I - Z_k Y_k) / 2,  Y_{k+1} = Y_k M,  Z_{k+1} = M Z_k
// converge quadratically to (T/c)^(1/2) and (T/c)^(-1/2). Matrices n x n row-major.
__global__ void k_ns_init(const double* __restrict__ T, int n, double inv_c, double* __restrict__ Y,
                          double* __restrict__ Z) {
    const int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (idx >= (int64_t)n * n) return;
    const int64_t i = idx / n, j = idx % n;
    Y[idx] = T[idx] * inv_c;
    Z[idx] = (i == j) ? 1.0 : 0.0;
}

// M = (3 I - P) / 2 with P = Z Y; dev[idx] = |P - I| entry (the residual of Z Y = I).
__global__ void k_ns_m(const double* __restrict__ P, int n, double* __restrict__ M, double* __restrict__ dev) {
    const int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (idx >= (int64_t)n * n) return;
    const bool d = (idx / n) == (idx % n);
    const double pv = P[idx];
    M[idx] = 0.5 * ((d ? 3.0 : 0.0) - pv);
    dev[idx] = fabs(pv - (d ? 1.0 : 0.0));
}

// F[k][col] = T^-1/2[k][col] sqrt(n_col) for the first b columns, T^-1/2 = Z / sqrt(c);
// t0[col] = n_col (T^-1/2)[col][col], t1[col] = n_col (T^1/2)[col][col] (T^1/2 = Y sqrt(c)).
__global__ void k_ns_finish(const double* __restrict__ Z, const double* __restrict__ Y, const int* __restrict__ counts,
                            int nT, int b, double c, double* __restrict__ F, double* __restrict__ t0,
                            double* __restrict__ t1) {
    const int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (idx >= (int64_t)nT * b) return;
    const int64_t k = idx / b;
    const int col = (int)(idx % b);
    const double rs = 1.0 / sqrt(c);
    const double nc = (double)counts[col];
    F[idx] = Z[k * nT + col] * rs * sqrt(nc);
    if (k == 0) {
        t0[col] = nc * Z[(int64_t)col * nT + col] * rs;
        t1[col] = nc * Y[(int64_t)col * nT + col] * sqrt(c);
    }
}

// Pattern sanity: row pointers monotone from 0 to nnz, columns in range and strictly
// increasing within each row (the band energy binary-searches the rows).
// One wave per row (grid-stride): row bounds, then every adjacent pair of the row's
// columns at once (strictly increasing); every thread also range-checks the columns
// t = global thread index, t + stride, ... One flag for any violation.
__global__ __launch_bounds__(256) void k_validate_pattern(int n, int64_t nnz, const int64_t* __restrict__ rp,
                                                         const int32_t* __restrict__ col, int* __restrict__ bad) {
    const int lane = threadIdx.x & 63;
    const int64_t nwaves = (int64_t)gridDim.x * (blockDim.x / 64);
    bool fail = false;
    for (int64_t i = (int64_t)blockIdx.x * (blockDim.x / 64) + (threadIdx.x >> 6); i < n; i += nwaves) {
        const int64_t a = rp[i], b = rp[i + 1];
        if (a < 0 || b < a || b > nnz || (i == 0 && a != 0) || (i == n - 1 && b != nnz)) {
            fail = true;
            continue;
        }
        for (int64_t t = a + 1 + lane; t < b; t += 64)
            if (col[t - 1] >= col[t]) fail = true;
    }
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < nnz; t += stride) {
        const int32_t c = col[t];
        if (c < 0 || c >= n) fail = true;
    }
    if (fail) atomicOr(bad, 1);
}
void validate_pattern_launch(int n, int64_t nnz, const int64_t* rp, const int32_t* col, int* bad, hipStream_t s) {
    const unsigned grid = std::max(1u, std::min<unsigned>(grid_for(n, 4), 16384));
    k_validate_pattern<<<grid, 256, 0, s>>>(n, nnz, rp, col, bad);
}

// Fpad[j][i][c] = F[j*b + i][c] for i, c < b; zero in the padding.
__global__ void k_pad_F(const double* __restrict__ F, int v, int b, int ld, double* __restrict__ Fpad) {
    const int64_t mat = (int64_t)ld * ld;
    const int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (idx >= v * mat) return;
    const int j = (int)(idx / mat);
    const int i = (int)((idx % mat) / ld), c = (int)(idx % ld);
    Fpad[idx] = (i < b && c < b) ? F[((int64_t)j * b + i) * b + c] : 0.0;
}

// One wavefront per pattern row: P values, the diagonal and the raw asymmetry.
template <typename T>
__global__ __launch_bounds__(256) void k_gather(int n, const int64_t* __restrict__ prp, const int32_t* __restrict__ pcol,
                                                const int32_t* __restrict__ color, const int8_t* __restrict__ sign,
                                                const T* __restrict__ X, int ld, int sym, double* __restrict__ pval,
                                                double* __restrict__ row_trace, double* __restrict__ row_asym) {
    const int lane = threadIdx.x & 63;
    const int64_t m = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (m >= n) return;
    const int cm = color[m];
    const double sm = (double)sign[m];
    const T* __restrict__ xm = X + m * ld;
    double tr = 0.0, asym = 0.0;
    for (int64_t t = prp[m] + lane; t < prp[m + 1]; t += 64) {
        const int nn = pcol[t];
        const double raw = (double)sign[nn] * (double)xm[color[nn]];
        const double rt = sm * (double)X[(int64_t)nn * ld + cm];
        const double v = 0.5 * (raw + rt);
        asym = fmax(asym, fabs(raw - v));
        const double out = sym ? v : raw;
        pval[t] = out;
        if (nn == m) tr = out;
    }
    for (int off = 32; off > 0; off >>= 1) {
        tr += __shfl_xor(tr, off);          // only one lane holds the diagonal: order is irrelevant
        asym = fmax(asym, __shfl_xor(asym, off));
    }
    if (lane == 0) {
        row_trace[m] = tr;
        row_asym[m] = asym;
    }
}

// One wavefront per row: sum over H entries present in the pattern of H_mn P_mn.
// The pattern row is staged in a per-wavefront LDS slice when it has at most
// kEnergyLds entries, so each lane's binary search reads LDS instead of making a
// chain of dependent global loads (found positions and the order of the sums are
// the same either way).
constexpr int kEnergyLds = 512;

template <typename V>
__global__ __launch_bounds__(256) void k_energy(int n, const int32_t* __restrict__ hrp, const int32_t* __restrict__ hcol,
                                                const V* __restrict__ hval, const int64_t* __restrict__ prp,
                                                const int32_t* __restrict__ pcol, const double* __restrict__ pval,
                                                double* __restrict__ row_e) {
    __shared__ int32_t prow_lds[4][kEnergyLds];
    const int lane = threadIdx.x & 63;
    const int w = __builtin_amdgcn_readfirstlane(static_cast<int>(threadIdx.x >> 6));
    const int64_t m = (int64_t)blockIdx.x * 4 + w;
    if (m >= n) return;
    const int64_t ps = prp[m], pe = prp[m + 1];
    const bool staged = pe - ps <= kEnergyLds;                      // uniform over the wavefront
    int32_t* prow = prow_lds[w];
    if (staged) {
        for (int64_t i = lane; i < pe - ps; i += 64) prow[i] = pcol[ps + i];
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront", "local");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront", "local");
    }
    double e = 0.0;
    for (int32_t t = hrp[m] + lane; t < hrp[m + 1]; t += 64) {
        const int nn = hcol[t];
        int64_t lo = ps, hi = pe;          // binary search nn in the sorted pattern row
        bool hit;
        if (staged) {
            int a = 0, b = static_cast<int>(pe - ps);
            while (a < b) {
                const int mid = (a + b) >> 1;
                if (prow[mid] < nn) a = mid + 1; else b = mid;
            }
            lo = ps + a;
            hit = lo < pe && prow[a] == nn;
        } else {
            while (lo < hi) {
                const int64_t mid = (lo + hi) >> 1;
                if (pcol[mid] < nn) lo = mid + 1; else hi = mid;
            }
            hit = lo < pe && pcol[lo] == nn;
        }
        if (hit) e += (double)hval[t] * pval[lo];
    }
    for (int off = 32; off > 0; off >>= 1) e += __shfl_xor(e, off);
    if (lane == 0) row_e[m] = e;
}

// One wavefront per pattern row: sum of P_mn^2 over the row (fixed order per row).
__global__ __launch_bounds__(256) void k_row_sq(int n, const int64_t* __restrict__ prp,
                                                const double* __restrict__ pval, double* __restrict__ row_sq) {
    const int lane = threadIdx.x & 63;
    const int64_t m = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (m >= n) return;
    double q = 0.0;
    for (int64_t t = prp[m] + lane; t < prp[m + 1]; t += 64) q += pval[t] * pval[t];
    for (int off = 32; off > 0; off >>= 1) q += __shfl_xor(q, off);
    if (lane == 0) row_sq[m] = q;
}

// Deterministic two-level sum: block b sums v[b*chunk ...) in a fixed tree.
__global__ void k_block_sum(const double* __restrict__ v, int64_t n, int64_t chunk, double* __restrict__ out) {
    __shared__ double sm[256];
    const int64_t s = blockIdx.x * chunk, e = min(n, s + chunk);
    double acc = 0.0;
    for (int64_t i = s + threadIdx.x; i < e; i += 256) acc += v[i];
    sm[threadIdx.x] = acc;
    __syncthreads();
    for (int k = 128; k > 0; k >>= 1) {
        if (threadIdx.x < k) sm[threadIdx.x] += sm[threadIdx.x + k];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[blockIdx.x] = sm[0];
}

__global__ void k_block_max(const double* __restrict__ v, int64_t n, double* __restrict__ out) {
    __shared__ double sm[256];
    double m = 0.0;
    for (int64_t i = blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) m = fmax(m, v[i]);
    sm[threadIdx.x] = m;
    __syncthreads();
    for (int k = 128; k > 0; k >>= 1) {
        if (threadIdx.x < k) sm[threadIdx.x] = fmax(sm[threadIdx.x], sm[threadIdx.x + k]);
        __syncthreads();
    }
    if (threadIdx.x == 0) out[blockIdx.x] = sm[0];
}

constexpr int kSumBlocks = 256;

// out = sum(v[0..n)) with a fixed order: kSumBlocks partial sums, then one block.
void det_sum(const double* v, int64_t n, double* tmp, double* out, hipStream_t s) {
    const int64_t chunk = std::max<int64_t>(1, (n + kSumBlocks - 1) / kSumBlocks);
    const int nb = (int)((n + chunk - 1) / chunk);
    k_block_sum<<<std::max(1, nb), 256, 0, s>>>(v, n, chunk, tmp);
    k_block_sum<<<1, 256, 0, s>>>(tmp, std::max(1, nb), std::max(1, nb), out);
}

void det_max(const double* v, int64_t n, double* tmp, double* out, hipStream_t s) {
    k_block_max<<<kSumBlocks, 256, 0, s>>>(v, n, tmp);
    k_block_max<<<1, 256, 0, s>>>(tmp, kSumBlocks, out);
}

// ------------------------------------------------------------------ plan

// Newton-Schulz scratch (one nT x nT product buffer, also the Gershgorin scratch of
// 2 nT + 16 doubles taken in three 256-byte-aligned pieces).
int64_t ns_scratch_doubles(int64_t nT) { return std::max<int64_t>(nT * nT, 2 * nT + 16) + 128; }

struct DmPlan {
    LzPlan lz;
    int nTmax = 0;
    bool use_eig = false;     // dense diagonalisation (rocSOLVER) instead of the pole expansion
    size_t eig_ws = 0;
    size_t pole_ws = 0;
    bool sep_X = false;
    bool energy = false;      // also the energy-weighted estimate (X_E = H X)
    bool hprime = false;      // also H' = S^-1/2 H S^-1/2 extracted after S^-1/2 (FP64 products)
    bool nonorth = false;     // density of a non-orthogonal basis: Lanczos on H' from S^-1/2 r
    bool ns = false;          // T^-1/2 by the coupled Newton-Schulz iteration (overlap path)
};

struct DmBufs {
    LzBufs lz;
    double *T = nullptr, *lam = nullptr, *E = nullptr, *Y = nullptr, *F = nullptr, *Fpad = nullptr;
    void* pole_ws = nullptr;
    double *t0 = nullptr, *t1 = nullptr, *rows = nullptr, *tmp = nullptr, *res = nullptr;
    int* flags = nullptr;
    void* X = nullptr;
    void* XE = nullptr;       // H X (energy-weighted estimate)
    double *Y64 = nullptr, *Z1 = nullptr, *Z = nullptr, *h64 = nullptr;   // H' extraction (FP64)
    double* R0 = nullptr;     // non-orthogonal: the first block's triangular factor
    int* ones = nullptr;      // non-orthogonal pole path: B_0 = I for the pole solve
    double *nsY = nullptr, *nsZ = nullptr, *nsM = nullptr, *nsP = nullptr;   // Newton-Schulz (nT x nT)
    int32_t* rp32 = nullptr;
    void* eig_ws = nullptr;
};

void carve_dm(Arena& a, const DmPlan& p, DmBufs& bf) {
    carve_lanczos(a, p.lz, bf.lz);
    const int64_t nT = p.nTmax;
    const int64_t mat = (int64_t)p.lz.ld * p.lz.ld;
    bf.T = p.use_eig ? a.take<double>(nT * nT) : nullptr;
    bf.lam = a.take<double>(nT);
    bf.E = a.take<double>(nT);
    bf.Y = (p.use_eig || p.nonorth) ? a.take<double>(nT * p.lz.b) : nullptr;
    bf.F = a.take<double>(nT * p.lz.b);
    bf.Fpad = a.take<double>(std::max(1, p.lz.v_max) * mat);
    bf.t0 = a.take<double>(nT);
    bf.t1 = a.take<double>(nT);
    bf.rows = a.take<double>(3 * (int64_t)p.lz.n);
    bf.tmp = a.take<double>(4 * kSumBlocks);
    bf.res = a.take<double>(16);
    bf.flags = a.take<int>(16);
    bf.X = p.sep_X ? a.take<char>((size_t)p.lz.Np * p.lz.ld * p.lz.elem) : bf.lz.W;
    bf.XE = p.energy ? a.take<char>((size_t)p.lz.Np * p.lz.ld * p.lz.elem) : nullptr;
    if (p.hprime || p.nonorth) {
        const int64_t tall = p.lz.Np * p.lz.ld;
        bf.Y64 = a.take<double>(tall);
        bf.Z1 = a.take<double>(tall);
        bf.Z = a.take<double>(tall);
    }
    if (p.hprime) {
        bf.h64 = a.take<double>(std::max<int64_t>(1, p.lz.nnz));
        bf.rp32 = a.take<int32_t>(p.lz.n + 1);
    }
    if (p.nonorth) {
        bf.R0 = a.take<double>(mat);
        bf.ones = a.take<int>(p.lz.b);
    }
    if (p.ns) {
        bf.nsY = a.take<double>(nT * nT);
        bf.nsZ = a.take<double>(nT * nT);
        bf.nsM = a.take<double>(nT * nT);
        bf.nsP = a.take<double>(ns_scratch_doubles(nT));
    }
    bf.eig_ws = p.eig_ws ? a.take<char>(p.eig_ws) : nullptr;
    bf.pole_ws = p.pole_ws ? a.take<char>(p.pole_ws) : nullptr;
}

css_status plan_dm(const css_csr* H, int32_t b, int32_t depth, uint32_t flags, DmPlan& p) {
    CSS_TRY(plan_lanczos(H, b, depth, flags, p.lz));
    p.nTmax = std::max(1, p.lz.v_max) * b;
    p.sep_X = p.lz.twopass;
    // the pole solver takes b <= 128; wider blocks are diagonalised
    p.use_eig = (flags & CSS_SUBSPACE_EIG) != 0 || b > 128;
    if (p.use_eig) {
        p.eig_ws = eig_workspace_bytes(p.nTmax);
        if (p.eig_ws == 0) return CSS_E_DEVICE;
    } else {
        p.pole_ws = pole_workspace_bytes(std::max(1, p.lz.v_max), b);
    }
    return CSS_OK;
}

size_t dm_workspace_bytes(const DmPlan& p) {
    Arena a;
    DmBufs bf;
    carve_dm(a, p, bf);
    return a.used + 256;
}

template <typename T>
void launch_gather(int n, const int64_t* prp, const int32_t* pcol, const int32_t* color, const int8_t* sign,
                   const void* X, int ld, int sym, double* pval, double* rt, double* ra, hipStream_t s) {
    k_gather<T><<<grid_for(n, 4), 256, 0, s>>>(n, prp, pcol, color, sign, static_cast<const T*>(X), ld, sym, pval,
                                               rt, ra);
}

}  // namespace
}  // namespace css

using namespace css;

namespace css {
namespace {

// The density-matrix path; with pe_val also the energy-weighted estimate.
css_status dm_run(const css_csr* H, const int32_t* color, const int8_t* sign, int32_t n_colors, double mu, double kT,
                  int32_t depth, double spin_deg, const int64_t* p_row_ptr, const int32_t* p_col, int64_t p_nnz,
                  uint32_t flags, double* p_val, double* pe_val, double* e_band, double* trace, double* pe_trace,
                  css_info* info, void* ws, size_t ws_bytes, void* stream, int fn = kFnFermi,
                  const css_csr* H2 = nullptr, double* h2_val = nullptr, bool timed = true,
                  size_t pole_ws = 0) {
    if (!color || !sign || !p_row_ptr || !p_col || !p_val || !e_band || !trace || !ws || p_nnz < 1) return CSS_E_ARG;
    if (fn == kFnFermi && (!(kT > 0.0) || !std::isfinite(kT) || !std::isfinite(mu) || !(spin_deg > 0.0)))
        return CSS_E_ARG;
    const bool ns = fn == kFnInvSqrt && !(flags & CSS_SUBSPACE_EIG);
    if (fn == kFnInvSqrt) flags |= CSS_SUBSPACE_EIG;
    DmPlan p;
    CSS_TRY(plan_dm(H, n_colors, depth, flags, p));
    if (pole_ws && !p.use_eig) p.pole_ws = pole_ws;      // the caller's pole budget (the rest of its scratch)
    p.ns = ns;
    p.energy = pe_val != nullptr;
    p.hprime = h2_val != nullptr;
    if (p.hprime) {
        // H' extraction: H2 shares S's size, and its nnz fits the reserved FP64 copy
        if (fn != kFnInvSqrt || !H2 || !H2->row_ptr || !H2->col || !H2->val || H2->n != H->n || H2->nnz < 1 ||
            H2->nnz > H->nnz || p_nnz >= (int64_t(1) << 31))
            return CSS_E_ARG;
    }
    if (ws_bytes < dm_workspace_bytes(p)) return CSS_E_WORKSPACE;
    Arena a;
    a.base = static_cast<char*>(ws);
    a.cap = ws_bytes;
    DmBufs bf;
    carve_dm(a, p, bf);
    if (a.overflow) return CSS_E_WORKSPACE;
    hipStream_t s = as_stream(stream);
    const LzPlan& lz = p.lz;

    // phase events (timed = false: none, for callers that must not allocate)
    hipEvent_t ev[6] = {};
    if (timed)
        for (auto& e : ev) CSS_HIP_TRY(hipEventCreate(&e));
    struct Guard {
        hipEvent_t* e;
        ~Guard() { for (int i = 0; i < 6; ++i) if (e[i]) (void)hipEventDestroy(e[i]); }
    } guard{ev};
    if (timed) CSS_HIP_TRY(hipEventRecord(ev[0], s));

    {
        fill_launch<int>(bf.flags, 0, 16, s);
        validate_pattern_launch(lz.n, p_nnz, p_row_ptr, p_col, bf.flags, s);
        int pbad = 0;
        CSS_HIP_TRY(hipMemcpyAsync(&pbad, bf.flags, sizeof(int), hipMemcpyDeviceToHost, s));
        CSS_HIP_TRY(hipStreamSynchronize(s));
        if (pbad) return CSS_E_CSR;
    }
    int v_eff = 0, brk = 0;
    double md = 0.0;
    CSS_TRY(run_lanczos_pass1(H, color, sign, lz, bf.lz, s, &v_eff, &brk, &md));
    double ortho = NAN;
    if (flags & CSS_DIAG_ORTHO) CSS_TRY(lanczos_ortho_err(lz, bf.lz, v_eff, s, &ortho));
    if (timed) CSS_HIP_TRY(hipEventRecord(ev[1], s));

    // Fermi operator in the Krylov subspace: F = g f(T) E_1 B_0 and the quadrature sums
    const int nT = v_eff * lz.b;
    const int64_t mat = (int64_t)lz.ld * lz.ld;
    int npoles = 0;
    if (p.ns) {
        // T^-1/2 E_1 B_0 by the coupled Newton-Schulz iteration on T / c, c the
        // Gershgorin upper bound; a non-positive bound or no convergence in 60
        // iterations means T (so S) is not positive definite
        fill_launch<int>(bf.flags, 0, 16, s);
        k_assemble_T<<<grid_for((int64_t)nT * nT, 256), 256, 0, s>>>(bf.lz.A, bf.lz.B, v_eff, lz.b, lz.ld, bf.T,
                                                                     bf.flags);
        int hbad = 0;
        CSS_HIP_TRY(hipMemcpyAsync(&hbad, bf.flags, sizeof(int), hipMemcpyDeviceToHost, s));
        CSS_HIP_TRY(hipStreamSynchronize(s));
        if (hbad) return CSS_E_NONFINITE;
        double glo = 0.0, ghi = 0.0;
        CSS_TRY(subspace_spectral_bounds(bf.lz.A, bf.lz.B, v_eff, lz.b, lz.ld, bf.nsP,
                                         sizeof(double) * ns_scratch_doubles(p.nTmax), &glo, &ghi, s));
        if (!(ghi > 0.0)) return CSS_E_NONFINITE;
        const int64_t nn = (int64_t)nT * nT;
        k_ns_init<<<grid_for(nn, 256), 256, 0, s>>>(bf.T, nT, 1.0 / ghi, bf.nsY, bf.nsZ);
        bool conv = false;
        for (int it = 0; it < 60 && !conv; ++it) {
            CSS_TRY(gemm_rowmajor(nT, bf.nsZ, bf.nsY, bf.nsP, bf.eig_ws, p.eig_ws, s));         // P = Z Y
            k_ns_m<<<grid_for(nn, 256), 256, 0, s>>>(bf.nsP, nT, bf.nsM, bf.T);               // M, |ZY - I|
            det_max(bf.T, nn, bf.tmp, bf.res + 8, s);
            double r = 0.0;
            CSS_HIP_TRY(hipMemcpyAsync(&r, bf.res + 8, sizeof(double), hipMemcpyDeviceToHost, s));
            CSS_TRY(gemm_rowmajor(nT, bf.nsY, bf.nsM, bf.nsP, bf.eig_ws, p.eig_ws, s));         // P = Y M
            std::swap(bf.nsY, bf.nsP);
            CSS_TRY(gemm_rowmajor(nT, bf.nsM, bf.nsZ, bf.nsP, bf.eig_ws, p.eig_ws, s));         // P = M Z
            std::swap(bf.nsZ, bf.nsP);
            CSS_HIP_TRY(hipStreamSynchronize(s));
            if (!std::isfinite(r)) return CSS_E_NONFINITE;
            conv = r <= 1e-9;          // the update above then leaves an error of order r^2
        }
        if (!conv) return CSS_E_NONFINITE;
        if (timed) CSS_HIP_TRY(hipEventRecord(ev[2], s));
        k_ns_finish<<<grid_for((int64_t)nT * lz.b, 256), 256, 0, s>>>(bf.nsZ, bf.nsY, bf.lz.counts, nT, lz.b, ghi,
                                                                       bf.F, bf.t0, bf.t1);
        det_sum(bf.t0, lz.b, bf.tmp, bf.res + 2, s);
        det_sum(bf.t1, lz.b, bf.tmp + kSumBlocks, bf.res + 3, s);
    } else if (p.use_eig) {
        fill_launch<int>(bf.flags, 0, 16, s);
        k_assemble_T<<<grid_for((int64_t)nT * nT, 256), 256, 0, s>>>(bf.lz.A, bf.lz.B, v_eff, lz.b, lz.ld, bf.T,
                                                                     bf.flags);
        int hbad = 0;
        CSS_HIP_TRY(hipMemcpyAsync(&hbad, bf.flags, sizeof(int), hipMemcpyDeviceToHost, s));
        CSS_HIP_TRY(hipStreamSynchronize(s));
        if (hbad) return CSS_E_NONFINITE;
        CSS_TRY(eig(bf.T, nT, bf.lam, bf.E, bf.flags + 1, bf.eig_ws, p.eig_ws, s));
        if (timed) CSS_HIP_TRY(hipEventRecord(ev[2], s));
        k_occ_y<<<grid_for((int64_t)nT * lz.b, 256), 256, 0, s>>>(bf.T, bf.lam, bf.lz.counts, nT, lz.b, fn, mu, kT,
                                                                    spin_deg, bf.Y);
        gemm_f64_launch(nT, lz.b, nT, bf.T, 1, nT, bf.Y, lz.b, 1, bf.F, lz.b, 1, s);
        k_quad_terms<<<grid_for(nT, 256), 256, 0, s>>>(bf.T, bf.lam, bf.lz.counts, nT, lz.b, fn, mu, kT, spin_deg,
                                                       bf.t0, bf.t1, bf.flags + 2);
        det_sum(bf.t0, nT, bf.tmp, bf.res + 2, s);
        det_sum(bf.t1, nT, bf.tmp + kSumBlocks, bf.res + 3, s);
    } else {
        fill_launch<int>(bf.flags, 0, 16, s);
        CSS_TRY(subspace_fermi_poles(bf.lz.A, bf.lz.B, v_eff, lz.b, lz.ld, bf.lz.counts, mu, kT, spin_deg, bf.F,
                                     bf.res + 2, bf.pole_ws, p.pole_ws, &npoles, s));
        if (timed) CSS_HIP_TRY(hipEventRecord(ev[2], s));
    }
    k_pad_F<<<grid_for(v_eff * mat, 256), 256, 0, s>>>(bf.F, v_eff, lz.b, lz.ld, bf.Fpad);
    if (timed) CSS_HIP_TRY(hipEventRecord(ev[3], s));

    // reconstruction X = sum_j Q_j F_j
    if (lz.twopass) {
        CSS_TRY(run_lanczos_pass2(H, color, sign, lz, bf.lz, v_eff, bf.Fpad, bf.X, s));
    } else if (lz.fp32) {
        update_launch<float>(static_cast<float*>(bf.X), nullptr, 0.0, static_cast<const float*>(slot_ptr(lz, bf.lz, 0)),
                             lz.Np * lz.ld, v_eff, bf.Fpad, mat, false, 1.0, lz.Np, lz.ld, bf.lz.stage, nullptr, s);
    } else {
        update_launch<double>(static_cast<double*>(bf.X), nullptr, 0.0,
                              static_cast<const double*>(slot_ptr(lz, bf.lz, 0)), lz.Np * lz.ld, v_eff, bf.Fpad, mat,
                              false, 1.0, lz.Np, lz.ld, bf.lz.stage, nullptr, s);
    }
    if (timed) CSS_HIP_TRY(hipEventRecord(ev[4], s));

    // extraction on the pattern, trace, band energy
    const int sym = (flags & CSS_SYMMETRIZE) ? 1 : 0;
    double* rt = bf.rows;
    double* ra = bf.rows + lz.n;
    double* re = bf.rows + 2 * (int64_t)lz.n;
    if (lz.fp32)
        launch_gather<float>(lz.n, p_row_ptr, p_col, color, sign, bf.X, lz.ld, sym, p_val, rt, ra, s);
    else
        launch_gather<double>(lz.n, p_row_ptr, p_col, color, sign, bf.X, lz.ld, sym, p_val, rt, ra, s);
    if (H->val_dtype == CSS_F64)
        k_energy<double><<<grid_for(lz.n, 4), 256, 0, s>>>(lz.n, H->row_ptr, H->col, static_cast<const double*>(H->val),
                                                           p_row_ptr, p_col, p_val, re);
    else
        k_energy<float><<<grid_for(lz.n, 4), 256, 0, s>>>(lz.n, H->row_ptr, H->col, static_cast<const float*>(H->val),
                                                          p_row_ptr, p_col, p_val, re);
    det_sum(rt, lz.n, bf.tmp + 2 * kSumBlocks, bf.res + 0, s);
    det_sum(re, lz.n, bf.tmp + 3 * kSumBlocks, bf.res + 1, s);
    det_max(ra, lz.n, bf.tmp, bf.res + 4, s);
    // ||P||_F^2 on the pattern for the idempotency defect (rows of ra reused in stream order)
    k_row_sq<<<grid_for(lz.n, 4), 256, 0, s>>>(lz.n, p_row_ptr, p_val, ra);
    det_sum(ra, lz.n, bf.tmp + kSumBlocks, bf.res + 6, s);
    if (pe_val) {
        // energy-weighted estimate: X_E = H X, gathered as P (the rows' scratch is reused
        // after the reductions above, in stream order)
        CSS_TRY(lanczos_spmm(H, lz, bf.lz, bf.X, bf.XE, s));
        if (lz.fp32)
            launch_gather<float>(lz.n, p_row_ptr, p_col, color, sign, bf.XE, lz.ld, sym, pe_val, rt, ra, s);
        else
            launch_gather<double>(lz.n, p_row_ptr, p_col, color, sign, bf.XE, lz.ld, sym, pe_val, rt, ra, s);
        det_sum(rt, lz.n, bf.tmp + 2 * kSumBlocks, bf.res + 5, s);
    }
    if (h2_val) {
        // H' = S^-1/2 H S^-1/2 read off S^-1/2 (H Y) o^T: Y is S^-1/2 applied to the
        // probes (X above), S^-1/2 the sparse estimate just gathered; FP64 products
        fill_launch<int>(bf.flags + 3, 0, 4, s);
        csr_validate_launch(lz.n, H2->nnz, H2->row_ptr, H2->col, bf.flags + 3, s);
        int vbad[2] = {0, 0};
        CSS_HIP_TRY(hipMemcpyAsync(vbad, bf.flags + 3, 2 * sizeof(int), hipMemcpyDeviceToHost, s));
        CSS_HIP_TRY(hipStreamSynchronize(s));
        if (vbad[1]) return CSS_E_CSR;
        const int64_t tall = lz.Np * lz.ld;
        if (lz.fp32)
            k_widen<float><<<grid_for(tall, 256), 256, 0, s>>>(static_cast<const float*>(bf.X), bf.Y64, tall);
        else
            CSS_HIP_TRY(hipMemcpyAsync(bf.Y64, bf.X, tall * sizeof(double), hipMemcpyDeviceToDevice, s));
        const double* h2v = static_cast<const double*>(H2->val);
        if (H2->val_dtype == CSS_F32) {
            k_widen<float><<<grid_for(H2->nnz, 256), 256, 0, s>>>(static_cast<const float*>(H2->val), bf.h64,
                                                                   H2->nnz);
            h2v = bf.h64;
        } else if (H2->val_dtype != CSS_F64) {
            return CSS_E_ARG;
        }
        k_narrow_rp<<<grid_for(lz.n + 1, 256), 256, 0, s>>>(p_row_ptr, bf.rp32, lz.n + 1);
        if (!spmm_launch<double>(SpmmArgs<double>{lz.n, H2->row_ptr, H2->col, h2v, bf.Y64, bf.Z1, lz.ld}, s) ||
            !spmm_launch<double>(SpmmArgs<double>{lz.n, bf.rp32, p_col, p_val, bf.Z1, bf.Z, lz.ld}, s))
            return CSS_E_UNSUPPORTED;
        launch_gather<double>(lz.n, p_row_ptr, p_col, color, sign, bf.Z, lz.ld, sym, h2_val, rt, ra, s);
        det_sum(rt, lz.n, bf.tmp + 2 * kSumBlocks, bf.res + 5, s);
    }
    if (timed) CSS_HIP_TRY(hipEventRecord(ev[5], s));
    double hres[8];
    int hinfo[2] = {0, 0};
    CSS_HIP_TRY(hipMemcpyAsync(hres, bf.res, 7 * sizeof(double), hipMemcpyDeviceToHost, s));
    CSS_HIP_TRY(hipMemcpyAsync(hinfo, bf.flags + 1, 2 * sizeof(int), hipMemcpyDeviceToHost, s));
    CSS_HIP_TRY(hipStreamSynchronize(s));
    CSS_HIP_TRY(hipGetLastError());
    if (hinfo[0] != 0) return CSS_E_EIG;
    if (hinfo[1] != 0) return CSS_E_NONFINITE;
    *trace = hres[0];
    *e_band = hres[1];
    if ((pe_val || h2_val) && pe_trace) *pe_trace = hres[5];
    if (info) {
        *info = css_info{};
        info->depth_eff = v_eff;
        info->n_colors = lz.b;
        info->breakdown = brk;
        info->spmm_kernel = bf.lz.use_grp ? 1 : 0;
        info->min_diag_r = md;
        info->ortho_err = ortho;
        info->idem_defect = fn == kFnFermi ? hres[0] - hres[6] / spin_deg : NAN;
        info->asym_max = hres[4];
        info->n_poles = npoles;
        info->trace_krylov = hres[2];
        info->e_band_krylov = hres[3];
        for (int k = 0; timed && k < 5; ++k) {
            float ms = 0.f;
            if (hipEventElapsedTime(&ms, ev[k], ev[k + 1]) == hipSuccess) info->t_phase_ms[k] = ms;
        }
        float tot = 0.f;
        if (timed && hipEventElapsedTime(&tot, ev[0], ev[5]) == hipSuccess) info->t_phase_ms[5] = tot;
    }
    return CSS_OK;
}

// Density matrix of a non-orthogonal basis (Eq.(6)): rho~ = S^-1/2 Phi rho^K Phi^T r~ r^T
// with r~ = S^-1/2 r and the block Krylov space of H' from r~; S^-1/2 sparse.
css_status nonorth_run(const css_csr* Hp, const css_csr* Sih, const css_csr* He, const css_csr* Se,
                       const int32_t* color, const int8_t* sign, int32_t n_colors, double mu, double kT,
                       int32_t depth, double spin_deg, const int64_t* p_row_ptr, const int32_t* p_col, int64_t p_nnz,
                       uint32_t flags, double* p_val, double* e_band, double* n_elec, double* trace, css_info* info,
                       void* ws, size_t ws_bytes, void* stream) {
    if (!Hp || !Sih || !color || !sign || !p_row_ptr || !p_col || !p_val || !trace || !ws || p_nnz < 1)
        return CSS_E_ARG;
    if (!(kT > 0.0) || !std::isfinite(kT) || !std::isfinite(mu) || !(spin_deg > 0.0)) return CSS_E_ARG;
    if (!Sih->row_ptr || !Sih->col || !Sih->val || Sih->n != Hp->n || Sih->val_dtype != CSS_F64 || Sih->nnz < 1 ||
        Sih->nnz >= (int64_t(1) << 31))
        return CSS_E_ARG;
    if ((e_band && !He) || (n_elec && !Se)) return CSS_E_ARG;
    for (const css_csr* M : {He, Se})
        if (M && (M->n != Hp->n || !M->row_ptr || !M->col || !M->val || M->nnz < 1 ||
                  (M->val_dtype != CSS_F64 && M->val_dtype != CSS_F32)))
            return CSS_E_ARG;
    DmPlan p;
    CSS_TRY(plan_dm(Hp, n_colors, depth, flags, p));
    if (p.lz.twopass) return CSS_E_UNSUPPORTED;
    p.nonorth = true;
    if (ws_bytes < dm_workspace_bytes(p)) return CSS_E_WORKSPACE;
    Arena a;
    a.base = static_cast<char*>(ws);
    a.cap = ws_bytes;
    DmBufs bf;
    carve_dm(a, p, bf);
    if (a.overflow) return CSS_E_WORKSPACE;
    hipStream_t s = as_stream(stream);
    const LzPlan& lz = p.lz;
    const int64_t tall = lz.Np * lz.ld;

    hipEvent_t ev[6] = {};
    for (auto& e : ev) CSS_HIP_TRY(hipEventCreate(&e));
    struct Guard {
        hipEvent_t* e;
        ~Guard() { for (int i = 0; i < 6; ++i) if (e[i]) (void)hipEventDestroy(e[i]); }
    } guard{ev};
    CSS_HIP_TRY(hipEventRecord(ev[0], s));

    // inputs: the pattern and the sparse S^-1/2 (and H, S for the sums)
    fill_launch<int>(bf.flags, 0, 16, s);
    validate_pattern_launch(lz.n, p_nnz, p_row_ptr, p_col, bf.flags, s);
    csr_validate_launch(lz.n, Sih->nnz, Sih->row_ptr, Sih->col, bf.flags + 3, s);
    if (He) csr_validate_launch(lz.n, He->nnz, He->row_ptr, He->col, bf.flags + 5, s);
    if (Se) csr_validate_launch(lz.n, Se->nnz, Se->row_ptr, Se->col, bf.flags + 7, s);
    int vbad[9] = {};
    CSS_HIP_TRY(hipMemcpyAsync(vbad, bf.flags, 9 * sizeof(int), hipMemcpyDeviceToHost, s));
    CSS_HIP_TRY(hipStreamSynchronize(s));
    if (vbad[0] || vbad[4] || vbad[6] || vbad[8]) return CSS_E_CSR;
    const double* sv = static_cast<const double*>(Sih->val);

    // r~ = S^-1/2 r (FP64), then the Lanczos pass from it
    k_probe_block<<<grid_for(tall, 256), 256, 0, s>>>(color, sign, lz.n, lz.Np, lz.ld, bf.Y64);
    k_fill0<<<grid_for(tall, 256), 256, 0, s>>>(bf.Z1, tall);
    if (!spmm_launch<double>(SpmmArgs<double>{lz.n, Sih->row_ptr, Sih->col, sv, bf.Y64, bf.Z1, lz.ld}, s))
        return CSS_E_UNSUPPORTED;
    int v_eff = 0, brk = 0;
    double md = 0.0;
    CSS_TRY(run_lanczos_pass1(Hp, color, sign, lz, bf.lz, s, &v_eff, &brk, &md, bf.Z1, bf.R0));
    double ortho = NAN;
    if (flags & CSS_DIAG_ORTHO) CSS_TRY(lanczos_ortho_err(lz, bf.lz, v_eff, s, &ortho));
    CSS_HIP_TRY(hipEventRecord(ev[1], s));

    // rho^K = g f(T); F = g f(T) E_1 R0
    const int nT = v_eff * lz.b;
    const int64_t mat = (int64_t)lz.ld * lz.ld;
    int npoles = 0;
    fill_launch<int>(bf.flags, 0, 16, s);
    if (p.use_eig) {
        // by diagonalisation: F = U g f(Lambda) U[0:b,:]^T R0
        k_assemble_T<<<grid_for((int64_t)nT * nT, 256), 256, 0, s>>>(bf.lz.A, bf.lz.B, v_eff, lz.b, lz.ld, bf.T,
                                                                     bf.flags);
        int hbad = 0;
        CSS_HIP_TRY(hipMemcpyAsync(&hbad, bf.flags, sizeof(int), hipMemcpyDeviceToHost, s));
        CSS_HIP_TRY(hipStreamSynchronize(s));
        if (hbad) return CSS_E_NONFINITE;
        CSS_TRY(eig(bf.T, nT, bf.lam, bf.E, bf.flags + 1, bf.eig_ws, p.eig_ws, s));
        CSS_HIP_TRY(hipEventRecord(ev[2], s));
        k_occ_y_r0<<<grid_for((int64_t)nT * lz.b, 256), 256, 0, s>>>(bf.T, bf.lam, bf.R0, nT, lz.b, lz.ld, mu, kT,
                                                                      spin_deg, bf.Y);
        gemm_f64_launch(nT, lz.b, nT, bf.T, 1, nT, bf.Y, lz.b, 1, bf.F, lz.b, 1, s);
        k_quad_terms_r0<<<grid_for(nT, 256), 256, 0, s>>>(bf.T, bf.lam, bf.R0, nT, lz.b, lz.ld, mu, kT, spin_deg,
                                                          bf.t0, bf.t1);
        det_sum(bf.t0, nT, bf.tmp, bf.res + 2, s);
        det_sum(bf.t1, nT, bf.tmp + kSumBlocks, bf.res + 3, s);
    } else {
        // by the pole expansion with B_0 = I (F is linear in B_0), then F = F_I R0
        k_fill_ones<<<grid_for(lz.b, 256), 256, 0, s>>>(bf.ones, lz.b);
        CSS_TRY(subspace_fermi_poles(bf.lz.A, bf.lz.B, v_eff, lz.b, lz.ld, bf.ones, mu, kT, spin_deg, bf.Y,
                                     bf.res + 6, bf.pole_ws, p.pole_ws, &npoles, s));
        CSS_HIP_TRY(hipEventRecord(ev[2], s));
        gemm_f64_launch(nT, lz.b, lz.b, bf.Y, lz.b, 1, bf.R0, lz.ld, 1, bf.F, lz.b, 1, s);
        k_krylov_sums_r0<<<1, kR0SumThreads, 0, s>>>(bf.lz.A, bf.lz.B, bf.F, bf.R0, v_eff, lz.b, lz.ld, bf.res + 2);
    }
    k_pad_F<<<grid_for(v_eff * mat, 256), 256, 0, s>>>(bf.F, v_eff, lz.b, lz.ld, bf.Fpad);
    CSS_HIP_TRY(hipEventRecord(ev[3], s));

    // X' = sum_j Q_j F_j, then X = S^-1/2 X' (FP64)
    if (lz.fp32) {
        update_launch<float>(static_cast<float*>(bf.X), nullptr, 0.0, static_cast<const float*>(slot_ptr(lz, bf.lz, 0)),
                             tall, v_eff, bf.Fpad, mat, false, 1.0, lz.Np, lz.ld, bf.lz.stage, nullptr, s);
        k_widen<float><<<grid_for(tall, 256), 256, 0, s>>>(static_cast<const float*>(bf.X), bf.Y64, tall);
    } else {
        update_launch<double>(static_cast<double*>(bf.X), nullptr, 0.0,
                              static_cast<const double*>(slot_ptr(lz, bf.lz, 0)), tall, v_eff, bf.Fpad, mat, false,
                              1.0, lz.Np, lz.ld, bf.lz.stage, nullptr, s);
        CSS_HIP_TRY(hipMemcpyAsync(bf.Y64, bf.X, tall * sizeof(double), hipMemcpyDeviceToDevice, s));
    }
    if (!spmm_launch<double>(SpmmArgs<double>{lz.n, Sih->row_ptr, Sih->col, sv, bf.Y64, bf.Z, lz.ld}, s))
        return CSS_E_UNSUPPORTED;
    CSS_HIP_TRY(hipEventRecord(ev[4], s));

    // extraction with the probes r, the diagonal sum, H.P and S.P
    const int sym = (flags & CSS_SYMMETRIZE) ? 1 : 0;
    double* rt = bf.rows;
    double* ra = bf.rows + lz.n;
    double* re = bf.rows + 2 * (int64_t)lz.n;
    launch_gather<double>(lz.n, p_row_ptr, p_col, color, sign, bf.Z, lz.ld, sym, p_val, rt, ra, s);
    det_sum(rt, lz.n, bf.tmp + 2 * kSumBlocks, bf.res + 0, s);
    det_max(ra, lz.n, bf.tmp, bf.res + 4, s);
    for (int t = 0; t < 2; ++t) {
        const css_csr* M = t == 0 ? He : Se;
        if (!M) continue;
        if (M->val_dtype == CSS_F64)
            k_energy<double><<<grid_for(lz.n, 4), 256, 0, s>>>(lz.n, M->row_ptr, M->col,
                                                               static_cast<const double*>(M->val), p_row_ptr, p_col,
                                                               p_val, re);
        else
            k_energy<float><<<grid_for(lz.n, 4), 256, 0, s>>>(lz.n, M->row_ptr, M->col,
                                                              static_cast<const float*>(M->val), p_row_ptr, p_col,
                                                              p_val, re);
        det_sum(re, lz.n, bf.tmp + 3 * kSumBlocks, bf.res + (t == 0 ? 1 : 5), s);
    }
    CSS_HIP_TRY(hipEventRecord(ev[5], s));
    double hres[8] = {};
    int hinfo = 0;
    CSS_HIP_TRY(hipMemcpyAsync(hres, bf.res, 6 * sizeof(double), hipMemcpyDeviceToHost, s));
    CSS_HIP_TRY(hipMemcpyAsync(&hinfo, bf.flags + 1, sizeof(int), hipMemcpyDeviceToHost, s));
    CSS_HIP_TRY(hipStreamSynchronize(s));
    CSS_HIP_TRY(hipGetLastError());
    if (hinfo != 0) return CSS_E_EIG;
    *trace = hres[0];
    if (e_band) *e_band = hres[1];
    if (n_elec) *n_elec = hres[5];
    if (info) {
        *info = css_info{};
        info->depth_eff = v_eff;
        info->n_colors = lz.b;
        info->breakdown = brk;
        info->spmm_kernel = bf.lz.use_grp ? 1 : 0;
        info->min_diag_r = md;
        info->ortho_err = ortho;
        info->idem_defect = NAN;      // P S P = P is the non-orthogonal relation; not measured
        info->asym_max = hres[4];
        info->n_poles = npoles;
        info->trace_krylov = hres[2];
        info->e_band_krylov = hres[3];
        for (int k = 0; k < 5; ++k) {
            float ms = 0.f;
            if (hipEventElapsedTime(&ms, ev[k], ev[k + 1]) == hipSuccess) info->t_phase_ms[k] = ms;
        }
        float tot = 0.f;
        if (hipEventElapsedTime(&tot, ev[0], ev[5]) == hipSuccess) info->t_phase_ms[5] = tot;
    }
    return CSS_OK;
}

}  // namespace
}  // namespace css

extern "C" css_status css_density_matrix_nonorth(const css_csr* Hp, const css_csr* S_isqrt, const css_csr* H,
                                                 const css_csr* S, const int32_t* color, const int8_t* sign,
                                                 int32_t n_colors, double mu, double kT, int32_t depth,
                                                 double spin_deg, const int64_t* p_row_ptr, const int32_t* p_col,
                                                 int64_t p_nnz, uint32_t flags, double* p_val, double* e_band,
                                                 double* n_elec, double* trace, css_info* info, void* ws,
                                                 size_t ws_bytes, void* stream) {
    return css::nonorth_run(Hp, S_isqrt, H, S, color, sign, n_colors, mu, kT, depth, spin_deg, p_row_ptr, p_col,
                            p_nnz, flags, p_val, e_band, n_elec, trace, info, ws, ws_bytes, stream);
}

extern "C" css_status css_density_matrix(const css_csr* H, const int32_t* color, const int8_t* sign,
                                         int32_t n_colors, double mu, double kT, int32_t depth, double spin_deg,
                                         const int64_t* p_row_ptr, const int32_t* p_col, int64_t p_nnz,
                                         uint32_t flags, double* p_val, double* e_band, double* trace,
                                         css_info* info, void* ws, size_t ws_bytes, void* stream) {
    return css::dm_run(H, color, sign, n_colors, mu, kT, depth, spin_deg, p_row_ptr, p_col, p_nnz, flags, p_val,
                       nullptr, e_band, trace, nullptr, info, ws, ws_bytes, stream);
}

namespace css {
namespace {

// Scratch of css_density_matrix_noalloc: a file-scope device array, one copy on each
// GPU the library runs on, held until the process ends. Host code never uses the
// array's name as an address: each device's address comes from hipGetSymbolAddress
// on that device's first call and is kept per device.
constexpr size_t kNoAllocBytes = size_t(256) << 20;
constexpr int kNoAllocMinPoles = 64;
__device__ __align__(256) unsigned char scratch[kNoAllocBytes];
std::mutex g_scratch_mu;
void* g_scratch[64] = {};

css_status scratch_of_current_device(void** out) {
    int dev = 0;
    CSS_HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= 64) return CSS_E_DEVICE;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch[dev]) {
        void* ptr = nullptr;
        if (hipGetSymbolAddress((void**)&ptr, HIP_SYMBOL(scratch)) != hipSuccess || ptr == nullptr)
            return CSS_E_DEVICE;
        g_scratch[dev] = ptr;
    }
    *out = g_scratch[dev];
    return CSS_OK;
}

}  // namespace
}  // namespace css

extern "C" css_status css_density_matrix_noalloc(const css_csr* H, const int32_t* color, const int8_t* sign,
                                                 int32_t n_colors, double mu, double kT, int32_t depth,
                                                 double spin_deg, const int64_t* p_row_ptr, const int32_t* p_col,
                                                 int64_t p_nnz, uint32_t flags, double* p_val, double* e_band,
                                                 double* trace, css_info* info, void* stream) {
    if (flags & CSS_SUBSPACE_EIG) return CSS_E_UNSUPPORTED;        // rocSOLVER allocates its own memory
    DmPlan p;
    CSS_TRY(plan_dm(H, n_colors, depth, flags, p));
    if (p.use_eig) return CSS_E_UNSUPPORTED;                       // n_colors > 128: dense eigensolver
    // every buffer but the pole solver's, which takes the rest of the scratch: at least
    // kNoAllocMinPoles poles must fit (the solver itself fails with CSS_E_WORKSPACE if a
    // wider spectrum needs more than fit)
    p.pole_ws = 0;
    const size_t rest = dm_workspace_bytes(p) + 256;
    const size_t min_poles = pole_workspace_bytes(std::max(1, p.lz.v_max), n_colors, kNoAllocMinPoles);
    if (rest + min_poles > kNoAllocBytes) return CSS_E_WORKSPACE;
    void* ws = nullptr;
    CSS_TRY(scratch_of_current_device(&ws));
    return css::dm_run(H, color, sign, n_colors, mu, kT, depth, spin_deg, p_row_ptr, p_col, p_nnz, flags, p_val,
                       nullptr, e_band, trace, nullptr, info, ws, kNoAllocBytes, stream, kFnFermi, nullptr, nullptr,
                       false, kNoAllocBytes - rest);
}

extern "C" css_status css_energy_density_matrix(const css_csr* H, const int32_t* color, const int8_t* sign,
                                                int32_t n_colors, double mu, double kT, int32_t depth,
                                                double spin_deg, const int64_t* p_row_ptr, const int32_t* p_col,
                                                int64_t p_nnz, uint32_t flags, double* p_val, double* pe_val,
                                                double* e_band, double* trace, double* pe_trace, css_info* info,
                                                void* ws, size_t ws_bytes, void* stream) {
    if (!pe_val) return CSS_E_ARG;
    return css::dm_run(H, color, sign, n_colors, mu, kT, depth, spin_deg, p_row_ptr, p_col, p_nnz, flags, p_val,
                       pe_val, e_band, trace, pe_trace, info, ws, ws_bytes, stream);
}

extern "C" css_status css_inv_sqrt_overlap(const css_csr* S, const int32_t* color, const int8_t* sign,
                                           int32_t n_colors, int32_t depth, const int64_t* p_row_ptr,
                                           const int32_t* p_col, int64_t p_nnz, uint32_t flags, double* y_val,
                                           double* trace, double* s_dot, css_info* info, void* ws, size_t ws_bytes,
                                           void* stream) {
    if (!trace) return CSS_E_ARG;
    double sd = 0.0;
    CSS_TRY(css::dm_run(S, color, sign, n_colors, 0.0, 1.0, depth, 1.0, p_row_ptr, p_col, p_nnz, flags, y_val,
                        nullptr, &sd, trace, nullptr, info, ws, ws_bytes, stream, css::kFnInvSqrt));
    if (s_dot) *s_dot = sd;
    return CSS_OK;
}

extern "C" css_status css_transform_hamiltonian(const css_csr* H, const css_csr* S, const int32_t* color,
                                                const int8_t* sign, int32_t n_colors, int32_t depth,
                                                const int64_t* p_row_ptr, const int32_t* p_col, int64_t p_nnz,
                                                uint32_t flags, double* y_val, double* hp_val, double* y_trace,
                                                double* hp_trace, css_info* info, void* ws, size_t ws_bytes,
                                                void* stream) {
    if (!H || !hp_val || !y_trace) return CSS_E_ARG;
    double sd = 0.0, ht = 0.0;
    CSS_TRY(css::dm_run(S, color, sign, n_colors, 0.0, 1.0, depth, 1.0, p_row_ptr, p_col, p_nnz, flags, y_val,
                        nullptr, &sd, y_trace, &ht, info, ws, ws_bytes, stream, css::kFnInvSqrt, H, hp_val));
    if (hp_trace) *hp_trace = ht;
    return CSS_OK;
}

namespace css {
namespace {

// Root of c(mu) - n_e on [lo, hi], c(lo) = c_lo < n_e < c_hi = c(hi), by Chandrupatla's
// bracketing method (Adv. Eng. Software 28, 1997): the bracket [x1, x2] always
// holds the root, x1 the newest point and x3 the point last dropped; the next point
// is x1 + t (x2 - x1), with t from inverse quadratic interpolation through the
// three points where that interpolant is monotone on the bracket (xi = (x1 - x2) /
// (x3 - x2), phi = (f1 - f2) / (f3 - f2) satisfy phi^2 < xi and (1 - phi)^2 < 1 - xi),
// bisection (t = 1/2) otherwise, and t kept a tolerance away from the ends. Stops at
// a bracket of 2 xtol or a residual |c - n_e| <= ftol. eval(mu, &c) computes c(mu);
// *evals counts the calls.
template <typename Eval>
css_status bracket_root(Eval&& eval, double lo, double hi, double c_lo, double c_hi, double n_e, double xtol,
                        double ftol, double* root, double* c_root, int* evals) {
    double x1 = lo, f1 = c_lo - n_e, x2 = hi, f2 = c_hi - n_e, x3 = hi, f3 = f2;
    double t = 0.5;
    *evals = 0;
    for (int it = 0; it < 200; ++it) {
        const double xt = x1 + t * (x2 - x1);
        double ct = 0.0;
        CSS_TRY(eval(xt, &ct));
        ++*evals;
        const double ft = ct - n_e;
        if ((ft < 0.0) == (f1 < 0.0)) {             // the root lies between xt and x2
            x3 = x1;
            f3 = f1;
        } else {                                    // between x1 and xt
            x3 = x2;
            f3 = f2;
            x2 = x1;
            f2 = f1;
        }
        x1 = xt;
        f1 = ft;
        const bool one = std::fabs(f1) <= std::fabs(f2);
        const double xb = one ? x1 : x2, fb = one ? f1 : f2;
        if (std::fabs(fb) <= ftol || std::fabs(x2 - x1) <= 2.0 * xtol) {
            *root = xb;
            *c_root = fb + n_e;
            return CSS_OK;
        }
        const double tl = std::min(0.5, xtol / std::fabs(x2 - x1));
        const double xi = (x1 - x2) / (x3 - x2), phi = (f1 - f2) / (f3 - f2);
        if (phi * phi < xi && (1.0 - phi) * (1.0 - phi) < 1.0 - xi)
            t = f1 / (f2 - f1) * f3 / (f2 - f3) + (x3 - x1) / (x2 - x1) * f1 / (f3 - f1) * f2 / (f3 - f2);
        else
            t = 0.5;
        t = std::min(1.0 - tl, std::max(tl, t));
    }
    const bool one = std::fabs(f1) <= std::fabs(f2);
    *root = one ? x1 : x2;
    *c_root = (one ? f1 : f2) + n_e;
    return CSS_OK;
}

}  // namespace
}  // namespace css

extern "C" css_status css_find_mu(const css_csr* H, const int32_t* color, const int8_t* sign, int32_t n_colors,
                                  double n_electrons, double kT, int32_t depth, double spin_deg, uint32_t flags,
                                  double* mu, double* count, css_info* info, void* ws, size_t ws_bytes,
                                  void* stream) {
    if (!H || !color || !sign || !mu || !ws) return CSS_E_ARG;
    if (!(kT > 0.0) || !std::isfinite(kT) || !(spin_deg > 0.0) || !std::isfinite(spin_deg)) return CSS_E_ARG;
    if (!(n_electrons > 0.0) || !(n_electrons < spin_deg * (double)H->n)) return CSS_E_ARG;
    DmPlan p;
    CSS_TRY(plan_dm(H, n_colors, depth, flags, p));
    if (ws_bytes < dm_workspace_bytes(p)) return CSS_E_WORKSPACE;
    Arena a;
    a.base = static_cast<char*>(ws);
    a.cap = ws_bytes;
    DmBufs bf;
    carve_dm(a, p, bf);
    if (a.overflow) return CSS_E_WORKSPACE;
    hipStream_t s = as_stream(stream);
    const LzPlan& lz = p.lz;

    hipEvent_t ev[4] = {};
    for (auto& e : ev) CSS_HIP_TRY(hipEventCreate(&e));
    struct Guard {
        hipEvent_t* e;
        ~Guard() { for (int i = 0; i < 4; ++i) if (e[i]) (void)hipEventDestroy(e[i]); }
    } guard{ev};
    CSS_HIP_TRY(hipEventRecord(ev[0], s));
    int v_eff = 0, brk = 0;
    double md = 0.0;
    CSS_TRY(run_lanczos_pass1(H, color, sign, lz, bf.lz, s, &v_eff, &brk, &md));
    CSS_HIP_TRY(hipEventRecord(ev[1], s));

    const int nT = v_eff * lz.b;
    double hres[5] = {};
    int evals = 0;
    if (p.use_eig) {
        // eigenpairs of T, weights, bisection on the device
        fill_launch<int>(bf.flags, 0, 16, s);
        k_assemble_T<<<grid_for((int64_t)nT * nT, 256), 256, 0, s>>>(bf.lz.A, bf.lz.B, v_eff, lz.b, lz.ld, bf.T,
                                                                     bf.flags);
        int hbad = 0;
        CSS_HIP_TRY(hipMemcpyAsync(&hbad, bf.flags, sizeof(int), hipMemcpyDeviceToHost, s));
        CSS_HIP_TRY(hipStreamSynchronize(s));
        if (hbad) return CSS_E_NONFINITE;
        CSS_TRY(eig(bf.T, nT, bf.lam, bf.E, bf.flags + 1, bf.eig_ws, p.eig_ws, s));
        CSS_HIP_TRY(hipEventRecord(ev[2], s));
        k_quad_weights<<<grid_for(nT, 256), 256, 0, s>>>(bf.T, bf.lz.counts, nT, lz.b, bf.t0);
        k_mu_bisect<<<1, kMuThreads, 0, s>>>(bf.lam, bf.t0, nT, n_electrons, kT, spin_deg, 1e-13, bf.res);
        CSS_HIP_TRY(hipGetLastError());
        CSS_HIP_TRY(hipEventRecord(ev[3], s));
        int hinfo = 0;
        CSS_HIP_TRY(hipMemcpyAsync(hres, bf.res, 5 * sizeof(double), hipMemcpyDeviceToHost, s));
        CSS_HIP_TRY(hipMemcpyAsync(&hinfo, bf.flags + 1, sizeof(int), hipMemcpyDeviceToHost, s));
        CSS_HIP_TRY(hipStreamSynchronize(s));
        if (hinfo != 0) return CSS_E_EIG;
        evals = (int)hres[2];
    } else {
        // the count at each trial mu from the pole expansion (the Krylov trace of
        // css_density_matrix), root by Chandrupatla's bracketing method on the
        // Gershgorin bracket widened by 50 kT, where the count is 0 and g N to within
        // g N e^-50
        double glo = 0.0, ghi = 0.0;
        CSS_TRY(subspace_spectral_bounds(bf.lz.A, bf.lz.B, v_eff, lz.b, lz.ld, bf.pole_ws, p.pole_ws, &glo, &ghi, s));
        CSS_HIP_TRY(hipEventRecord(ev[2], s));
        auto eval = [&](double m, double* out) -> css_status {
            int np = 0;
            CSS_TRY(subspace_fermi_poles(bf.lz.A, bf.lz.B, v_eff, lz.b, lz.ld, bf.lz.counts, m, kT, spin_deg, bf.F,
                                         bf.res + 6, bf.pole_ws, p.pole_ws, &np, s));
            double h = 0.0;
            CSS_HIP_TRY(hipMemcpyAsync(&h, bf.res + 6, sizeof(double), hipMemcpyDeviceToHost, s));
            CSS_HIP_TRY(hipStreamSynchronize(s));
            if (!std::isfinite(h)) return CSS_E_NONFINITE;
            *out = h;
            return CSS_OK;
        };
        const double lo = glo - 50.0 * kT, hi = ghi + 50.0 * kT;
        const double xtol = 1e-13 * std::max(1.0, std::max(std::fabs(lo), std::fabs(hi)));
        CSS_TRY(bracket_root(eval, lo, hi, 0.0, spin_deg * (double)lz.n, n_electrons, xtol, 1e-12 * n_electrons,
                           &hres[0], &hres[1], &evals));
        CSS_HIP_TRY(hipEventRecord(ev[3], s));
        CSS_HIP_TRY(hipStreamSynchronize(s));
    }
    if (!std::isfinite(hres[0]) || !std::isfinite(hres[1])) return CSS_E_NONFINITE;
    *mu = hres[0];
    if (count) *count = hres[1];
    if (info) {
        *info = css_info{};
        info->depth_eff = v_eff;
        info->n_colors = lz.b;
        info->breakdown = brk;
        info->spmm_kernel = bf.lz.use_grp ? 1 : 0;
        info->n_evals = evals;
        info->min_diag_r = md;
        info->ortho_err = NAN;
        info->idem_defect = NAN;
        info->trace_krylov = hres[1];
        for (int k = 0; k < 3; ++k) {
            float ms = 0.f;
            if (hipEventElapsedTime(&ms, ev[k], ev[k + 1]) == hipSuccess) info->t_phase_ms[k] = ms;
        }
        float tot = 0.f;
        if (hipEventElapsedTime(&tot, ev[0], ev[3]) == hipSuccess) info->t_phase_ms[5] = tot;
    }
    return CSS_OK;
}

extern "C" css_status css_workspace_size(int32_t entry, int32_t n, int64_t nnz, int32_t n_colors, int32_t depth,
                                         uint32_t flags, size_t* bytes) {
    if (!bytes || n < 1) return CSS_E_ARG;
    if (entry == CSS_ENTRY_COLOR) {
        *bytes = color_workspace_bytes(n);
        return CSS_OK;
    }
    if (entry == CSS_ENTRY_SPMM) {
        if (nnz < 0 || nnz >= (int64_t(1) << 31)) return CSS_E_ARG;
        *bytes = spmm_workspace_bytes(n, nnz);
        return CSS_OK;
    }
    if (entry != CSS_ENTRY_LANCZOS && entry != CSS_ENTRY_DENSITY && entry != CSS_ENTRY_ENERGY_DENSITY &&
        entry != CSS_ENTRY_FIND_MU && entry != CSS_ENTRY_INV_SQRT && entry != CSS_ENTRY_TRANSFORM_H &&
        entry != CSS_ENTRY_DENSITY_NONORTH)
        return CSS_E_ARG;
    // shape-only CSRs for planning; H's value type is not an argument, so the size
    // covers both (values in the other precision need a converted copy)
    size_t most = 0;
    for (const int vt : {CSS_F32, CSS_F64}) {
        css_csr H{n, nnz, reinterpret_cast<const int32_t*>(1), reinterpret_cast<const int32_t*>(1),
                  reinterpret_cast<const void*>(1), vt};
        if (entry == CSS_ENTRY_LANCZOS) {
            LzPlan p;
            CSS_TRY(plan_lanczos(&H, n_colors, depth, flags, p));
            most = std::max(most, lanczos_workspace_bytes(p));
        } else {
            DmPlan p;
            const bool eig = entry == CSS_ENTRY_INV_SQRT || entry == CSS_ENTRY_TRANSFORM_H ||
                             (entry == CSS_ENTRY_FIND_MU && n_colors > 128);
            CSS_TRY(plan_dm(&H, n_colors, depth, eig ? (flags | CSS_SUBSPACE_EIG) : flags, p));
            p.energy = entry == CSS_ENTRY_ENERGY_DENSITY;
            p.hprime = entry == CSS_ENTRY_TRANSFORM_H;
            p.nonorth = entry == CSS_ENTRY_DENSITY_NONORTH;
            p.ns = (entry == CSS_ENTRY_INV_SQRT || entry == CSS_ENTRY_TRANSFORM_H) && !(flags & CSS_SUBSPACE_EIG);
            most = std::max(most, dm_workspace_bytes(p));
        }
    }
    *bytes = most;
    return CSS_OK;
}

extern "C" int32_t css_block_ld(int32_t n_colors) { return n_colors > 0 ? block_ld(n_colors) : 0; }

extern "C" const char* css_status_string(css_status s) {
    switch (s) {
        case CSS_OK: return "ok";
        case CSS_E_ARG: return "invalid argument";
        case CSS_E_CSR: return "malformed CSR matrix or colouring";
        case CSS_E_WORKSPACE: return "workspace too small";
        case CSS_E_DEVICE: return "HIP runtime or library error";
        case CSS_E_BREAKDOWN_AT_1: return "the first Krylov block is degenerate";
        case CSS_E_NONFINITE: return "non-finite value in H or in the projected matrix";
        case CSS_E_EIG: return "subspace eigensolver failed";
        case CSS_E_UNSUPPORTED: return "option or size not supported";
        case CSS_E_CAPACITY: return "output array too small";
        default: return "unknown status";
    }
}
