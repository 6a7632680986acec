// Fermi-Dirac operator inside the Krylov subspace by a pole expansion of Eq.(7).
//
// Eq.(7) writes rho^K as a contour integral of f(z) times the resolvent
// (z - H^K)^-1. Only F = g f(T) E_1 B_0 (T = H^K, block tridiagonal with v
// blocks of b) is needed. This file evaluates it as a finite sum of
// resolvents instead of diagonalising T:
//
//   f(x) = (1 - tanh(y))/2,  y = (x - mu)/(2 kT),
//   tanh(y) ~ sum_p c_p y / (1 + kappa_p^2 y^2)      (truncated Lambert continued fraction)
//
// The truncation at depth M equals y [(D + i y E)^-1]_11 with D = diag(1,3,5,..)
// and E the tridiagonal of ones; with K = D^-1/2 E D^-1/2 = W diag(kappa) W^T
// the poles are y = +-i/kappa_p and c_p = 2 W[0,p]^2 (kappa_p > 0). Each term
// is  Y (I + kappa^2 Y^2)^-1 = Im[(I - i kappa Y)^-1] / kappa, so with Y = (T - mu)/(2kT)
//
//   F = g [ E_1 B_0 / 2 - sum_p (c_p / (2 kappa_p)) Im Z_p ],
//   (I - i kappa_p Y) Z_p = E_1 B_0.
//
// I - i kappa Y has all singular values >= 1 and positive definite Hermitian
// part, so its block elimination needs no pivoting and is well conditioned.
// Each Z_p comes from Schur complements taken from the last block upward,
//   S_v = D_v,  S_j = D_j - U_j S_{j+1}^-1 L_{j+1},  G_j = S_j^-1 L_j,
//   Z_1 = S_1^-1 R_1,  Z_{j+1} = -G_{j+1} Z_j,
// with D_j = I - i a (A_j - mu), L_{j+1} = -i a B_j, U_j = -i a B_j^T, a = kappa/(2kT).
// The truncation depth is chosen from a Gershgorin bound of T so that the
// rational approximation error stays near double-precision rounding.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <map>
#include <mutex>
#include <vector>

#include "css_common.h"
#include "mfma_util.h"
#include "subspace.h"

namespace css {
namespace {

// ------------------------------------------------------------------ host: pole table

// Eigenpairs of a small symmetric tridiagonal matrix T (diagonal d, off-diagonal e,
// e[i] coupling i and i + 1): the eigenvalues ascending and the first component of
// each unit eigenvector (all the pole table needs).
//
// Eigenvalues by bisection on the Sturm count: the number of eigenvalues of T below
// x equals the number of negative pivots q_i of the LDL^T factorisation of T - x I,
// q_0 = d_0 - x, q_i = d_i - x - e_{i-1}^2 / q_{i-1} (Sylvester's law of inertia).
// Each eigenvalue is bisected inside the Gershgorin interval to a width of a few
// ulps. First components by inverse iteration: solve (T - lambda I) y = x twice from
// x = (1, ..., 1), by Gaussian elimination with row interchanges on the band, and
// normalise.
int sturm_count(const std::vector<double>& d, const std::vector<double>& e, double x) {
    const int n = static_cast<int>(d.size());
    int neg = 0;
    double q = 1.0;
    for (int i = 0; i < n; ++i) {
        const double off = i > 0 ? e[i - 1] * e[i - 1] / q : 0.0;
        q = d[i] - x - off;
        if (q == 0.0) q = -1e-300;          // a zero pivot counts as negative, nudged off zero
        if (q < 0.0) ++neg;
    }
    return neg;
}

// y := (T - lambda I)^-1 y for tridiagonal T (n >= 1), partial pivoting; zero pivots
// (lambda exactly an eigenvalue) are replaced by a tiny value, as inverse iteration allows.
void shifted_solve(const std::vector<double>& d, const std::vector<double>& e, double lambda, std::vector<double>& y) {
    const int n = static_cast<int>(d.size());
    // row i holds u0[i] (diagonal), u1[i], u2[i] (first, second superdiagonal)
    std::vector<double> u0(n), u1(n, 0.0), u2(n, 0.0), lo(n, 0.0);
    for (int i = 0; i < n; ++i) {
        u0[i] = d[i] - lambda;
        if (i + 1 < n) u1[i] = e[i];
    }
    std::vector<double> sub(n, 0.0);                 // subdiagonal entry below each diagonal
    for (int i = 0; i + 1 < n; ++i) sub[i] = e[i];
    const double tiny = 1e-300;
    for (int i = 0; i + 1 < n; ++i) {
        // rows i and i + 1: columns i .. i + 2
        if (std::fabs(sub[i]) > std::fabs(u0[i])) {
            // interchange: row i + 1 becomes the pivot row
            const double r0 = sub[i], r1 = u0[i + 1], r2 = (i + 1 < n - 1) ? u1[i + 1] : 0.0;
            const double s0 = u0[i], s1 = u1[i], s2 = u2[i];
            u0[i] = r0; u1[i] = r1; u2[i] = r2;
            std::swap(y[i], y[i + 1]);
            const double m = s0 / r0;
            lo[i] = m;
            u0[i + 1] = s1 - m * r1;
            if (i + 1 < n - 1) u1[i + 1] = s2 - m * r2;
            y[i + 1] -= m * y[i];
        } else {
            const double piv = u0[i] != 0.0 ? u0[i] : tiny;
            u0[i] = piv;
            const double m = sub[i] / piv;
            lo[i] = m;
            u0[i + 1] -= m * u1[i];
            if (i + 1 < n - 1) u1[i + 1] -= m * u2[i];
            y[i + 1] -= m * y[i];
        }
    }
    if (u0[n - 1] == 0.0) u0[n - 1] = tiny;
    for (int i = n - 1; i >= 0; --i) {
        double acc = y[i];
        if (i + 1 < n) acc -= u1[i] * y[i + 1];
        if (i + 2 < n) acc -= u2[i] * y[i + 2];
        y[i] = acc / u0[i];
    }
}

void tridiag_eig_first_row(std::vector<double>& d, std::vector<double> e, std::vector<double>& z) {
    const int n = static_cast<int>(d.size());
    const std::vector<double> diag = d;
    double glo = INFINITY, ghi = -INFINITY;
    for (int i = 0; i < n; ++i) {
        const double r = (i > 0 ? std::fabs(e[i - 1]) : 0.0) + (i + 1 < n ? std::fabs(e[i]) : 0.0);
        glo = std::min(glo, diag[i] - r);
        ghi = std::max(ghi, diag[i] + r);
    }
    z.assign(n, 0.0);
    for (int k = 0; k < n; ++k) {
        double a = glo, b = ghi;                     // count(a) <= k < count(b)
        for (int it = 0; it < 200; ++it) {
            const double mid = 0.5 * (a + b);
            if (mid <= a || mid >= b) break;         // no double between a and b
            if (sturm_count(diag, e, mid) > k) b = mid; else a = mid;
        }
        const double lambda = 0.5 * (a + b);
        std::vector<double> y(n, 1.0);
        for (int it = 0; it < 3; ++it) {
            shifted_solve(diag, e, lambda, y);
            double nrm = 0.0;
            for (double v : y) nrm = std::max(nrm, std::fabs(v));
            for (double& v : y) v /= nrm;
        }
        double s2 = 0.0;
        for (double v : y) s2 += v * v;
        d[k] = lambda;
        z[k] = y[0] / std::sqrt(s2);
    }
}

struct PoleTable {
    std::vector<double> kappa, weight;   // weight = c_p / (2 kappa_p)
};

std::mutex g_pole_mu;
std::map<int, PoleTable> g_poles;

const PoleTable& pole_table(int M) {
    std::lock_guard<std::mutex> lock(g_pole_mu);
    auto it = g_poles.find(M);
    if (it != g_poles.end()) return it->second;
    std::vector<double> d(M, 0.0), e(M - 1), z;
    for (int k = 0; k + 1 < M; ++k) e[k] = 1.0 / std::sqrt((2.0 * k + 1.0) * (2.0 * k + 3.0));
    tridiag_eig_first_row(d, e, z);
    PoleTable t;
    for (int p = 0; p < M; ++p)
        if (d[p] > 1e-12) {
            t.kappa.push_back(d[p]);
            t.weight.push_back(2.0 * z[p] * z[p] / (2.0 * d[p]));
        }
    return g_poles.emplace(M, std::move(t)).first->second;
}

// Truncation depth for |y| <= ymax. The depth the fraction needs for an error of
// 1e-14 grows like 6 sqrt(ymax) (measured: 28 levels at |y| = 20, 58 at 100, 102 at
// 320); four more poles bring the error to at most 9e-16 for |y| from 0.5 to 6000
// (measured on a grid of 60 values), below the rounding of the rest of the path.
int depth_for(double ymax) {
    const double y = std::min(1e6, std::max(0.0, ymax));
    const int M = static_cast<int>(std::ceil(6.0 * std::sqrt(y))) + 8;
    return std::max(16, (M + 1) / 2 * 2);
}
constexpr int kMaxDepth = 512;       // at most 256 poles (|y| up to about 6800)

// ------------------------------------------------------------------ device

// Gershgorin interval of T, one wavefront per row: lo[row], hi[row].
__global__ __launch_bounds__(256) void k_gersh(const double* __restrict__ A, const double* __restrict__ B, int v, int b,
                                               int ld, double* __restrict__ lo, double* __restrict__ hi) {
    const int lane = threadIdx.x & 63;
    const int row = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (row >= v * b) return;
    const int j = row / b, r = row % b;
    const int64_t mat = (int64_t)ld * ld;
    double rad = 0.0;
    for (int c = lane; c < b; c += 64) {
        if (c != r) rad += fabs(A[j * mat + (int64_t)r * ld + c]);
        if (j > 0) rad += fabs(B[(j - 1) * mat + (int64_t)r * ld + c]);
        if (j + 1 < v) rad += fabs(B[j * mat + (int64_t)c * ld + r]);
    }
    for (int off = 32; off > 0; off >>= 1) rad += __shfl_xor(rad, off);
    if (lane == 0) {
        const double dg = A[j * mat + (int64_t)r * ld + r];
        lo[row] = dg - rad;
        hi[row] = dg + rad;
    }
}

__global__ void k_minmax(const double* __restrict__ lo, const double* __restrict__ hi, int n, double* __restrict__ out) {
    __shared__ double smin[256], smax[256];
    double a = INFINITY, z = -INFINITY;
    for (int i = threadIdx.x; i < n; i += 256) {
        a = fmin(a, lo[i]);
        z = fmax(z, hi[i]);
    }
    smin[threadIdx.x] = a;
    smax[threadIdx.x] = z;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s) {
            smin[threadIdx.x] = fmin(smin[threadIdx.x], smin[threadIdx.x + s]);
            smax[threadIdx.x] = fmax(smax[threadIdx.x], smax[threadIdx.x + s]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) { out[0] = smin[0]; out[1] = smax[0]; }
}

constexpr int kPoleThreads = 1024;
constexpr int kPoleWaves = kPoleThreads / 64;

typedef double pd4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ pd4 mfma64(double a, double b, pd4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// One workgroup per pole: backward Schur sweep with in-place Gauss-Jordan inversion
// of each complex b x b Schur complement (no pivoting), then the forward sweep.
// The b x b products run on FP64 MFMA 16x16x4 tiles, one tile at a time per wave
// (lane l supplies A[l%16][l/16], B[l/16][l%16]; result r of lane l is D[l/16+4r][l%16]).
// Writes W_p = weight_p * Im Z_p (nT x b, row-major) for pole p = blockIdx.x.
__global__ __launch_bounds__(kPoleThreads) void k_pole_solve_generic(const double* __restrict__ A, const double* __restrict__ B,
                                                             int v, int b, int ld, double mu, double inv2kT,
                                                             const double* __restrict__ kappa,
                                                             const double* __restrict__ weight,
                                                             const int* __restrict__ counts, double* Gbuf,
                                                             double* Sglob, int use_lds, double* __restrict__ Wout) {
    extern __shared__ double lds[];
    __shared__ double colr[128], coli[128], pinv[2];
    const int p = blockIdx.x;
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6, lr = lane >> 4, lc = lane & 15;
    const int bb = b * b;
    const int nt = (b + 15) / 16;          // output tiles per dimension
    const int ntiles = nt * nt;
    const int64_t mat = (int64_t)ld * ld;
    const double a = kappa[p] * inv2kT;
    const double wgt = weight[p];
    double* Sr = use_lds ? lds : Sglob + (int64_t)p * 2 * bb;
    double* Si = Sr + bb;
    double* Gp = Gbuf + (int64_t)p * v * 2 * bb;          // G_j at Gp + j*2bb (Re, then Im)
    double* Wp = Wout + (int64_t)p * v * bb;
    const int per = (bb + kPoleThreads - 1) / kPoleThreads;

    for (int j = v - 1; j >= 0; --j) {
        // S = I - i a (A_j - mu) + i a B_j^T G_{j+1}: tile products into registers, then LDS
        const double* Aj = A + j * mat;
        const double* Bj = B + j * mat;
        const double* Gr1 = Gp + (int64_t)(j + 1) * 2 * bb;
        const double* Gi1 = Gr1 + bb;
        for (int t = wave; t < ntiles; t += kPoleWaves) {
            const int m0 = (t / nt) * 16, c0 = (t % nt) * 16;
            pd4 tr = {0, 0, 0, 0}, ti = {0, 0, 0, 0};
            if (j + 1 < v) {
                const int mr = m0 + lc, cc = c0 + lc;
                for (int k0 = 0; k0 < b; k0 += 4) {
                    const int k = k0 + lr;
                    const bool kv = k < b;
                    const double av = (kv && mr < b) ? Bj[(int64_t)k * ld + mr] : 0.0;     // (B_j^T)[m][k]
                    const double gr = (kv && cc < b) ? Gr1[k * b + cc] : 0.0;
                    const double gi = (kv && cc < b) ? Gi1[k * b + cc] : 0.0;
                    tr = mfma64(av, gr, tr);
                    ti = mfma64(av, gi, ti);
                }
            }
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = m0 + lr + 4 * r, col = c0 + lc;
                if (row < b && col < b) {
                    const double dg = (row == col) ? 1.0 : 0.0;
                    Sr[row * b + col] = dg - a * ti[r];
                    Si[row * b + col] = -a * (Aj[(int64_t)row * ld + col] - (row == col ? mu : 0.0)) + a * tr[r];
                }
            }
        }
        __syncthreads();
        // Gauss-Jordan inverse in place
        for (int k = 0; k < b; ++k) {
            if (tid == 0) {
                const double xr = Sr[k * b + k], xi = Si[k * b + k];
                const double den = 1.0 / (xr * xr + xi * xi);
                pinv[0] = xr * den;
                pinv[1] = -xi * den;
            }
            if (tid < b) {
                colr[tid] = Sr[tid * b + k];
                coli[tid] = Si[tid * b + k];
            }
            __syncthreads();
            const double qr = pinv[0], qi = pinv[1];
            for (int c = tid; c < b; c += kPoleThreads) {
                const double xr = (c == k) ? 1.0 : Sr[k * b + c], xi = (c == k) ? 0.0 : Si[k * b + c];
                Sr[k * b + c] = xr * qr - xi * qi;
                Si[k * b + c] = xr * qi + xi * qr;
            }
            __syncthreads();
            for (int q = 0; q < per; ++q) {
                const int e = tid + kPoleThreads * q;
                if (e >= bb) break;
                const int r = e / b, c = e % b;
                if (r == k) continue;
                const double fr = colr[r], fi = coli[r];
                const double xr = (c == k) ? 0.0 : Sr[e], xi = (c == k) ? 0.0 : Si[e];
                const double pr = Sr[k * b + c], pi = Si[k * b + c];
                Sr[e] = xr - (fr * pr - fi * pi);
                Si[e] = xi - (fr * pi + fi * pr);
            }
            __syncthreads();
        }
        if (j > 0) {
            // G_j = S^-1 L_j = -i a S^-1 B_{j-1}
            const double* Bm = B + (j - 1) * mat;
            double* Gr = Gp + (int64_t)j * 2 * bb;
            double* Gi = Gr + bb;
            for (int t = wave; t < ntiles; t += kPoleWaves) {
                const int m0 = (t / nt) * 16, c0 = (t % nt) * 16;
                const int mr = m0 + lc, cc = c0 + lc;
                pd4 tr = {0, 0, 0, 0}, ti = {0, 0, 0, 0};
                for (int k0 = 0; k0 < b; k0 += 4) {
                    const int k = k0 + lr;
                    const bool kv = k < b;
                    const double sr = (kv && mr < b) ? Sr[mr * b + k] : 0.0;
                    const double si = (kv && mr < b) ? Si[mr * b + k] : 0.0;
                    const double bv = (kv && cc < b) ? Bm[(int64_t)k * ld + cc] : 0.0;
                    tr = mfma64(sr, bv, tr);
                    ti = mfma64(si, bv, ti);
                }
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int row = m0 + lr + 4 * r, col = c0 + lc;
                    if (row < b && col < b) {
                        Gr[row * b + col] = a * ti[r];
                        Gi[row * b + col] = -a * tr[r];
                    }
                }
            }
            __syncthreads();
        }
    }
    // forward sweep: Z_1 = S_1^-1 B_0 (column scaling by sqrt(n_c)), Z_{j+1} = -G_{j+1} Z_j
    for (int q = 0; q < per; ++q) {
        const int e = tid + kPoleThreads * q;
        if (e >= bb) break;
        const double sc = sqrt((double)counts[e % b]);
        Sr[e] *= sc;
        Si[e] *= sc;
        Wp[e] = wgt * Si[e];
    }
    __syncthreads();
    constexpr int kMaxTilesPerWave = 4;    // (128/16)^2 / 16 waves
    for (int j = 1; j < v; ++j) {
        const double* Gr = Gp + (int64_t)j * 2 * bb;
        const double* Gi = Gr + bb;
        pd4 nr[kMaxTilesPerWave], ni[kMaxTilesPerWave];
        int q = 0;
        for (int t = wave; t < ntiles; t += kPoleWaves, ++q) {
            const int m0 = (t / nt) * 16, c0 = (t % nt) * 16;
            const int mr = m0 + lc, cc = c0 + lc;
            pd4 re = {0, 0, 0, 0}, im = {0, 0, 0, 0};
            for (int k0 = 0; k0 < b; k0 += 4) {
                const int k = k0 + lr;
                const bool kv = k < b;
                const double gr = (kv && mr < b) ? Gr[mr * b + k] : 0.0;
                const double gi = (kv && mr < b) ? Gi[mr * b + k] : 0.0;
                const double zr = (kv && cc < b) ? Sr[k * b + cc] : 0.0;
                const double zi = (kv && cc < b) ? Si[k * b + cc] : 0.0;
                re = mfma64(gr, zr, re);
                re = mfma64(-gi, zi, re);
                im = mfma64(gr, zi, im);
                im = mfma64(gi, zr, im);
            }
            nr[q] = re;
            ni[q] = im;
        }
        __syncthreads();
        q = 0;
        for (int t = wave; t < ntiles; t += kPoleWaves, ++q) {
            const int m0 = (t / nt) * 16, c0 = (t % nt) * 16;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = m0 + lr + 4 * r, col = c0 + lc;
                if (row < b && col < b) {
                    Sr[row * b + col] = -nr[q][r];
                    Si[row * b + col] = -ni[q][r];
                    Wp[(int64_t)j * bb + row * b + col] = -wgt * ni[q][r];
                }
            }
        }
        __syncthreads();
    }
}

// Register-tiled Gauss-Jordan inverse (no pivoting) of the complex b x b matrix
// (Sr, Si) in LDS, b <= 96: thread (ty, tx) of a 32 x 32 grid keeps entries
// (ty + 32a, tx + 32c); the pivot row and column are broadcast through
// double-buffered LDS vectors, one barrier per pivot.
__device__ void gj_inverse_reg(double* Sr, double* Si, int b, double (*vec)[4][96]) {
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
    double xr[3][3], xi[3][3];
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const int i = ty + 32 * a, j = tx + 32 * c;
            const bool in = i < b && j < b;
            xr[a][c] = in ? Sr[i * b + j] : 0.0;
            xi[a][c] = in ? Si[i * b + j] : 0.0;
        }
    __syncthreads();
    for (int k = 0; k < b; ++k) {
        double(*v)[96] = vec[k & 1];      // [0] col re, [1] col im, [2] row re, [3] row im
        const int kb = k >> 5, kt = k & 31;
        if (tx == kt) {
#pragma unroll
            for (int c = 0; c < 3; ++c)
                if (c == kb) {
#pragma unroll
                    for (int a = 0; a < 3; ++a) {
                        const int i = ty + 32 * a;
                        if (i < b) { v[0][i] = xr[a][c]; v[1][i] = xi[a][c]; }
                    }
                }
        }
        if (ty == kt) {
#pragma unroll
            for (int a = 0; a < 3; ++a)
                if (a == kb) {
#pragma unroll
                    for (int c = 0; c < 3; ++c) {
                        const int j = tx + 32 * c;
                        if (j < b) { v[2][j] = xr[a][c]; v[3][j] = xi[a][c]; }
                    }
                }
        }
        __syncthreads();
        const double pr = v[2][k], pi = v[3][k];
        const double den = 1.0 / (pr * pr + pi * pi);
        const double qr = pr * den, qi = -pi * den;              // 1 / pivot
        double rr[3], ri[3], cr[3], ci[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const int j = tx + 32 * c;
            const double mr = j < b ? v[2][j] : 0.0, mi = j < b ? v[3][j] : 0.0;
            rr[c] = mr * qr - mi * qi;                          // pivot row / pivot
            ri[c] = mr * qi + mi * qr;
        }
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const int i = ty + 32 * a;
            cr[a] = i < b ? v[0][i] : 0.0;
            ci[a] = i < b ? v[1][i] : 0.0;
        }
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const int i = ty + 32 * a;
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const int j = tx + 32 * c;
                double nr, ni;
                if (i == k) {
                    nr = (j == k) ? qr : rr[c];
                    ni = (j == k) ? qi : ri[c];
                } else if (j == k) {
                    nr = -(cr[a] * qr - ci[a] * qi);
                    ni = -(cr[a] * qi + ci[a] * qr);
                } else {
                    nr = xr[a][c] - (cr[a] * rr[c] - ci[a] * ri[c]);
                    ni = xi[a][c] - (cr[a] * ri[c] + ci[a] * rr[c]);
                }
                xr[a][c] = nr;
                xi[a][c] = ni;
            }
        }
    }
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const int i = ty + 32 * a, j = tx + 32 * c;
            if (i < b && j < b) { Sr[i * b + j] = xr[a][c]; Si[i * b + j] = xi[a][c]; }
        }
    __syncthreads();
}

// b <= 96: one workgroup per pole with the Schur complement in LDS.
//   S_{v-1} = D_{v-1};  for j = v-1 .. 0:  S_j <- S_j^-1 (Gauss-Jordan);
//   G_j = -i a S_j^-1 B_{j-1} (kept in global for the forward sweep and staged in LDS);
//   S_{j-1} = D_{j-1} + i a B_{j-1}^T G_j.
// Forward: Z_0 = S_0^-1 B_0, Z_j = -G_j Z_{j-1}; W_p rows j*b.. = weight_p Im Z_j.
constexpr int kMaxTiles96 = 3;     // (96/16)^2 tiles over 16 waves

__global__ __launch_bounds__(kPoleThreads) void k_pole_solve(const double* __restrict__ A, const double* __restrict__ B,
                                                             int v, int b, int ld, double mu, double inv2kT,
                                                             const double* __restrict__ kappa,
                                                             const double* __restrict__ weight,
                                                             const int* __restrict__ counts, double* Gbuf,
                                                             double* __restrict__ Wout) {
    extern __shared__ double lds[];
    __shared__ double vec[2][4][96];
    const int p = blockIdx.x;
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6, lr = lane >> 4, lc = lane & 15;
    const int bb = b * b;
    const int nt = (b + 15) / 16;
    const int ntiles = nt * nt;
    const int64_t mat = (int64_t)ld * ld;
    const double a = kappa[p] * inv2kT;
    const double wgt = weight[p];
    double* Sr = lds;
    double* Si = lds + bb;
    double* Gp = Gbuf + (int64_t)p * v * 2 * bb;
    double* Wp = Wout + (int64_t)p * v * bb;

    // S_{v-1} = I - i a (A_{v-1} - mu)
    {
        const double* Aj = A + (v - 1) * mat;
        for (int e = tid; e < bb; e += kPoleThreads) {
            const int r = e / b, c = e % b;
            Sr[e] = (r == c) ? 1.0 : 0.0;
            Si[e] = -a * (Aj[(int64_t)r * ld + c] - (r == c ? mu : 0.0));
        }
    }
    __syncthreads();
    for (int j = v - 1; j >= 0; --j) {
        gj_inverse_reg(Sr, Si, b, vec);
        if (j == 0) break;
        // G_j = -i a S^-1 B_{j-1}: A operand S^-1 (LDS), B operand B_{j-1} (global); tiles go
        // straight to global (S^-1 is not overwritten before the barrier)
        const double* Bm = B + (j - 1) * mat;
        double* Gr = Gp + (int64_t)j * 2 * bb;
        double* Gi = Gr + bb;
        for (int t = wave; t < ntiles; t += kPoleWaves) {
            const int m0 = (t / nt) * 16, c0 = (t % nt) * 16;
            const int mr = m0 + lc, cc = c0 + lc;
            pd4 tr = {0, 0, 0, 0}, ti = {0, 0, 0, 0};
            for (int k0 = 0; k0 < b; k0 += 4) {
                const int k = k0 + lr;
                const bool kv = k < b;
                const double sr = (kv && mr < b) ? Sr[mr * b + k] : 0.0;
                const double si = (kv && mr < b) ? Si[mr * b + k] : 0.0;
                const double bv = (kv && cc < b) ? Bm[(int64_t)k * ld + cc] : 0.0;
                tr = mfma64(sr, bv, tr);
                ti = mfma64(si, bv, ti);
            }
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = m0 + lr + 4 * r, col = c0 + lc;
                if (row < b && col < b) {
                    Gr[row * b + col] = a * ti[r];      // Re(-i a (tr + i ti)) = a ti
                    Gi[row * b + col] = -a * tr[r];     // Im = -a tr
                }
            }
        }
        __syncthreads();
        // S_{j-1} = I - i a (A_{j-1} - mu) + i a B_{j-1}^T G_j: operands B_{j-1}^T and G_j (global);
        // the result overwrites the LDS matrix directly
        const double* Aj = A + (j - 1) * mat;
        for (int t = wave; t < ntiles; t += kPoleWaves) {
            const int m0 = (t / nt) * 16, c0 = (t % nt) * 16;
            const int mr = m0 + lc, cc = c0 + lc;
            pd4 tr = {0, 0, 0, 0}, ti = {0, 0, 0, 0};
            for (int k0 = 0; k0 < b; k0 += 4) {
                const int k = k0 + lr;
                const bool kv = k < b;
                const double av = (kv && mr < b) ? Bm[(int64_t)k * ld + mr] : 0.0;
                const double zr = (kv && cc < b) ? Gr[k * b + cc] : 0.0;
                const double zi = (kv && cc < b) ? Gi[k * b + cc] : 0.0;
                tr = mfma64(av, zr, tr);
                ti = mfma64(av, zi, ti);
            }
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = m0 + lr + 4 * r, col = c0 + lc;
                if (row < b && col < b) {
                    const double dg = (row == col) ? 1.0 : 0.0;
                    Sr[row * b + col] = dg - a * ti[r];
                    Si[row * b + col] = -a * (Aj[(int64_t)row * ld + col] - (row == col ? mu : 0.0)) + a * tr[r];
                }
            }
        }
        __syncthreads();
    }
    // forward sweep
    for (int e = tid; e < bb; e += kPoleThreads) {
        const double sc = sqrt((double)counts[e % b]);
        Sr[e] *= sc;
        Si[e] *= sc;
        Wp[e] = wgt * Si[e];
    }
    __syncthreads();
    for (int j = 1; j < v; ++j) {
        const double* Gr = Gp + (int64_t)j * 2 * bb;
        const double* Gi = Gr + bb;
        pd4 nr[kMaxTiles96], ni[kMaxTiles96];
#pragma unroll
        for (int q = 0; q < kMaxTiles96; ++q) {
            const int t = wave + kPoleWaves * q;
            nr[q] = pd4{0, 0, 0, 0};
            ni[q] = pd4{0, 0, 0, 0};
            if (t >= ntiles) continue;
            const int m0 = (t / nt) * 16, c0 = (t % nt) * 16;
            const int mr = m0 + lc, cc = c0 + lc;
            pd4 re = {0, 0, 0, 0}, im = {0, 0, 0, 0};
            for (int k0 = 0; k0 < b; k0 += 4) {
                const int k = k0 + lr;
                const bool kv = k < b;
                const double g_r = (kv && mr < b) ? Gr[mr * b + k] : 0.0;
                const double g_i = (kv && mr < b) ? Gi[mr * b + k] : 0.0;
                const double zr = (kv && cc < b) ? Sr[k * b + cc] : 0.0;
                const double zi = (kv && cc < b) ? Si[k * b + cc] : 0.0;
                re = mfma64(g_r, zr, re);
                re = mfma64(-g_i, zi, re);
                im = mfma64(g_r, zi, im);
                im = mfma64(g_i, zr, im);
            }
            nr[q] = re;
            ni[q] = im;
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < kMaxTiles96; ++q) {
            const int t = wave + kPoleWaves * q;
            if (t >= ntiles) continue;
            const int m0 = (t / nt) * 16, c0 = (t % nt) * 16;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = m0 + lr + 4 * r, col = c0 + lc;
                if (row < b && col < b) {
                    Sr[row * b + col] = -nr[q][r];
                    Si[row * b + col] = -ni[q][r];
                    Wp[(int64_t)j * bb + row * b + col] = -wgt * ni[q][r];
                }
            }
        }
        __syncthreads();
    }
}

// b <= 96, blocks of 16 (N = 16 NB rows, padded with the identity beyond b):
// one workgroup per pole, the complex Schur complement S (N x N, row stride
// N + 1) in LDS. Each S_j (complex symmetric) is inverted in place by block
// Gauss-Jordan without pivoting: wave 0 inverts the 16 x 16 diagonal block
// P = S_kk^-1 in registers, the row block (S_kj <- P S_kj) is computed on FP64 MFMA
// and the column block written as its signed transpose, the upper trailing blocks
// are updated on FP64 MFMA and mirrored, two barriers per block step, with the next
// pivot inverted during the trailing update (gj_inverse_blk). The next Schur
// complement is symmetric too and computed on its upper tiles. G_j (N x N, global)
// and the forward sweep are as in k_pole_solve_generic.
constexpr int kBlkThreads = 512;     // 8 waves: at most 256 registers per lane (199 used, no spills)
constexpr int kBlkWaves = kBlkThreads / 64;

// Wave 0: the 16 x 16 diagonal block at (o, o) of S inverted in registers (Gauss-Jordan
// without pivoting, MFMA D layout: lane l holds rows (l>>4)+4r, column l&15) into Pr/Pi
// (row stride 17). Step k needs the pivot (readlane), the pivot row in every row group
// (grp_bcast) and the pivot column in every lane of each row (col_bcast): VALU moves
// only. The step is one formula for every element, branch-free: with m = 0 in the pivot
// column and 1 elsewhere, and t_j = x_kj / p (j != k), t_k = 1 / p,
//   x_ij <- m_j x_ij - x_ik t_j   (rows i != k; gives -x_ik / p in the pivot column),
// and the pivot row is then replaced by t.
template <int NB>
__device__ __forceinline__ void pivot_inverse(const double* Sr, const double* Si, int o, double* Pr, double* Pi) {
    constexpr int SW = 16 * NB + 1;
    const int lane = threadIdx.x & 63, lr = lane >> 4, lc = lane & 15;
    double xr[4], xi[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        xr[r] = Sr[(o + lr + 4 * r) * SW + o + lc];
        xi[r] = Si[(o + lr + 4 * r) * SW + o + lc];
    }
    static_steps([&](auto kc) {
        constexpr int k = decltype(kc)::value, rk = k >> 2, g = k & 3;
        const bool pc = lc == k;                                          // pivot column
        const double pr = lane_read(xr[rk], 16 * g + k), pi = lane_read(xi[rk], 16 * g + k);
        const double den = recip_newton(pr * pr + pi * pi);
        const double qr = pr * den, qi = -pi * den;                       // 1 / pivot
        const double mr = grp_bcast<g>(xr[rk]), mi = grp_bcast<g>(xi[rk]);
        const double tr = pc ? qr : mr * qr - mi * qi;                    // t = pivot row / pivot
        const double ti = pc ? qi : mr * qi + mi * qr;
        const double m = pc ? 0.0 : 1.0;
        double cr[4], ci[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) {                                     // column k, my rows
            cr[r] = col_bcast<k>(xr[r]);
            ci[r] = col_bcast<k>(xi[r]);
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const double nr = __builtin_fma(xr[r], m, __builtin_fma(ci[r], ti, -cr[r] * tr));
            const double ni = __builtin_fma(xi[r], m, -__builtin_fma(cr[r], ti, ci[r] * tr));
            xr[r] = nr;
            xi[r] = ni;
        }
        const bool prow = lr == g;                                        // row k
        xr[rk] = prow ? tr : xr[rk];
        xi[rk] = prow ? ti : xi[rk];
    }, std::make_integer_sequence<int, 16>{});
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        Pr[(lr + 4 * r) * 17 + lc] = xr[r];
        Pi[(lr + 4 * r) * 17 + lc] = xi[r];
    }
}

// Trailing update of one tile with the new column block C (column kb) and the old
// row block (row kb): S_ij += C_ik S_kj (complex, FP64 MFMA). With mirror, the tile's
// transpose times sgn also goes to (jb, ib).
template <int NB>
__device__ __forceinline__ void trailing_tile(double* Sr, double* Si, int ib, int jb, int kb, bool mirror, double sgn) {
    constexpr int SW = 16 * NB + 1;
    const int lane = threadIdx.x & 63, lr = lane >> 4, lc = lane & 15;
    const int o = 16 * kb;
    pd4 cr, ci;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        cr[r] = Sr[(16 * ib + lr + 4 * r) * SW + 16 * jb + lc];
        ci[r] = Si[(16 * ib + lr + 4 * r) * SW + 16 * jb + lc];
    }
#pragma unroll
    for (int s4 = 0; s4 < 4; ++s4) {
        const int k = o + 4 * s4 + lr;
        const double ar = Sr[(16 * ib + lc) * SW + k], ai = Si[(16 * ib + lc) * SW + k];
        const double br = Sr[k * SW + 16 * jb + lc], bi = Si[k * SW + 16 * jb + lc];
        cr = mfma64(ar, br, cr);
        cr = mfma64(-ai, bi, cr);
        ci = mfma64(ar, bi, ci);
        ci = mfma64(ai, br, ci);
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        Sr[(16 * ib + lr + 4 * r) * SW + 16 * jb + lc] = cr[r];
        Si[(16 * ib + lr + 4 * r) * SW + 16 * jb + lc] = ci[r];
    }
    if (mirror) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            Sr[(16 * jb + lc) * SW + 16 * ib + lr + 4 * r] = sgn * cr[r];
            Si[(16 * jb + lc) * SW + 16 * ib + lr + 4 * r] = sgn * ci[r];
        }
    }
}

// S (16 NB x 16 NB complex symmetric, in LDS) replaced by its inverse, block
// Gauss-Jordan without pivoting. After the pivots K = {0 .. k-1} the matrix is
// [[A_KK^-1, A_KK^-1 A_KU], [-A_UK A_KK^-1, Schur complement]]: symmetric within K x K
// and U x U and antisymmetric between them (M_UK = -M_KU^T). Block step k therefore
// needs only the row block R_kj = P S_kj (P = S_kk^-1, symmetric): the column block
// -S_ik P equals -R_ki^T for i > k and R_ki^T for i < k. The trailing update
// S_ij += C_ik S_kj (old row block) is computed for i <= j and mirrored with that sign
// rule. P holds two pivot inverses (re/im, 16 x 17 each; P + 2*272 q for buffer q).
// Per block step: waves 0 .. NB-2 compute the row tiles into registers and write the
// column block; barrier; wave 0 updates the next diagonal tile and inverts it into the
// other buffer (look-ahead) while waves 1 .. 7 update the other upper trailing tiles;
// barrier; the row tiles go to row k at the start of the next step (the tile in
// column k+1 is superseded there by the next column block) with S_kk <- P.
template <int NB>
__device__ void gj_inverse_blk(double* Sr, double* Si, double* P) {
    constexpr int SW = 16 * NB + 1, PB = 2 * 16 * 17;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, lr = lane >> 4, lc = lane & 15;
    if (wave == 0) pivot_inverse<NB>(Sr, Si, 0, P, P + 16 * 17);
    __syncthreads();
    pd4 hr = {0, 0, 0, 0}, hi = {0, 0, 0, 0};             // this wave's row tile of the previous step
    int hj = -1;                                          // its block column (-1: none)
    auto put_row = [&](int kprev, int skip) {             // row tiles and P of block step kprev
        const int op = 16 * kprev;
        if (hj >= 0 && hj != skip) {
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                Sr[(op + lr + 4 * r) * SW + 16 * hj + lc] = hr[r];
                Si[(op + lr + 4 * r) * SW + 16 * hj + lc] = hi[r];
            }
        }
        if (wave == kBlkWaves - 1) {
            const double* Qr = P + (kprev & 1) * PB;
            const double* Qi = Qr + 16 * 17;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                Sr[(op + lr + 4 * r) * SW + op + lc] = Qr[(lr + 4 * r) * 17 + lc];
                Si[(op + lr + 4 * r) * SW + op + lc] = Qi[(lr + 4 * r) * 17 + lc];
            }
        }
    };
    for (int kb = 0; kb < NB; ++kb) {
        const int o = 16 * kb;
        const double* Pr = P + (kb & 1) * PB;
        const double* Pi = Pr + 16 * 17;
        if (kb > 0) put_row(kb - 1, kb);
        hj = -1;
        if (wave < NB - 1) {                                  // row block R_kj = P S_kj
            const int jb = wave < kb ? wave : wave + 1;
            pd4 cr = {0, 0, 0, 0}, ci = {0, 0, 0, 0};
#pragma unroll
            for (int s4 = 0; s4 < 4; ++s4) {
                const int k = 4 * s4 + lr;
                const double ar = Pr[lc * 17 + k], ai = Pi[lc * 17 + k];
                const double br = Sr[(o + k) * SW + 16 * jb + lc], bi = Si[(o + k) * SW + 16 * jb + lc];
                cr = mfma64(ar, br, cr);
                cr = mfma64(-ai, bi, cr);
                ci = mfma64(ar, bi, ci);
                ci = mfma64(ai, br, ci);
            }
            const double sg = jb < kb ? 1.0 : -1.0;           // column block C_jk = sg R_kj^T
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                Sr[(16 * jb + lc) * SW + o + lr + 4 * r] = sg * cr[r];
                Si[(16 * jb + lc) * SW + o + lr + 4 * r] = sg * ci[r];
            }
            hr = cr;
            hi = ci;
            hj = jb;
        }
        __syncthreads();
        if constexpr (NB > 1) {
            const int k1 = kb + 1;
            const bool ahead = k1 < NB;                        // a next pivot exists
            if (ahead && wave == 0) {
                trailing_tile<NB>(Sr, Si, k1, k1, kb, false, 1.0);
                __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");   // the tile's LDS writes before its reads
                double* Qr = P + (k1 & 1) * PB;
                pivot_inverse<NB>(Sr, Si, 16 * k1, Qr, Qr + 16 * 17);
            } else {
                // the upper trailing tiles i <= j (i, j != kb), mirrored: all of them to every
                // wave in the last block step, all but (k1, k1) to waves 1.. before it
                const int w0 = ahead ? wave - 1 : wave, nw = ahead ? kBlkWaves - 1 : kBlkWaves;
                constexpr int NU = (NB - 1) * NB / 2;
                for (int t = w0; t < NU; t += nw) {
                    int ib = 0, rem = t;                        // t-th pair i <= j of 0 .. NB-2
                    while (rem >= NB - 1 - ib) { rem -= NB - 1 - ib; ++ib; }
                    int jb = ib + rem;
                    ib += ib >= kb;
                    jb += jb >= kb;
                    if (ahead && ib == k1 && jb == k1) continue;
                    trailing_tile<NB>(Sr, Si, ib, jb, kb, ib != jb, (ib < kb) == (jb < kb) ? 1.0 : -1.0);
                }
            }
        }
        __syncthreads();
    }
    put_row(NB - 1, -1);
    __syncthreads();
}

template <int NB>
__global__ __launch_bounds__(kBlkThreads) void k_pole_solve_blk(const double* __restrict__ A,
                                                                 const double* __restrict__ B, int v, int b, int ld,
                                                                 double mu, double inv2kT,
                                                                 const double* __restrict__ kappa,
                                                                 const double* __restrict__ weight,
                                                                 const int* __restrict__ counts, double* Gbuf,
                                                                 double* __restrict__ Wout) {
    constexpr int N = 16 * NB, SW = N + 1, NTL = NB * NB;
    constexpr int MAXQ = (NTL + kBlkWaves - 1) / kBlkWaves;
    extern __shared__ double lds[];
    double* Sr = lds;
    double* Si = lds + N * SW;
    double* P = lds + 2 * N * SW;          // two 16 x 17 complex pivot inverses
    const int p = blockIdx.x, tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6, lr = lane >> 4, lc = lane & 15;
    const int64_t mat = (int64_t)ld * ld, nn = (int64_t)N * N;
    const double a = kappa[p] * inv2kT;
    const double wgt = weight[p];
    double* Gp = Gbuf + (int64_t)p * v * 2 * nn;
    double* Wp = Wout + (int64_t)p * v * b * b;
    // S = D_{v-1} = I - i a (A_{v-1} - mu) on the leading b x b block, identity beyond
    {
        const double* Aj = A + (int64_t)(v - 1) * mat;
        for (int e = tid; e < N * N; e += kBlkThreads) {
            const int r = e / N, c = e % N;
            Sr[r * SW + c] = (r == c) ? 1.0 : 0.0;
            Si[r * SW + c] = (r < b && c < b) ? -a * (Aj[(int64_t)r * ld + c] - (r == c ? mu : 0.0)) : 0.0;
        }
    }
    __syncthreads();
    for (int j = v - 1; j >= 0; --j) {
        int zoff = 0;                                          // as in the forward sweep below
        asm volatile("" : "+v"(zoff));
        double* Sr = lds + zoff;
        double* Si = lds + zoff + N * SW;
        gj_inverse_blk<NB>(Sr, Si, P);
        if (j == 0) break;
        // G_j = -i a S_j^-1 B_{j-1} (B zero beyond b). B_{j-1} is upper triangular
        // (a Cholesky factor, or the product of two): column c has no entries below row
        // c, so tile column c0 needs the chunks of k < c0 + 16 only.
        const double* Bm = B + (int64_t)(j - 1) * mat;
        double* Gr = Gp + (int64_t)j * 2 * nn;
        double* Gi = Gr + nn;
        for (int t = wave; t < NTL; t += kBlkWaves) {
            const int m0 = (t / NB) * 16, c0 = (t % NB) * 16;
            pd4 tr2[2] = {{0, 0, 0, 0}, {0, 0, 0, 0}}, ti2[2] = {{0, 0, 0, 0}, {0, 0, 0, 0}};   // even / odd K steps
            constexpr int H = 8, NH = (N / 4 + H - 1) / H;      // K in chunks of 8 steps of global operands
            const int hmax = (c0 + 16 + 4 * H - 1) / (4 * H);
#pragma unroll
            for (int h = 0; h < NH; ++h) {
                if (h >= hmax) break;
                double bv[H];
#pragma unroll
                for (int q = 0; q < H; ++q) {
                    const int s4 = h * H + q;
                    bv[q] = s4 < N / 4 ? Bm[(int64_t)(4 * s4 + lr) * ld + c0 + lc] : 0.0;
                }
#pragma unroll
                for (int q = 0; q < H; ++q) {
                    const int s4 = h * H + q;
                    if (s4 >= N / 4) break;
                    const int k = 4 * s4 + lr;
                    tr2[q & 1] = mfma64(Sr[(m0 + lc) * SW + k], bv[q], tr2[q & 1]);
                    ti2[q & 1] = mfma64(Si[(m0 + lc) * SW + k], bv[q], ti2[q & 1]);
                }
                __builtin_amdgcn_sched_barrier(0);             // one chunk of operands live at a time
            }
            const pd4 tr = tr2[0] + tr2[1], ti = ti2[0] + ti2[1];
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = m0 + lr + 4 * r, col = c0 + lc;
                Gr[row * N + col] = a * ti[r];        // Re(-i a (tr + i ti)) = a ti
                Gi[row * N + col] = -a * tr[r];       // Im = -a tr
            }
        }
        __syncthreads();
        // S_{j-1} = I - i a (A_{j-1} - mu) + i a B_{j-1}^T G_j, complex symmetric
        // (B^T G_j = -i a B^T S_j^-1 B): the upper tiles m0 <= c0 only, each mirrored. Row
        // m of B^T has no entries beyond column m, so tile row m0 needs the chunks of
        // k < m0 + 16 only; the tiles are dealt from the last tile row up (costliest first).
        const double* Aj = A + (int64_t)(j - 1) * mat;
        constexpr int NU = NB * (NB + 1) / 2;
        for (int t = wave; t < NU; t += kBlkWaves) {
            int mb = NB - 1, rem = t;                          // tile rows NB-1, NB-2, ..: NB - mb tiles each
            while (rem >= NB - mb) { rem -= NB - mb; --mb; }
            const int m0 = 16 * mb, c0 = 16 * (mb + rem);
            pd4 tr2[2] = {{0, 0, 0, 0}, {0, 0, 0, 0}}, ti2[2] = {{0, 0, 0, 0}, {0, 0, 0, 0}};   // even / odd K steps
            constexpr int H = 8, NH = (N / 4 + H - 1) / H;      // K in chunks of 8 steps of global operands
            const int hmax = (m0 + 16 + 4 * H - 1) / (4 * H);
#pragma unroll
            for (int h = 0; h < NH; ++h) {
                if (h >= hmax) break;
                double av[H], zr[H], zi[H];
#pragma unroll
                for (int q = 0; q < H; ++q) {
                    const int s4 = h * H + q;
                    const int k = 4 * s4 + lr;
                    const bool in = s4 < N / 4;
                    av[q] = in ? Bm[(int64_t)k * ld + m0 + lc] : 0.0;
                    zr[q] = in ? Gr[k * N + c0 + lc] : 0.0;
                    zi[q] = in ? Gi[k * N + c0 + lc] : 0.0;
                }
#pragma unroll
                for (int q = 0; q < H; ++q) {
                    tr2[q & 1] = mfma64(av[q], zr[q], tr2[q & 1]);
                    ti2[q & 1] = mfma64(av[q], zi[q], ti2[q & 1]);
                }
                __builtin_amdgcn_sched_barrier(0);
            }
            const pd4 tr = tr2[0] + tr2[1], ti = ti2[0] + ti2[1];
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = m0 + lr + 4 * r, col = c0 + lc;
                const double am = (row < b && col < b) ? Aj[(int64_t)row * ld + col] - (row == col ? mu : 0.0) : 0.0;
                const double vr = (row == col ? 1.0 : 0.0) - a * ti[r], vi = -a * am + a * tr[r];
                Sr[row * SW + col] = vr;
                Si[row * SW + col] = vi;
                if (m0 != c0) {
                    Sr[col * SW + row] = vr;
                    Si[col * SW + row] = vi;
                }
            }
        }
        __syncthreads();
    }
    // Z_0 = S_0^-1 diag(sqrt(n_c)) into slot 0 of G (no G_0 exists) and W_p block 0 =
    // weight_p Im Z_0; the forward sweep Z_j = -G_j Z_{j-1} is k_pole_forward
    double* Zr0 = Gp;
    double* Zi0 = Gp + nn;
    for (int e = tid; e < N * N; e += kBlkThreads) {
        const int r = e / N, c = e % N;
        const double sc = c < b ? sqrt((double)counts[c]) : 0.0;
        const double zr = Sr[r * SW + c] * sc, zi = Si[r * SW + c] * sc;
        Zr0[e] = zr;
        Zi0[e] = zi;
        if (r < b && c < b) Wp[r * b + c] = wgt * zi;
    }
}

// Forward sweep of the block solve: Z_j = -G_j Z_{j-1}, W_p block j = weight_p Im Z_j,
// for j = 1 .. v-1. The columns of Z are independent, so workgroup (p, slab) follows
// the 16 CT columns 16 CT slab .. of pole p on its own: the slab of Z_{j-1} is in LDS
// (double buffered, one barrier per step), wave w computes rows 16 w .. +15 of Z_j
// (CT column tiles, so that each G_j row read serves CT tiles) with the rows of G_j
// (complex, global) of the next step already in flight.
template <int NB, int CT>
__global__ __launch_bounds__(64 * NB) void k_pole_forward(int v, int b, const double* __restrict__ weight,
                                                          const double* __restrict__ Gbuf,
                                                          double* __restrict__ Wout) {
    constexpr int N = 16 * NB, KS = N / 4, SC = 16 * CT;
    __shared__ double zb[2][2][N * SC];                   // [buffer][re, im][k * SC + column]
    const int p = blockIdx.x, c0 = SC * blockIdx.y;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, lr = lane >> 4, lc = lane & 15;
    const int64_t nn = (int64_t)N * N;
    const double wgt = weight[p];
    const double* Gp = Gbuf + (int64_t)p * v * 2 * nn;
    double* Wp = Wout + (int64_t)p * v * b * b;
    for (int e = threadIdx.x; e < N * SC; e += 64 * NB) {
        const int k = e / SC, c = e % SC;
        zb[0][0][e] = Gp[(int64_t)k * N + c0 + c];
        zb[0][1][e] = Gp[nn + (int64_t)k * N + c0 + c];
    }
    __syncthreads();
    const int m0 = 16 * wave;
    auto load_g = [&](int j, double (&g)[2][KS]) {
        const double* Gr = Gp + (int64_t)min(j, v - 1) * 2 * nn + (int64_t)(m0 + lc) * N + lr;
#pragma unroll
        for (int s4 = 0; s4 < KS; ++s4) {
            g[0][s4] = Gr[4 * s4];
            g[1][s4] = Gr[nn + 4 * s4];
        }
    };
    auto step = [&](int j, const double (&g)[2][KS]) {
        const int cur = (j - 1) & 1;
        // even and odd K steps in separate accumulators (four independent MFMA chains
        // per column tile), added at the end
        pd4 nr[CT][2], ni[CT][2];
#pragma unroll
        for (int t = 0; t < CT; ++t) nr[t][0] = nr[t][1] = ni[t][0] = ni[t][1] = pd4{0, 0, 0, 0};
#pragma unroll
        for (int s4 = 0; s4 < KS; ++s4) {
            const int k = 4 * s4 + lr, h = s4 & 1;
#pragma unroll
            for (int t = 0; t < CT; ++t) {
                const double zr = zb[cur][0][k * SC + 16 * t + lc], zi = zb[cur][1][k * SC + 16 * t + lc];
                nr[t][h] = mfma64(g[0][s4], zr, nr[t][h]);
                nr[t][h] = mfma64(-g[1][s4], zi, nr[t][h]);
                ni[t][h] = mfma64(g[0][s4], zi, ni[t][h]);
                ni[t][h] = mfma64(g[1][s4], zr, ni[t][h]);
            }
        }
        pd4 nrs[CT], nis[CT];
#pragma unroll
        for (int t = 0; t < CT; ++t) {
            nrs[t] = nr[t][0] + nr[t][1];
            nis[t] = ni[t][0] + ni[t][1];
        }
#pragma unroll
        for (int t = 0; t < CT; ++t)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = m0 + lr + 4 * r, col = c0 + 16 * t + lc;
                zb[cur ^ 1][0][row * SC + 16 * t + lc] = -nrs[t][r];
                zb[cur ^ 1][1][row * SC + 16 * t + lc] = -nis[t][r];
                if (row < b && col < b) Wp[(int64_t)j * b * b + row * b + col] = -wgt * nis[t][r];
            }
        lds_barrier();                                    // Z_j complete; Z_{j-1} no longer read
    };
    double ga[2][KS], gb[2][KS];
    load_g(1, ga);
    for (int j = 1; j < v; j += 2) {
        load_g(j + 1, gb);                                // clamped: the last step again at the end
        step(j, ga);
        if (j + 1 >= v) break;
        load_g(j + 2, ga);
        step(j + 1, gb);
    }
}

size_t pole_blk_lds_bytes(int nb) { return sizeof(double) * (2 * (size_t)16 * nb * (16 * nb + 1) + 4 * 16 * 17); }

// F = g (E_1 B_0 / 2 - sum_p W_p), poles summed in order.
__global__ void k_pole_sum(const double* __restrict__ Wout, int npole, int64_t nTb, int b,
                           const int* __restrict__ counts, double g, double* __restrict__ F) {
    const int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (idx >= nTb) return;
    double s = 0.0;
    for (int p = 0; p < npole; ++p) s += Wout[(int64_t)p * nTb + idx];
    const int64_t row = idx / b;
    const int c = (int)(idx % b);
    const double e1b0 = (row == c) ? sqrt((double)counts[c]) : 0.0;
    F[idx] = g * (0.5 * e1b0 - s);
}

// trace_K = sum_c sqrt(n_c) F[c][c];  E_K = sum_c sqrt(n_c) (A_1 F_1 + B_1^T F_2)[c][c].
// One work-group of kKsThreads: a wavefront per colour c (lanes over k), then a
// fixed tree over the colours. b <= kKsMaxB.
constexpr int kKsThreads = 1024;
constexpr int kKsMaxB = 128;

__global__ __launch_bounds__(kKsThreads) void k_krylov_sums(const double* __restrict__ A, const double* __restrict__ B,
                                                            const double* __restrict__ F,
                                                            const int* __restrict__ counts, int v, int b, int ld,
                                                            double* __restrict__ out) {
    __shared__ double st[kKsMaxB], se[kKsMaxB];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    for (int c = threadIdx.x; c < kKsMaxB; c += kKsThreads) st[c] = se[c] = 0.0;
    __syncthreads();
    for (int c = w; c < b; c += kKsThreads / 64) {
        double tf = 0.0;
        for (int k = lane; k < b; k += 64) {
            tf += A[(int64_t)c * ld + k] * F[(int64_t)k * b + c];
            if (v > 1) tf += B[(int64_t)k * ld + c] * F[(int64_t)(b + k) * b + c];
        }
        for (int off = 32; off > 0; off >>= 1) tf += __shfl_xor(tf, off);
        if (lane == 0) {
            const double sc = sqrt((double)counts[c]);
            st[c] = sc * F[(int64_t)c * b + c];
            se[c] = sc * tf;
        }
    }
    __syncthreads();
    for (int h = kKsMaxB / 2; h > 0; h >>= 1) {
        if (threadIdx.x < h) {
            st[threadIdx.x] += st[threadIdx.x + h];
            se[threadIdx.x] += se[threadIdx.x + h];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) { out[0] = st[0]; out[1] = se[0]; }
}

int max_lds() {
    static std::atomic<int> cached{-1};        // same value from any thread
    int c = cached.load(std::memory_order_relaxed);
    if (c < 0) {
        int dev = 0, val = 65536;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&val, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess)
            val = 65536;
        cached.store(val, std::memory_order_relaxed);
        c = val;
    }
    return c;
}

}  // namespace

size_t pole_workspace_bytes(int v, int b, int max_poles) {
    const int64_t np = max_poles > 0 ? max_poles : kMaxDepth / 2 + 1;
    const int64_t bb = (int64_t)b * b;
    const int64_t n16 = 16 * (int64_t)((b + 15) / 16);
    const int64_t gmat = std::max(bb, n16 * n16);          // G blocks (padded for the blocked solver)
    return sizeof(double) * (size_t)(np * (v * 2 * gmat + v * bb + 2 * bb) + 2 * np + 2 * (int64_t)v * b + 16) + 4096;
}

css_status subspace_fermi_poles(const double* A, const double* B, int v, int b, int ld, const int* counts,
                                double mu, double kT, double g, double* F, double* sums, void* ws, size_t ws_bytes,
                                int* npoles_out, hipStream_t s) {
    if (b > 128) return CSS_E_UNSUPPORTED;
    const int nT = v * b;
    const int64_t bb = (int64_t)b * b;
    Arena ar;
    ar.base = static_cast<char*>(ws);
    ar.cap = ws_bytes;
    double* glo = ar.take<double>(nT);
    double* ghi = ar.take<double>(nT);
    double* range = ar.take<double>(16);
    k_gersh<<<grid_for(nT, 4), 256, 0, s>>>(A, B, v, b, ld, glo, ghi);
    k_minmax<<<1, 256, 0, s>>>(glo, ghi, nT, range);
    double hr[2];
    CSS_HIP_TRY(hipMemcpyAsync(hr, range, sizeof(hr), hipMemcpyDeviceToHost, s));
    CSS_HIP_TRY(hipStreamSynchronize(s));
    if (!std::isfinite(hr[0]) || !std::isfinite(hr[1])) return CSS_E_NONFINITE;
    const double ymax = std::max(std::fabs(hr[0] - mu), std::fabs(hr[1] - mu)) / (2.0 * kT);
    const int M = depth_for(ymax);
    if (M > kMaxDepth) return CSS_E_UNSUPPORTED;       // spectrum too wide for kT: more than 256 poles
    const PoleTable& pt = pole_table(M);
    const int np = static_cast<int>(pt.kappa.size());
    double* kap = ar.take<double>(np);
    double* wgt = ar.take<double>(np);
    const int nb16 = (b + 15) / 16;
    const int64_t gmat = std::max<int64_t>(bb, (int64_t)256 * nb16 * nb16);
    double* Gbuf = ar.take<double>((int64_t)np * v * 2 * gmat);
    double* Wout = ar.take<double>((int64_t)np * v * bb);
    const size_t lds_bytes = sizeof(double) * 2 * bb;
    const bool use_lds = lds_bytes + 8192 <= (size_t)max_lds();
    double* Sg = use_lds ? nullptr : ar.take<double>((int64_t)np * 2 * bb);
    if (ar.overflow) return CSS_E_WORKSPACE;
    CSS_HIP_TRY(hipMemcpyAsync(kap, pt.kappa.data(), sizeof(double) * np, hipMemcpyHostToDevice, s));
    CSS_HIP_TRY(hipMemcpyAsync(wgt, pt.weight.data(), sizeof(double) * np, hipMemcpyHostToDevice, s));
    const size_t blk_lds = pole_blk_lds_bytes(nb16);
    const bool used_blk = b <= 96 && ld == 16 * nb16 && blk_lds <= (size_t)max_lds();
    if (used_blk) {
        switch (nb16) {
#define CSS_POLE(NB)                                                                                              \
    case NB:                                                                                                      \
        k_pole_solve_blk<NB><<<np, kBlkThreads, blk_lds, s>>>(A, B, v, b, ld, mu, 1.0 / (2.0 * kT), kap, wgt,    \
                                                               counts, Gbuf, Wout);                               \
        break;
            CSS_POLE(1) CSS_POLE(2) CSS_POLE(3) CSS_POLE(4) CSS_POLE(5) CSS_POLE(6)
#undef CSS_POLE
            default: return CSS_E_UNSUPPORTED;
        }
    } else if (b <= 96 && use_lds)
        k_pole_solve<<<np, kPoleThreads, lds_bytes, s>>>(A, B, v, b, ld, mu, 1.0 / (2.0 * kT), kap, wgt, counts, Gbuf,
                                                         Wout);
    else
        k_pole_solve_generic<<<np, kPoleThreads, use_lds ? lds_bytes : 0, s>>>(A, B, v, b, ld, mu, 1.0 / (2.0 * kT),
                                                                                kap, wgt, counts, Gbuf, Sg,
                                                                                use_lds ? 1 : 0, Wout);
    if (used_blk && v > 1) {
        switch (nb16) {
#define CSS_FWD(NB, CT) \
    case NB: k_pole_forward<NB, CT><<<dim3(np, NB / CT), 64 * NB, 0, s>>>(v, b, wgt, Gbuf, Wout); break;
            CSS_FWD(1, 1) CSS_FWD(2, 2) CSS_FWD(3, 1) CSS_FWD(4, 2) CSS_FWD(5, 1) CSS_FWD(6, 1)
#undef CSS_FWD
            default: break;
        }
    }
    k_pole_sum<<<grid_for((int64_t)nT * b, 256), 256, 0, s>>>(Wout, np, (int64_t)nT * b, b, counts, g, F);
    k_krylov_sums<<<1, kKsThreads, 0, s>>>(A, B, F, counts, v, b, ld, sums);     // b <= 128 checked above
    if (npoles_out) *npoles_out = np;
    CSS_HIP_TRY(hipGetLastError());
    return CSS_OK;
}

css_status subspace_spectral_bounds(const double* A, const double* B, int v, int b, int ld, void* ws, size_t ws_bytes,
                                    double* lo, double* hi, hipStream_t s) {
    const int nT = v * b;
    Arena ar;
    ar.base = static_cast<char*>(ws);
    ar.cap = ws_bytes;
    double* glo = ar.take<double>(nT);
    double* ghi = ar.take<double>(nT);
    double* range = ar.take<double>(16);
    if (ar.overflow) return CSS_E_WORKSPACE;
    k_gersh<<<grid_for(nT, 4), 256, 0, s>>>(A, B, v, b, ld, glo, ghi);
    k_minmax<<<1, 256, 0, s>>>(glo, ghi, nT, range);
    double hr[2];
    CSS_HIP_TRY(hipMemcpyAsync(hr, range, sizeof(hr), hipMemcpyDeviceToHost, s));
    CSS_HIP_TRY(hipStreamSynchronize(s));
    if (!std::isfinite(hr[0]) || !std::isfinite(hr[1])) return CSS_E_NONFINITE;
    *lo = hr[0];
    *hi = hr[1];
    return CSS_OK;
}

}  // namespace css

extern "C" css_status css_fermi_poles(int32_t depth, double* kappa, double* weight, int32_t* npoles) {
    if (depth < 2 || depth > css::kMaxDepth || (depth & 1) || !npoles) return CSS_E_ARG;
    const css::PoleTable& t = css::pole_table(depth);
    *npoles = static_cast<int32_t>(t.kappa.size());
    for (size_t i = 0; i < t.kappa.size(); ++i) {
        if (kappa) kappa[i] = t.kappa[i];
        if (weight) weight[i] = t.weight[i];
    }
    return CSS_OK;
}
