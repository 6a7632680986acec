// Block Lanczos projection of H onto the block Krylov space of the CSS probes
// (Golub-Underwood process, text after Eq.(4)).
//
// Block recurrence, exact arithmetic:
//   H Q_j = Q_{j-1} B_{j-1}^T + Q_j A_j + Q_{j+1} B_j,  Q_0 = 0,
// so [Q_1..Q_k]^T H [Q_1..Q_k] is block tridiagonal (A_j diagonal, B_j below,
// B_j^T above). One step here:
//   W   = H Q_j                                   (CSR SpMM)
//   A_j = sym(Q_j^T W)                            (MFMA Gram)
//   W  <- W - Q_j A_j - Q_{j-1} B_{j-1}^T          (MFMA block update)
//   [re-orthogonalise W against Q_j, Q_{j-1} (local) or all Q (full), adding
//    the symmetrised Q_j coefficient to A_j]
//   W   = Q_{j+1} R by Cholesky QR on W^T W (twice with CholQR2), B_j = R;
//   stop when W^T W is not positive definite or min diag R <= 1e-10 ||H||_inf.
// The first block Q_1 = r B_0^-1 comes from the probes with B_0 = diag(sqrt n_c).
//
// No host synchronisation inside the loop: a breakdown sets a device flag
// that turns the remaining kernels of the run into no-ops. Every reduction is
// in a fixed order, so a second pass that replays the stored coefficients
// regenerates the basis bitwise (used when the basis is not stored).

#include <hip/hip_runtime.h>

#include <algorithm>
#include <type_traits>
#include <cmath>
#include <vector>

#include "css_common.h"
#include "dense.h"
#include "driver.h"
#include "hist.h"
#include "spmm.h"

namespace css {
namespace {

// ||H||_inf in two levels: one wavefront per row (sum of |H_mn|), each
// work-group's maximum to part[blockIdx.x]; k_max_reduce then takes the maximum
// of the parts (order independent, hence deterministic).
constexpr int kRowMaxBlocks = 1024;

template <typename V>
__global__ __launch_bounds__(256) void k_row_abs_max(int n, const int32_t* __restrict__ rp, const V* __restrict__ val,
                                                     double* __restrict__ part, int* __restrict__ state) {
    __shared__ double wm[4];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    double mx = 0.0;
    bool finite = true;
    for (int64_t i = (int64_t)blockIdx.x * 4 + w; i < n; i += (int64_t)gridDim.x * 4) {
        double s = 0.0;
        for (int32_t t = rp[i] + lane; t < rp[i + 1]; t += 64) {
            const double v = (double)val[t];
            finite = finite && isfinite(v);
            s += fabs(v);
        }
        for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
        mx = fmax(mx, s);
    }
    if (!finite) atomicOr(&state[1], 2);
    if (lane == 0) wm[w] = mx;
    __syncthreads();
    if (threadIdx.x == 0) part[blockIdx.x] = fmax(fmax(wm[0], wm[1]), fmax(wm[2], wm[3]));
}

// max over an array (deterministic: max is order independent)
__global__ void k_max_reduce(const double* __restrict__ v, int64_t n, double* __restrict__ out) {
    __shared__ double sm[256];
    double m = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += blockDim.x) m = fmax(m, v[i]);
    sm[threadIdx.x] = m;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s) sm[threadIdx.x] = fmax(sm[threadIdx.x], sm[threadIdx.x + s]);
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = sm[0];
}

// *acc = max(*acc, max |M_t[r][c] - [t == diag and r == c]| over r, c < b) for
// t = blockIdx.y, M_t = M + t*ld*ld. The maximum of non-negative doubles is taken on
// their bit patterns (an order-independent atomic maximum, so the result does not
// depend on the order of the work-groups); a NaN entry makes the result NaN.
__global__ __launch_bounds__(256) void k_ortho_max(const double* __restrict__ M, int b, int ld, int diag,
                                                   unsigned long long* __restrict__ acc) {
    __shared__ double sm[256];
    const int t = blockIdx.y;
    const int64_t per = (int64_t)b * b;
    const double* Mt = M + t * (int64_t)ld * ld;
    double m = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < per; i += (int64_t)gridDim.x * 256) {
        const int r = static_cast<int>(i / b), c = static_cast<int>(i % b);
        double v = Mt[(int64_t)r * ld + c];
        if (t == diag && r == c) v -= 1.0;
        v = fabs(v);
        if (!(v <= m)) m = (m != m) ? m : v;
    }
    sm[threadIdx.x] = m;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s) {
            const double o = sm[threadIdx.x + s];
            if (!(o <= sm[threadIdx.x]) && sm[threadIdx.x] == sm[threadIdx.x]) sm[threadIdx.x] = o;
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) atomicMax(acc, static_cast<unsigned long long>(__double_as_longlong(fabs(sm[0]))));
}

template <typename S, typename D>
__global__ void k_convert(const S* __restrict__ in, D* __restrict__ out, int64_t n) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < n) out[i] = D(in[i]);
}

__global__ void k_check_counts(const int* __restrict__ counts, int b, int* __restrict__ state) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c < b && counts[c] == 0) atomicOr(&state[1], 8);
}

template <typename T>
__global__ void k_zero(T* __restrict__ p, int64_t n) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < n) p[i] = T(0);
}

// Q_1[m, c(m)] = s_m / sqrt(n_c); all other entries (and padded rows) zero.
template <typename T>
__global__ void k_init_q1(const int32_t* __restrict__ color, const int8_t* __restrict__ sign,
                          const int* __restrict__ counts, int n, int64_t Np, int ld, T* __restrict__ Q) {
    const int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (idx >= Np * ld) return;
    const int64_t m = idx / ld;
    const int c = static_cast<int>(idx % ld);
    T v = T(0);
    if (m < n && color[m] == c) v = T((double)sign[m] / sqrt((double)counts[c]));
    Q[idx] = v;
}

__global__ void k_zero_small(double* __restrict__ p, int64_t n) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0.0;
}

template <typename T>
void zero_tall(T* p, int64_t count, hipStream_t s) {
    k_zero<T><<<grid_for(count, 256), 256, 0, s>>>(p, count);
}

template <typename T>
bool launch_spmm_t(const css_csr* H, const LzBufs& bf, const T* V, T* W, int ld, hipStream_t s) {
    const T* val = bf.hval ? static_cast<const T*>(bf.hval) : static_cast<const T*>(H->val);
    SpmmArgs<T> a{H->n, H->row_ptr, H->col, val, V, W, ld};
    if (bf.use_grp && spmm_grouped_launch(a, bf.grp, s)) return true;
    return spmm_launch(a, s);
}

__global__ void k_tau(double* __restrict__ scal) { scal[1] = 1e-10 * scal[0]; }

__global__ void k_set_int(int* __restrict__ p, int v) { *p = v; }

// ------------------------------------------------------------------ one step

template <typename T>
struct Step {
    const css_csr* H;
    const LzPlan& p;
    const LzBufs& bf;
    hipStream_t s;

    int64_t mat() const { return (int64_t)p.ld * p.ld; }
    int64_t tall() const { return p.Np * p.ld; }
    // Block holding Q_j (0-based): stored basis slot j, two-pass slot j % 3.
    T* q(int j) const { return static_cast<T*>(slot_ptr(p, bf, p.twopass ? j % 3 : j)); }
    // BF16 copy of Q_j (nullptr unless FP32 with full re-orthogonalisation)
    void* q16(int j) const {
        return bf.basis16 ? static_cast<void*>(static_cast<char*>(bf.basis16) + (size_t)j * p.Np * p.ld * 2)
                          : nullptr;
    }

    void gram(const T* X, int64_t xstride, int nprod, const T* Y, double* out, int64_t out_stride, bool sym,
              int mode, void* yplanes = nullptr, const double* hinf = nullptr,
              const GramExtra& ex = GramExtra()) const {
        gram_blocks_launch<T>(X, xstride, nprod, Y, p.Np, p.ld, sym, p.partial_mats, bf.partial, out, out_stride, mode,
                              bf.state, s, yplanes, hinf, ex);
    }
    void update(T* out, const T* in, double alpha, const T* X, int64_t xstride, int nprod, const double* S,
                int64_t sstride, bool trans, double scale, void* out16 = nullptr) const {
        update_launch<T>(out, in, alpha, X, xstride, nprod, S, sstride, trans, scale, p.Np, p.ld, bf.stage, bf.state,
                         s, out16);
    }

    // Step j (0-based). replay: regenerate Q_{j+1} from stored coefficients
    // (no Gram, no Cholesky). last: j == v_max - 1, no QR of W.
    bool run(int j, bool replay, bool last) const {
        const int ld = p.ld;
        T* W = static_cast<T*>(bf.W);
        T* Wt = static_cast<T*>(bf.Wt);
        T* Qj = q(j);
        double* Aj = bf.A + j * mat();
        double* Apre = bf.Apre + j * mat();
        if (!launch_spmm_t<T>(H, bf, Qj, W, ld, s)) return false;
        if (!replay) {                                                       // A_j = sym(Q_j^T W), also into Aj
            GramExtra ex;
            ex.copy = Aj;
            gram(Qj, 0, 1, W, Apre, 0, false, 1, nullptr, nullptr, ex);
        }
        if (j > 0)                                                           // W -= Q_j A_j + Q_{j-1} B^T
            update2_launch<T>(W, W, 1.0, Qj, Apre, false, q(j - 1), bf.B + (j - 1) * mat(), true, -1.0, p.Np, p.ld,
                              bf.stage, bf.state, s);
        else
            update(W, W, 1.0, Qj, 0, 1, Apre, 0, false, -1.0);                // W -= Q_j A_j
        if (p.reorth == 1 || (p.reorth == 2 && p.twopass)) {
            // local: coefficients against Q_{j-1} and Q_j, one block at a time
            const int first = std::max(0, j - 1);
            const int np = j - first + 1;
            double* C = p.twopass ? bf.C + (int64_t)j * p.max_coef * mat() : bf.C;
            if (!replay)
                for (int t = 0; t < np; ++t) {
                    GramExtra ex;                                   // A_j += sym(C) of Q_j
                    if (t == np - 1) {
                        ex.sym_to = Aj;
                        ex.sym_p = 0;
                    }
                    gram(q(first + t), 0, 1, W, C + t * mat(), 0, false, 0, nullptr, nullptr, ex);
                }
            for (int t = 0; t < np; ++t) update(W, W, 1.0, q(first + t), 0, 1, C + t * mat(), 0, false, -1.0);
        } else if (p.reorth == 2) {
            // full: coefficients against Q_0..Q_j (contiguous stored slots), batched; with
            // the alternating schedule, odd steps only against Q_{j-1}, Q_j
            const int first = (p.reorth_alt && (j & 1)) ? std::max(0, j - 1) : 0;
            const int np = j + 1 - first;
            const int cap = (int)std::max<int64_t>(1, p.partial_mats);
            for (int t0 = 0; t0 < np; t0 += cap) {
                const int cnt = std::min(cap, np - t0);
                GramExtra ex;                                       // A_j += sym(C) of Q_j (the last product)
                if (np - 1 < t0 + cnt) {
                    ex.sym_to = Aj;
                    ex.sym_p = np - 1 - t0;
                }
                gram(q(first + t0), tall(), cnt, W, bf.C + t0 * mat(), mat(), false, 0, bf.yplanes, bf.scal, ex);
            }
            // the corrections are of the size of the loss of orthogonality: with FP32 blocks
            // they read the BF16 copies of the basis (half the bytes of the stored blocks)
            bool done = false;
            if constexpr (std::is_same<T, float>::value) {
                if (bf.basis16)
                    done = update_correction_bf16_launch(W, W, 1.0, q16(first), tall(), np, bf.C, mat(), false, -1.0,
                                                         p.Np, p.ld, bf.stage, bf.state, s);
            }
            if (!done)
                update_correction_launch<T>(W, W, 1.0, q(first), tall(), np, bf.C, mat(), false, -1.0, p.Np, p.ld,
                                            bf.stage, bf.state, s);
        }
        if (last) return true;
        double* R1inv = p.twopass ? bf.R1inv + j * mat() : bf.R1inv;
        double* R2inv = p.twopass ? bf.R2inv + j * mat() : bf.R2inv;
        qr(j, q(j + 1), q16(j + 1), bf.B + j * mat(), R1inv, R2inv, replay);  // W = Q_{j+1} B_j
        return true;
    }

    // W = Qn R by Cholesky QR (twice with CholQR2); R into Rout. Factorisation idx
    // records its smallest pivots at min_diag[2 idx ..] and fails as step idx.
    void qr(int idx, T* Qn, void* Qn16, double* Rout, double* R1inv, double* R2inv, bool replay) const {
        const int ld = p.ld;
        T* W = static_cast<T*>(bf.W);
        T* Wt = static_cast<T*>(bf.Wt);
        if (!replay) {
            gram(W, 0, 1, W, bf.G, 0, true, 0);                               // G = W^T W
            chol_inv_launch(bf.G, p.b, ld, bf.scal + 1, p.cholqr2 ? bf.R1 : Rout, R1inv, bf.chol_scratch,
                            bf.state, 2 * idx, bf.min_diag, s);
        }
        if (p.cholqr2) {
            update(Wt, nullptr, 0.0, W, 0, 1, R1inv, 0, false, 1.0);           // Wt = W R1^-1
            if (!replay) {
                gram(Wt, 0, 1, Wt, bf.G, 0, true, 0);
                // Wt^T Wt = I + E, E of the first pass's loss of orthogonality: the series
                // factorisation when |E|^3 is below the working precision's rounding
                const double bound = tuning().chol_series == 2 ? -1.0 : (p.fp32 ? 1e-4 : 2e-6);
                chol_inv_near_identity_launch(bf.G, p.b, ld, bound, bf.R2, R2inv, bf.chol_scratch, bf.state,
                                              2 * idx + 1, bf.min_diag, s);
                trmm_upper_launch(bf.R2, bf.R1, Rout, ld, bf.state, s);      // R = R2 R1
            }
            update(Qn, nullptr, 0.0, Wt, 0, 1, R2inv, 0, false, 1.0, Qn16);    // Qn = Wt R2^-1
        } else {
            update(Qn, nullptr, 0.0, W, 0, 1, R1inv, 0, false, 1.0, Qn16);     // Qn = W R1^-1
        }
    }
};

// Start block (FP64, Np x ld, zero padding) into W in the Lanczos precision.
template <typename T>
__global__ void k_start_block(const double* __restrict__ in, T* __restrict__ W, int64_t n) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < n) W[i] = T(in[i]);
}

template <typename T>
css_status prepare(const css_csr* H, const int32_t* color, const int8_t* sign, const LzPlan& p, LzBufs& bf,
                   hipStream_t s) {
    k_zero<int><<<1, 64, 0, s>>>(bf.state, 16);
    csr_validate_launch(p.n, p.nnz, H->row_ptr, H->col, bf.state, s);
    CSS_HIP_TRY(hipGetLastError());
    int hst[16];
    CSS_HIP_TRY(hipMemcpyAsync(hst, bf.state, sizeof(hst), hipMemcpyDeviceToHost, s));
    CSS_HIP_TRY(hipStreamSynchronize(s));
    if (hst[1]) return CSS_E_CSR;
    if (p.grp_ok) spmm_grp_prepare(p.n, H->row_ptr, H->col, bf.grp, bf.state + 4, s);
    double* part = static_cast<double*>(bf.W);     // W (>= 256 x 16 elements) is free until the first SpMM
    const unsigned rgrid = std::min<unsigned>(kRowMaxBlocks, grid_for(p.n, 4));
    if (H->val_dtype == CSS_F64)
        k_row_abs_max<double><<<rgrid, 256, 0, s>>>(p.n, H->row_ptr, static_cast<const double*>(H->val), part,
                                                     bf.state);
    else
        k_row_abs_max<float><<<rgrid, 256, 0, s>>>(p.n, H->row_ptr, static_cast<const float*>(H->val), part,
                                                    bf.state);
    k_max_reduce<<<1, 256, 0, s>>>(part, rgrid, bf.scal);
    k_tau<<<1, 1, 0, s>>>(bf.scal);
    k_zero<int><<<grid_for(p.b, 256), 256, 0, s>>>(bf.counts, p.b);
    colour_hist(color, p.n, p.b, bf.counts, bf.state + 1, 4, s);
    k_check_counts<<<grid_for(p.b, 256), 256, 0, s>>>(bf.counts, p.b, bf.state);
    CSS_HIP_TRY(hipMemcpyAsync(hst, bf.state, sizeof(hst), hipMemcpyDeviceToHost, s));
    CSS_HIP_TRY(hipStreamSynchronize(s));
    if (hst[1] & 2) return CSS_E_NONFINITE;
    if (hst[1]) return CSS_E_CSR;
    // grouped SpMM where the 16 x |U_g| blocks hold at most kGroupFill times the
    // nonzeros, unless the tuning asks for the CSR kernel
    const bool blocks = p.grp_ok && tuning().kernel != 2 && spmm_grp_worthwhile(p.nnz, hst[4], hst[5]);
    bf.use_grp = blocks;
    bf.grp.blocks_ready = blocks;
    if (p.convert_h) {
        if (p.fp32)
            k_convert<double, float><<<grid_for(p.nnz, 256), 256, 0, s>>>(static_cast<const double*>(H->val),
                                                                           static_cast<float*>(bf.hval), p.nnz);
        else
            k_convert<float, double><<<grid_for(p.nnz, 256), 256, 0, s>>>(static_cast<const float*>(H->val),
                                                                           static_cast<double*>(bf.hval), p.nnz);
    }
    if (blocks)
        spmm_grp_fill<T>(p.n, H->row_ptr, bf.hval ? static_cast<const T*>(bf.hval) : static_cast<const T*>(H->val),
                         bf.grp, s);
    zero_tall<T>(static_cast<T*>(bf.W), p.Np * p.ld, s);
    if (bf.Wt) zero_tall<T>(static_cast<T*>(bf.Wt), p.Np * p.ld, s);
    const int64_t mat = (int64_t)p.ld * p.ld;
    k_zero_small<<<grid_for(p.v_max * mat, 256), 256, 0, s>>>(bf.A, p.v_max * mat);
    k_zero_small<<<grid_for(p.v_max * mat, 256), 256, 0, s>>>(bf.Apre, p.v_max * mat);
    k_zero_small<<<grid_for(p.v_max * mat, 256), 256, 0, s>>>(bf.B, p.v_max * mat);
    (void)sign;
    CSS_HIP_TRY(hipGetLastError());
    return CSS_OK;
}

template <typename T>
css_status pass1_t(const css_csr* H, const int32_t* color, const int8_t* sign, const LzPlan& p, LzBufs& bf,
                   hipStream_t s, int* v_eff, int* breakdown, double* min_diag, const double* start, double* R0) {
    CSS_TRY(prepare<T>(H, color, sign, p, bf, s));
    Step<T> st{H, p, bf, s};
    if (start) {
        // general first block: Q_1 R_0 = start by the step's Cholesky QR
        k_start_block<T><<<grid_for(p.Np * p.ld, 256), 256, 0, s>>>(start, static_cast<T*>(bf.W), p.Np * p.ld);
        k_zero_small<<<grid_for((int64_t)p.ld * p.ld, 256), 256, 0, s>>>(R0, (int64_t)p.ld * p.ld);
        st.qr(0, st.q(0), st.q16(0), R0, bf.R1inv, bf.R2inv, false);
        int hst[16];
        CSS_HIP_TRY(hipGetLastError());
        CSS_HIP_TRY(hipMemcpyAsync(hst, bf.state, sizeof(hst), hipMemcpyDeviceToHost, s));
        CSS_HIP_TRY(hipStreamSynchronize(s));
        if (hst[0]) return CSS_E_BREAKDOWN_AT_1;
        zero_tall<T>(static_cast<T*>(bf.W), p.Np * p.ld, s);
        if (bf.Wt) zero_tall<T>(static_cast<T*>(bf.Wt), p.Np * p.ld, s);
    } else {
        k_init_q1<T><<<grid_for(p.Np * p.ld, 256), 256, 0, s>>>(color, sign, bf.counts, p.n, p.Np, p.ld, st.q(0));
        if constexpr (std::is_same<T, float>::value) {
            if (bf.basis16) bf16_copy_launch(st.q(0), st.q16(0), p.Np * p.ld, s);
        }
    }
    for (int j = 0; j < p.v_max; ++j)
        if (!st.run(j, false, j == p.v_max - 1)) return CSS_E_UNSUPPORTED;
    CSS_HIP_TRY(hipGetLastError());
    int hst[16];
    CSS_HIP_TRY(hipMemcpyAsync(hst, bf.state, sizeof(hst), hipMemcpyDeviceToHost, s));
    std::vector<double> md(2 * std::max(1, p.v_max));
    CSS_HIP_TRY(hipMemcpyAsync(md.data(), bf.min_diag, sizeof(double) * md.size(), hipMemcpyDeviceToHost, s));
    CSS_HIP_TRY(hipStreamSynchronize(s));
    *breakdown = hst[0] ? 1 : 0;
    *v_eff = hst[0] ? hst[2] / 2 + 1 : p.v_max;
    double m = INFINITY;
    for (int j = 0; j < *v_eff - (hst[0] ? 0 : 1); ++j) m = std::min(m, md[2 * j]);
    *min_diag = m;
    return CSS_OK;
}

template <typename T>
css_status pass2_t(const css_csr* H, const int32_t* color, const int8_t* sign, const LzPlan& p, const LzBufs& bf,
                   int v_eff, const double* Fpad, void* Xv, hipStream_t s) {
    Step<T> st{H, p, bf, s};
    T* X = static_cast<T*>(Xv);
    k_set_int<<<1, 1, 0, s>>>(bf.state, 0);
    k_init_q1<T><<<grid_for(p.Np * p.ld, 256), 256, 0, s>>>(color, sign, bf.counts, p.n, p.Np, p.ld, st.q(0));
    zero_tall<T>(X, p.Np * p.ld, s);
    const int64_t mat = (int64_t)p.ld * p.ld;
    for (int j = 0; j < v_eff; ++j) {
        st.update(X, X, 1.0, st.q(j), 0, 1, Fpad + j * mat, 0, false, 1.0);    // X += Q_j F_j
        if (j < v_eff - 1 && !st.run(j, true, false)) return CSS_E_UNSUPPORTED;
    }
    CSS_HIP_TRY(hipGetLastError());
    return CSS_OK;
}

template <typename T>
css_status ortho_err_t(const LzPlan& p, const LzBufs& bf, int v_eff, hipStream_t s, double* out) {
    const int64_t mat = (int64_t)p.ld * p.ld;
    const int64_t tall = p.Np * p.ld;
    double* acc = bf.scal + 2;
    k_zero_small<<<1, 64, 0, s>>>(acc, 1);
    // products per launch: bounded by the staged outputs, and by the partial buffers
    // at the chunk count that keeps FP32 running sums short
    const int64_t by_partials = p.partial_mats / gram_min_chunks(p.Np, p.ld, (int)p.elem);
    const int64_t by_stage = std::max({2, p.v_max, p.max_coef}) + 1;
    const int cap = static_cast<int>(std::max<int64_t>(1, std::min(by_partials, by_stage)));
    for (int j = 0; j < v_eff; ++j) {
        const T* Qj = static_cast<const T*>(slot_ptr(p, bf, j));
        for (int t0 = 0; t0 <= j; t0 += cap) {
            const int cnt = std::min(cap, j + 1 - t0);
            // out[t] = Q_{t0+t}^T Q_j; no state flag, so a breakdown does not skip it
            gram_blocks_launch<T>(static_cast<const T*>(slot_ptr(p, bf, t0)), tall, cnt, Qj, p.Np, p.ld, false,
                                  p.partial_mats, bf.partial, bf.stage, mat, 0, nullptr, s);
            k_ortho_max<<<dim3(grid_for((int64_t)p.b * p.b, 256 * 8), cnt), 256, 0, s>>>(
                bf.stage, p.b, p.ld, j - t0, reinterpret_cast<unsigned long long*>(acc));
        }
    }
    CSS_HIP_TRY(hipGetLastError());
    CSS_HIP_TRY(hipMemcpyAsync(out, acc, sizeof(double), hipMemcpyDeviceToHost, s));
    CSS_HIP_TRY(hipStreamSynchronize(s));
    return CSS_OK;
}

}  // namespace

css_status lanczos_ortho_err(const LzPlan& p, const LzBufs& bf, int v_eff, hipStream_t s, double* out) {
    if (p.twopass) {
        *out = NAN;
        return CSS_OK;
    }
    if (p.fp32) return ortho_err_t<float>(p, bf, v_eff, s, out);
    return ortho_err_t<double>(p, bf, v_eff, s, out);
}

css_status lanczos_spmm(const css_csr* H, const LzPlan& p, const LzBufs& bf, const void* V, void* W, hipStream_t s) {
    const bool ok = p.fp32 ? launch_spmm_t<float>(H, bf, static_cast<const float*>(V), static_cast<float*>(W), p.ld, s)
                           : launch_spmm_t<double>(H, bf, static_cast<const double*>(V), static_cast<double*>(W),
                                                   p.ld, s);
    if (!ok) return CSS_E_UNSUPPORTED;
    CSS_HIP_TRY(hipGetLastError());
    return CSS_OK;
}

// ------------------------------------------------------------------ plan / carve

css_status plan_lanczos(const css_csr* H, int32_t b, int32_t depth, uint32_t flags, LzPlan& p) {
    if (!H || H->n < 1 || !H->row_ptr || !H->col || !H->val) return CSS_E_ARG;
    if (H->val_dtype != CSS_F64 && H->val_dtype != CSS_F32) return CSS_E_ARG;
    if (H->nnz < 0 || H->nnz >= (int64_t(1) << 31)) return CSS_E_CSR;
    if (b < 1 || b > H->n || depth < 1) return CSS_E_ARG;
    if (b > kMaxColors) return CSS_E_UNSUPPORTED;
    const uint32_t prec = flags & CSS_PREC_MASK;
    if (prec != CSS_PREC_FP64 && prec != CSS_PREC_FP32) return CSS_E_UNSUPPORTED;
    p.n = H->n;
    p.nnz = H->nnz;
    p.b = b;
    p.depth = depth;
    p.v_max = std::min(depth, H->n / b);
    p.ld = block_ld(b);
    p.Np = padded_rows(H->n);
    p.fp32 = prec == CSS_PREC_FP32;
    p.elem = p.fp32 ? 4 : 8;
    p.twopass = (flags & CSS_BASIS_TWOPASS) != 0;
    p.reorth = (flags & CSS_REORTH_FULL) ? 2 : ((flags & CSS_REORTH_LOCAL) ? 1 : 0);
    p.reorth_alt = p.reorth == 2 && (flags & CSS_REORTH_ALTERNATE) != 0;
    if (p.twopass && p.reorth == 2) return CSS_E_UNSUPPORTED;
    p.cholqr2 = (flags & CSS_CHOLQR2) != 0;
    p.convert_h = (p.fp32 && H->val_dtype == CSS_F64) || (!p.fp32 && H->val_dtype == CSS_F32);
    p.nslots = p.twopass ? 3 : std::max(1, p.v_max);
    p.max_coef = p.reorth == 2 ? p.v_max : (p.reorth == 1 ? 2 : 0);
    // partial Gram buffers: enough chunks for a single product, and at least 32
    // chunks per product for the batched full re-orthogonalisation Gram
    const int64_t single = std::min<int64_t>(gram_partial_mats(p.ld), std::max<int64_t>(1, p.Np / 64));
    const int64_t batched = std::min<int64_t>(32, std::max<int64_t>(1, p.Np / 64)) * std::max(1, p.max_coef);
    // FP32: enough chunks that no wave keeps an FP32 running sum over more than a few hundred rows
    const int64_t bounded = gram_min_chunks(p.Np, p.ld, (int)p.elem) * std::max(1, p.max_coef);
    p.partial_mats = std::max<int64_t>(1, std::max({single, batched, bounded}));
    p.grp_ok = (flags & CSS_SPMM_CSR) == 0 && p.ld <= 128;
    return CSS_OK;
}

void carve_lanczos(Arena& a, const LzPlan& p, LzBufs& bf) {
    const int64_t mat = (int64_t)p.ld * p.ld;
    const int64_t tall_bytes = p.Np * p.ld * (int64_t)p.elem;
    bf.basis = a.take<char>((size_t)p.nslots * tall_bytes);
    bf.basis16 = (p.fp32 && p.reorth == 2 && !p.twopass) ? a.take<char>((size_t)p.nslots * p.Np * p.ld * 2) : nullptr;
    bf.W = a.take<char>(tall_bytes);
    bf.Wt = p.cholqr2 ? a.take<char>(tall_bytes) : nullptr;
    bf.yplanes = (p.fp32 && p.reorth == 2) ? a.take<char>((size_t)3 * p.Np * p.ld * 2) : nullptr;
    bf.hval = p.convert_h ? a.take<char>((size_t)p.nnz * p.elem) : nullptr;
    const int v = std::max(1, p.v_max);
    bf.A = a.take<double>(v * mat);
    bf.Apre = a.take<double>(v * mat);
    bf.B = a.take<double>(v * mat);
    bf.C = a.take<double>((p.twopass ? v : 1) * std::max(1, p.max_coef) * mat);
    bf.R1inv = a.take<double>((p.twopass ? v : 1) * mat);
    bf.R2inv = a.take<double>((p.twopass ? v : 1) * mat);
    bf.G = a.take<double>(mat);
    bf.R1 = a.take<double>(mat);
    bf.R2 = a.take<double>(mat);
    bf.partial = a.take<double>(p.partial_mats * mat);
    bf.stage = a.take<double>((int64_t)(std::max({2, p.v_max, p.max_coef}) + 1) * mat);
    bf.chol_scratch = a.take<double>(chol_scratch_bytes(p.b) / sizeof(double) + 1);
    bf.min_diag = a.take<double>(2 * v);
    bf.scal = a.take<double>(16);
    bf.state = a.take<int>(16);
    bf.counts = a.take<int>(p.b);
    if (p.grp_ok) carve_groups(a, p.n, p.nnz, p.elem, bf.grp);
}

css_status run_lanczos_pass1(const css_csr* H, const int32_t* color, const int8_t* sign, const LzPlan& p,
                             LzBufs& bf, hipStream_t s, int* v_eff, int* breakdown, double* min_diag,
                             const double* start, double* R0) {
    if (start && (p.twopass || !R0)) return CSS_E_UNSUPPORTED;
    if (p.fp32) return pass1_t<float>(H, color, sign, p, bf, s, v_eff, breakdown, min_diag, start, R0);
    return pass1_t<double>(H, color, sign, p, bf, s, v_eff, breakdown, min_diag, start, R0);
}

css_status run_lanczos_pass2(const css_csr* H, const int32_t* color, const int8_t* sign, const LzPlan& p,
                             const LzBufs& bf, int v_eff, const double* Fpad, void* X, hipStream_t s) {
    if (p.fp32) return pass2_t<float>(H, color, sign, p, bf, v_eff, Fpad, X, s);
    return pass2_t<double>(H, color, sign, p, bf, v_eff, Fpad, X, s);
}

size_t lanczos_workspace_bytes(const LzPlan& p) {
    Arena a;
    LzBufs bf;
    carve_lanczos(a, p, bf);
    return a.used + 256;
}

}  // namespace css

using namespace css;

extern "C" css_status css_block_lanczos(const css_csr* H, const int32_t* color, const int8_t* sign,
                                        int32_t n_colors, int32_t depth, uint32_t flags, double* A, double* B,
                                        css_info* info, void* ws, size_t ws_bytes, void* stream) {
    if (!color || !sign || !A || (depth > 1 && !B) || !ws) return CSS_E_ARG;
    LzPlan p;
    CSS_TRY(plan_lanczos(H, n_colors, depth, flags, p));
    if (ws_bytes < lanczos_workspace_bytes(p)) return CSS_E_WORKSPACE;
    Arena a;
    a.base = static_cast<char*>(ws);
    a.cap = ws_bytes;
    LzBufs bf;
    carve_lanczos(a, p, bf);
    if (a.overflow) return CSS_E_WORKSPACE;
    hipStream_t s = as_stream(stream);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (info) {
        CSS_HIP_TRY(hipEventCreate(&e0));
        CSS_HIP_TRY(hipEventCreate(&e1));
        CSS_HIP_TRY(hipEventRecord(e0, s));
    }
    int v_eff = 0, brk = 0;
    double md = 0.0;
    css_status st = run_lanczos_pass1(H, color, sign, p, bf, s, &v_eff, &brk, &md);
    if (st != CSS_OK) {
        if (e0) { (void)hipEventDestroy(e0); (void)hipEventDestroy(e1); }
        return st;
    }
    double ortho = NAN;
    if (flags & CSS_DIAG_ORTHO) {
        st = lanczos_ortho_err(p, bf, v_eff, s, &ortho);
        if (st != CSS_OK) {
            if (e0) { (void)hipEventDestroy(e0); (void)hipEventDestroy(e1); }
            return st;
        }
    }
    const int64_t mat = (int64_t)p.ld * p.ld;
    const int64_t bb = (int64_t)p.b * p.b;
    for (int j = 0; j < v_eff; ++j) copy_small_launch(bf.A + j * mat, p.ld, p.b, A + j * bb, s);
    for (int j = 0; j + 1 < v_eff; ++j) copy_small_launch(bf.B + j * mat, p.ld, p.b, B + j * bb, s);
    CSS_HIP_TRY(hipGetLastError());
    if (info) {
        CSS_HIP_TRY(hipEventRecord(e1, s));
        CSS_HIP_TRY(hipEventSynchronize(e1));
        float ms = 0.f;
        CSS_HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        *info = css_info{};
        info->depth_eff = v_eff;
        info->n_colors = p.b;
        info->breakdown = brk;
        info->spmm_kernel = bf.use_grp ? 1 : 0;
        info->min_diag_r = md;
        info->ortho_err = ortho;
        info->idem_defect = NAN;
        info->t_phase_ms[0] = ms;
        info->t_phase_ms[5] = ms;
    } else {
        CSS_HIP_TRY(hipStreamSynchronize(s));
    }
    return CSS_OK;
}
