// Internal: block Lanczos driver state shared by css_block_lanczos and
// css_density_matrix.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "css_common.h"
#include "spmm.h"

namespace css {

struct LzPlan {
    int32_t n = 0, b = 0, ld = 0, depth = 0, v_max = 0;
    int64_t Np = 0, nnz = 0;
    bool fp32 = false;        // blocks and SpMM in FP32
    bool twopass = false;     // no stored basis
    int reorth = 0;           // 0 none, 1 local, 2 full
    bool reorth_alt = false;  // full on even steps, local on odd steps
    bool cholqr2 = false;
    bool convert_h = false;   // H values converted into the workspace
    int nslots = 0;           // tall blocks kept for the basis
    int max_coef = 0;         // reorthogonalisation products per step
    int64_t partial_mats = 0;
    size_t elem = 8;
    bool grp_ok = false;      // grouped MFMA SpMM allowed (ld <= 128, not CSS_SPMM_CSR)
};

struct LzBufs {
    void* basis = nullptr;    // nslots x Np x ld
    void* basis16 = nullptr;  // FP32 with full re-orthogonalisation: BF16 copies of the basis blocks,
                              // read by the re-orthogonalisation correction (nslots x Np x ld)
    void* W = nullptr;
    void* Wt = nullptr;
    void* yplanes = nullptr;  // 3 x Np x ld bf16 (FP32, full reorth): W split once for the batched Gram
    void* hval = nullptr;     // converted H values (or nullptr)
    double* A = nullptr;      // v_max x ld x ld (final A_j)
    double* Apre = nullptr;   // v_max x ld x ld (A_j as used in the three-term update)
    double* B = nullptr;      // v_max x ld x ld
    double* C = nullptr;      // v_max x max_coef x ld x ld (reorth coefficients, two-pass) or max_coef x ld x ld
    double* R1inv = nullptr;  // v_max x ld x ld (two-pass) or 1
    double* R2inv = nullptr;  // v_max x ld x ld (two-pass, CholQR2) or 1
    double* G = nullptr;      // ld x ld
    double* R1 = nullptr;
    double* R2 = nullptr;
    double* partial = nullptr;
    double* stage = nullptr;      // staged small matrices for the block update ((max_prod + 1) x ld x ld)
    double* chol_scratch = nullptr;
    double* min_diag = nullptr;   // 2 * v_max
    double* scal = nullptr;       // 16 doubles: [0] ||H||_inf
    int* state = nullptr;         // 16 ints: [0] broken, [1] bad input, [2] fail step
    int* counts = nullptr;        // b colour counts
    SpmmGroups grp{};             // row-group unions (grp_ok)
    bool use_grp = false;         // host decision taken when H is validated
};

css_status plan_lanczos(const css_csr* H, int32_t n_colors, int32_t depth, uint32_t flags, LzPlan& p);
void carve_lanczos(Arena& a, const LzPlan& p, LzBufs& bf);

// Validates H (and colours), converts H if needed, builds Q_1 in slot 0 and
// runs pass 1. On return (stream synchronised) *v_eff and *breakdown are set.
// Also decides bf.use_grp.
// W = H V for an Np x ld block in the Lanczos precision, on the kernel the Lanczos
// steps use (the grouped kernel when it was prepared). Rows n..Np-1 of W are not written.
css_status lanczos_spmm(const css_csr* H, const LzPlan& p, const LzBufs& bf, const void* V, void* W, hipStream_t s);

// start (optional, device FP64 Np x ld, zero in the padding): the first block is
// then Q_1 with Q_1 R0 = start (Cholesky QR of the steps, R0 ld x ld upper) instead
// of the normalised probes; stored basis only.
css_status run_lanczos_pass1(const css_csr* H, const int32_t* color, const int8_t* sign, const LzPlan& p,
                             LzBufs& bf, hipStream_t s, int* v_eff, int* breakdown, double* min_diag,
                             const double* start = nullptr, double* R0 = nullptr);

// max |Q_t^T Q_j - [t == j] I| over t <= j < v_eff (b x b blocks) after pass 1, from the
// library's Gram products in the Lanczos precision; NaN with no stored basis. Host
// synchronising; uses the Gram partials, the staging buffer and scal[2].
css_status lanczos_ortho_err(const LzPlan& p, const LzBufs& bf, int v_eff, hipStream_t s, double* out);

// Pointer to the tall block holding Q_{j} (0-based j) after pass 1 with a stored basis.
inline void* slot_ptr(const LzPlan& p, const LzBufs& bf, int j) {
    return static_cast<char*>(bf.basis) + (size_t)j * p.Np * p.ld * p.elem;
}

// Two-pass: regenerate Q_0..Q_{v_eff-1} and accumulate X = sum_j Q_j F_j,
// F_j = Fpad + j*ld*ld (FP64). X is Np x ld of the block type.
css_status run_lanczos_pass2(const css_csr* H, const int32_t* color, const int8_t* sign, const LzPlan& p,
                             const LzBufs& bf, int v_eff, const double* Fpad, void* X, hipStream_t s);

}  // namespace css
