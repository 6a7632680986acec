// Internal dense block kernels (MFMA Gram / block update, small b x b FP64 ops).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace css {

// Tall blocks: Np x ld row-major, Np a multiple of kRowPad, rows >= n and
// columns >= b zero. Small matrices: ld x ld row-major FP64, zero outside b x b.

// Split-K Gram plan. out[p] = X_p^T Y (X_p = X + p*xstride) for p < nprod.
struct GramPlan {
    int ld, nprod, ntiles, nchunk;
    int64_t Np, rows_per_chunk;
    bool sym;
};
GramPlan gram_plan(int64_t Np, int ld, int nprod, bool sym, int64_t partial_cap_mats, int elem);
int64_t gram_partial_mats(int ld);                 // capacity (in ld x ld matrices) to reserve
// Chunks (partials per product) a Gram of Np rows needs so that no FP32 running sum
// is longer than a fixed row count (1 for FP64); reserve nprod times this.
int64_t gram_min_chunks(int64_t Np, int ld, int elem);

// Further outputs of a Gram's reduction, in place of separate small kernels:
// copy (mode 1): the symmetrised result also written here; sym_to, sym_p: for product
// sym_p of the launch, sym_to += (S + S^T)/2 as well (any mode).
struct GramExtra {
    double* copy = nullptr;
    double* sym_to = nullptr;
    int sym_p = -1;
};

// mode: 0 = plain, 1 = (S + S^T)/2, 2 = add (S + S^T)/2 into out (out += sym)
template <typename T>
void gram_launch(const GramPlan& g, const T* X, int64_t xstride, const T* Y, double* partial,
                 double* out, int64_t out_stride, int mode, const int* state, hipStream_t s,
                 const GramExtra& ex = GramExtra());

// OUT = alpha*IN + sum_p X_p * op_p(S_p),  op_p(S) = scale * (trans ? S^T : S)
// X_p = X + p*xstride (tall), S_p = S + p*sstride (small FP64). OUT may equal IN;
// OUT must not alias any X_p. stage (scratch): (nprod + 1)*ld*ld doubles. FP32 with
// ld = 16 NT, 3 <= NT <= 8: the products run on BF16 MFMA with both factors split
// in three parts (six products, each term as accurate as the FP32 product).
// out16 (FP32 only, may be nullptr): also a BF16 (nearest-even) copy of OUT, Np x ld.
template <typename T>
void update_launch(T* OUT, const T* IN, double alpha, const T* X, int64_t xstride, int nprod,
                   const double* S, int64_t sstride, bool trans, double scale, int64_t Np, int ld,
                   void* stage, const int* state, hipStream_t s, void* out16 = nullptr);

// out[i] = BF16 (nearest even) of in[i], i < n.
void bf16_copy_launch(const float* in, void* out, int64_t n, hipStream_t s);

// The re-orthogonalisation correction OUT = alpha IN + sum_p X16_p op(S_p) with the
// blocks X_p given by their BF16 copies (X16_p = X16 + p xstride, BF16 elements) and
// the coefficients rounded to one BF16 part: one BF16 MFMA product per term, each
// within 2^-8 |X||S| of the exact one (for coefficients of the size of a loss of
// orthogonality, far under FP32 rounding of OUT). stage: as update_launch. Returns
// false (nothing launched) when ld is not 16, 32, ..., 128.
bool update_correction_bf16_launch(float* OUT, const float* IN, double alpha, const void* X16, int64_t xstride,
                                   int nprod, const double* S, int64_t sstride, bool trans, double scale, int64_t Np,
                                   int ld, void* stage, const int* state, hipStream_t s);

// OUT = alpha*IN + X0 op0(S0) + X1 op1(S1) in one pass over OUT (two products with
// their own transposition), op_i(S) = scale * (trans_i ? S^T : S). stage: 3*ld*ld
// doubles. FP32: as update_launch.
template <typename T>
void update2_launch(T* OUT, const T* IN, double alpha, const T* X0, const double* S0, bool trans0, const T* X1,
                    const double* S1, bool trans1, double scale, int64_t Np, int ld, void* stage, const int* state,
                    hipStream_t s);

// Gram X_p^T Y (p < nprod, X_p = X + p xstride), mode as gram_launch, partial
// capacity cap_mats ld x ld FP64 matrices. FP32 blocks with ld a multiple of 16 up
// to 96: BF16 MFMA with three-part operand splits (each term no less accurate than
// the FP32 product; the whole tile is computed and sym is not used there);
// otherwise gram_plan + gram_launch. yplanes (FP32 split path, nprod > 1): room for
// Y's three BF16 planes (3 Np ld bf16), so that Y is split once for all products;
// nullptr splits Y inside every product. hinf (device, ||H||_inf; with yplanes):
// the products take two FP16 parts of scaled operands and three FP16 MFMA products
// instead (each term within 3 2^-22 of the exact one), for X blocks of unit-norm
// columns and Y bounded entrywise by ||H||_inf (the re-orthogonalisation Gram).
template <typename T>
void gram_blocks_launch(const T* X, int64_t xstride, int nprod, const T* Y, int64_t Np, int ld, bool sym,
                        int64_t cap_mats, double* partial, double* out, int64_t out_stride, int mode,
                        const int* state, hipStream_t s, void* yplanes = nullptr, const double* hinf = nullptr,
                        const GramExtra& ex = GramExtra());

// update_launch for coefficient blocks S_p that are small corrections (full
// reorthogonalisation after the three-term update). FP32 blocks with ld a multiple
// of 16 up to 128: products on BF16 MFMA with both factors split in two BF16 parts
// (relative error of each product term below 2^-15; stage holds the split
// coefficients, at most nprod*ld*ld doubles). FP64, and other ld: update_launch.
template <typename T>
void update_correction_launch(T* OUT, const T* IN, double alpha, const T* X, int64_t xstride, int nprod,
                              const double* S, int64_t sstride, bool trans, double scale, int64_t Np, int ld,
                              void* stage, const int* state, hipStream_t s);

// Cholesky G = R^T R of the leading b x b block, R and R^-1 (ld x ld, zero
// elsewhere). On failure (non-positive pivot, non-finite, min diag <= tau) sets
// state[0] = 1, state[2] = step, writes R^-1 = 0. Tracks min diag in *min_diag.
// tau: device scalar (min diag threshold) or nullptr for no threshold.
void chol_inv_launch(const double* G, int b, int ld, const double* tau, double* R, double* Rinv,
                     double* scratch, int* state, int step, double* min_diag, hipStream_t s);

// chol_inv_launch without a threshold for G near the identity: a second-order series
// (R^T R = G + O(|E|^3), R^-1 to the same order, E = G - I) when max |E_ij| <= thresh,
// the blocked factorisation otherwise (b <= 128; larger b always factorise).
void chol_inv_near_identity_launch(const double* G, int b, int ld, double thresh, double* R, double* Rinv,
                                   double* scratch, int* state, int step, double* min_diag, hipStream_t s);


// R = R2 * R1 (upper triangular, ld x ld)
void trmm_upper_launch(const double* R2, const double* R1, double* R, int ld, const int* state,
                       hipStream_t s);

// out (b x b, dense) = M (ld x ld) leading block
void copy_small_launch(const double* M, int ld, int b, double* out, hipStream_t s);

// Generic FP64 GEMM C = A B (+ beta C) with arbitrary element strides (MFMA).
void gemm_f64_launch(int M, int N, int K, const double* A, int64_t a_rs, int64_t a_cs,
                     const double* B, int64_t b_rs, int64_t b_cs, double* C, int64_t c_rs,
                     int64_t c_cs, hipStream_t s);

size_t chol_scratch_bytes(int b);

}  // namespace css
