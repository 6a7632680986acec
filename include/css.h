/*
 * css.h -- C ABI of the chromatic-superposition-state (CSS) density-matrix
 * library for AMD Instinct MI355X (gfx950).
 *
 * The method (arXiv 2605.20918) estimates the sparse finite-temperature
 * density matrix P = g f(H), f the Fermi-Dirac function of Eq.(1), on the
 * pairs of orbitals closer than a cutoff:
 *   1. colour the orbitals so that orbitals closer than the cutoff differ
 *      (greedy Welsh-Powell multicolouring, text around Eq.(2), Fig.1(b));
 *   2. build one +-1 probe per colour (Eq.(2), Fig.1(c));
 *   3. project H onto the block Krylov space of the probes by block Lanczos
 *      (text after Eq.(4));
 *   4. evaluate f exactly in that small space by diagonalisation (Eqs.(5)-(7))
 *      and read P_mn = s_n X[m, colour(n)] off X = f(H) r (Eqs.(3), (6)).
 *
 * Conventions for every entry point
 *   - Arrays documented "device" are device memory the caller owns (for
 *     example torch tensors); the library never allocates, frees or keeps them.
 *     Arrays documented "host" are ordinary host memory.
 *   - Scratch memory comes only from the caller's workspace `ws` of
 *     `ws_bytes` bytes (device, 256-byte aligned); query its size with
 *     css_workspace_size. The library keeps no allocation between calls.
 *   - `stream` is a hipStream_t passed as void* (NULL = the default stream).
 *     Work is enqueued on it in order; entry points that return host scalars
 *     synchronise that stream before returning.
 *   - Every entry point returns a css_status and never throws or aborts. On an
 *     error the outputs are unspecified. A Lanczos breakdown after the first
 *     block is not an error: it is reported through css_info.
 *   - Results are deterministic: the same inputs give bitwise identical
 *     outputs (no floating-point atomics in any reduction).
 */
#ifndef CSS_H
#define CSS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t css_status;
enum {
    CSS_OK = 0,
    CSS_E_ARG = 1,            /* bad scalar argument or NULL pointer */
    CSS_E_CSR = 2,            /* malformed CSR (row pointers, column range) or colours */
    CSS_E_WORKSPACE = 3,      /* ws_bytes smaller than css_workspace_size reports */
    CSS_E_DEVICE = 4,         /* HIP runtime error */
    CSS_E_BREAKDOWN_AT_1 = 5, /* the first Lanczos block already degenerates */
    CSS_E_NONFINITE = 6,      /* NaN or Inf in H or in the projected matrix */
    CSS_E_EIG = 7,            /* the subspace eigensolver failed */
    CSS_E_UNSUPPORTED = 8,    /* option or size outside what is implemented */
    CSS_E_CAPACITY = 9        /* an output array is smaller than the result */
};

/* value types of css_csr.val */
enum { CSS_F64 = 0, CSS_F32 = 1 };

/* flags (bitwise or) for css_block_lanczos / css_density_matrix / css_build_probes */
#define CSS_PREC_FP64      0x0u   /* SpMM and block products in FP64 */
#define CSS_PREC_FP32      0x1u   /* Krylov blocks and H stored in FP32; SpMM in FP32 with FP32
                                     accumulation (FP32 MFMA in the grouped kernel); Gram and
                                     block-update products on BF16/FP16 MFMA with operands split
                                     in two or three parts where the block width allows (each
                                     product term as accurate as the FP32 one), else FP32 MFMA;
                                     Gram partial sums in FP32 over at most a few hundred rows,
                                     reduced in FP64; the Cholesky factors, T, the subspace
                                     solve, the gather and every trace and energy sum in FP64.
                                     The other values of the precision bits (0x2, 0x3) return
                                     CSS_E_UNSUPPORTED. */
#define CSS_PREC_MASK      0x3u
#define CSS_BASIS_STORED   0x0u   /* keep every Krylov block for the reconstruction */
#define CSS_BASIS_TWOPASS  0x4u   /* store no basis; regenerate it in a second pass */
#define CSS_REORTH_NONE    0x0u
#define CSS_REORTH_LOCAL   0x8u   /* second Gram-Schmidt pass against Q_{j-1}, Q_j */
#define CSS_REORTH_FULL    0x10u  /* second Gram-Schmidt pass against Q_1..Q_j */
#define CSS_REORTH_MASK    0x18u
#define CSS_CHOLQR2        0x20u  /* repeat the Cholesky QR once */
#define CSS_SYMMETRIZE     0x40u  /* return (P + P^T)/2 instead of the raw estimate */
#define CSS_SIGNS_ONES     0x80u  /* probes with all signs +1 instead of random signs */
#define CSS_SUBSPACE_EIG   0x100u /* subspace Fermi operator by dense diagonalisation (rocSOLVER)
                                     instead of the default pole expansion of Eq.(7) */
#define CSS_SPMM_CSR       0x200u /* always use the row-parallel CSR SpMM kernel; by default the
                                     16-row grouped MFMA kernel is used where H's row groups
                                     are dense enough (see css_spmm_prepare) */
#define CSS_REORTH_ALTERNATE 0x800u /* with CSS_REORTH_FULL: the full pass on even steps
                                       only, the local pass on odd steps */
#define CSS_DIAG_ORTHO     0x400u /* css_block_lanczos / css_density_matrix /
                                     css_density_matrix_nonorth: measure the loss of
                                     orthogonality of the stored Krylov basis,
                                     info.ortho_err = max |Q^T Q - I| over all block pairs
                                     (v_eff (v_eff + 1) / 2 block Gram products in the Lanczos
                                     precision, counted in the Lanczos phase time); NaN with
                                     CSS_BASIS_TWOPASS or without the flag */

/* workspace query selectors */
enum { CSS_ENTRY_COLOR = 0, CSS_ENTRY_LANCZOS = 1, CSS_ENTRY_DENSITY = 2, CSS_ENTRY_SPMM = 3,
       CSS_ENTRY_ENERGY_DENSITY = 4, CSS_ENTRY_FIND_MU = 5, CSS_ENTRY_INV_SQRT = 6,
       CSS_ENTRY_TRANSFORM_H = 7, CSS_ENTRY_DENSITY_NONORTH = 8 };

/* Sparse symmetric H in CSR form; all pointers device. Column indices must be
 * sorted within each row; row_ptr[0] = 0, row_ptr[n] = nnz < 2^31. */
typedef struct {
    int32_t n;
    int64_t nnz;
    const int32_t* row_ptr;   /* device, n+1 */
    const int32_t* col;       /* device, nnz */
    const void* val;          /* device, nnz, of type val_dtype */
    int32_t val_dtype;        /* CSS_F64 or CSS_F32 */
} css_csr;

/* Diagnostics filled by css_block_lanczos / css_density_matrix (host struct). */
typedef struct {
    int32_t depth_eff;        /* Krylov blocks actually built (v_eff) */
    int32_t n_colors;         /* b */
    int32_t breakdown;        /* 1 if the recurrence stopped early on a degenerate block */
    int32_t n_poles;          /* poles of the Fermi expansion (0 with CSS_SUBSPACE_EIG) */
    int32_t spmm_kernel;      /* 1: the 16-row grouped MFMA SpMM ran, 0: the CSR kernel */
    int32_t n_evals;          /* css_find_mu: evaluations of the electron count (0 elsewhere) */
    double min_diag_r;        /* smallest diagonal of the Cholesky factors of W^T W */
    double asym_max;          /* max |P_raw - (P_raw + P_raw^T)/2| on the pattern */
    double trace_krylov;      /* sum_k g f(lambda_k) w_k (Krylov quadrature of Tr P) */
    double e_band_krylov;     /* sum_k lambda_k g f(lambda_k) w_k */
    double t_phase_ms[6];     /* lanczos, subspace solve, F padding, reconstruction, gather, total */
    double ortho_err;         /* max |Q^T Q - I| of the Krylov basis with CSS_DIAG_ORTHO, else NaN */
    double idem_defect;       /* css_density_matrix / css_energy_density_matrix: Tr P - ||P||_F^2 / g
                                 over the returned pattern values (g = spin_deg); for the Fermi-Dirac
                                 operator of Eq.(1), P = g f(H), it is g sum_k f_k (1 - f_k) >= 0,
                                 zero for a projector and small at small kT in a gapped system.
                                 NaN elsewhere */
} css_info;

/*
 * css_color -- conflict graph and greedy colouring (text around Eq.(2), Fig.1(b)).
 *   Orbitals m, n conflict when the minimum-image distance between their
 *   centres is within r_cut: d^2 = (dx*dx + dy*dy) + dz*dz <= r_cut*r_cut with
 *   dx -= L*rint(dx/L) in periodic directions (L = box[k] > 0), rounded
 *   without fused multiply-add. The pattern of P is this graph plus the
 *   diagonal. Colours follow first fit along the Welsh-Powell order (degree
 *   descending, index ascending); they are bitwise equal to the sequential
 *   greedy colouring.
 *   xyz        device, n x 3 doubles, row-major orbital centres
 *   n          number of orbitals (>= 1)
 *   box        host, 3 doubles: periodic box edges, 0 = open direction
 *   r_cut      cutoff distance (> 0)
 *   color      device int32[n] out (may be NULL in a size query)
 *   n_colors   host out: number of colours b
 *   p_row_ptr  device int64[n+1] out: pattern row pointers
 *   p_col      device int32[*p_nnz] out: sorted pattern columns; NULL = size query
 *              (then only p_row_ptr and *p_nnz are produced)
 *   p_nnz      host in/out: in = capacity of p_col, out = nnz of the pattern;
 *              CSS_E_CAPACITY if the capacity is too small
 *   rounds     host out (may be NULL): fixed-point colouring sweeps used (the
 *              last one found no change)
 */
css_status css_color(const double* xyz, int32_t n, const double box[3], double r_cut,
                     int32_t* color, int32_t* n_colors,
                     int64_t* p_row_ptr, int32_t* p_col, int64_t* p_nnz, int32_t* rounds,
                     void* ws, size_t ws_bytes, void* stream);

/*
 * css_build_probes -- signs and colour counts of the CSS probes (Eq.(2), Fig.1(c)).
 *   Probe c is r_c[m] = sign[m] for colour(m) = c, 0 otherwise. sign[m] = +1
 *   when the top bit of the (m+1)-th SplitMix64 output from state `seed` is 0,
 *   else -1 (all +1 with CSS_SIGNS_ONES).
 *   color        device int32[n], values in [0, n_colors)
 *   sign         device int8[n] out
 *   color_count  device int32[n_colors] out: orbitals per colour
 *   Returns CSS_E_CSR if a colour is out of range or a colour owns no orbital
 *   (synchronises the stream to check).
 */
css_status css_build_probes(const int32_t* color, int32_t n, int32_t n_colors, uint64_t seed,
                            uint32_t flags, int8_t* sign, int32_t* color_count, void* stream);

/*
 * css_spmm_prepare -- column unions for the grouped SpMM kernel (a layout of
 *   the sparse-dense product of css_spmm; no arithmetic of the method).
 *   For every group of 16 consecutive rows: the sorted union U of their column
 *   indices, and H's values of those rows as a dense 16 x |U| block.
 *   ws    device, css_workspace_size(CSS_ENTRY_SPMM, n, nnz, ...) bytes, owned
 *         by the caller; pass it to css_spmm while H (structure and values)
 *         stays unchanged.
 *   Validates H's structure and synchronises the stream. Returns CSS_E_CSR for
 *   a malformed H, CSS_E_UNSUPPORTED if a group of 16 rows holds more than 8192
 *   nonzeros or the blocks would hold more than 4 times H's nonzeros (rows whose
 *   neighbours share few columns; css_spmm then needs ws = NULL).
 */
css_status css_spmm_prepare(const css_csr* H, void* ws, size_t ws_bytes, void* stream);

/*
 * css_spmm -- W = H V for a dense block V of b columns (the sparse-dense
 *   product the whole method reduces to, text after Eq.(10)).
 *   V, W  device, n x ld row-major, element type = H's value type; ld >= b,
 *         ld a multiple of 16 (css_block_ld(b) gives the library's choice)
 *   ws    NULL: row-parallel CSR kernel. Else a workspace filled by
 *         css_spmm_prepare for this H: the grouped MFMA kernel when ld <= 128
 *         and V, W are 16-byte aligned, the CSR kernel otherwise. The grouped
 *         kernel needs a finite V (a block's zeros multiply every V row of
 *         its union).
 *   Columns b..ld-1 of W are H times those columns of V (zero when V's are).
 *   H is not validated here (css_spmm_prepare, css_block_lanczos and
 *   css_density_matrix do).
 */
css_status css_spmm(const css_csr* H, const void* V, void* W, int32_t b, int32_t ld,
                    const void* ws, size_t ws_bytes, void* stream);

/*
 * css_block_lanczos -- block Lanczos projection (text after Eq.(4)).
 *   Builds Q_1 = r B_0^-1 from the probes and runs the block recurrence
 *   H Q_j = Q_{j-1} B_{j-1}^T + Q_j A_j + Q_{j+1} B_j for
 *   j = 1..min(depth, floor(n/b)), stopping early if W^T W is not positive
 *   definite or min diag R <= 1e-10 ||H||_inf.
 *   A  device, depth*b*b doubles out: A_j row-major at A + (j-1)*b*b
 *   B  device, (depth-1)*b*b doubles out: B_j (upper triangular) at B + (j-1)*b*b
 *   info host out (may be NULL).
 *   Only the first info->depth_eff blocks of A (depth_eff-1 of B) are defined.
 */
css_status css_block_lanczos(const css_csr* H, const int32_t* color, const int8_t* sign,
                             int32_t n_colors, int32_t depth, uint32_t flags,
                             double* A, double* B, css_info* info,
                             void* ws, size_t ws_bytes, void* stream);

/*
 * css_density_matrix -- the CSS estimate of P = g f(H) on a pattern
 *   (Eqs.(1)-(7) with S = I). Block Lanczos, then F = [g f(T)]_{:,1} B_0 for the
 *   block-tridiagonal projected H (B_0 = diag(sqrt n_c)): by default from the
 *   contour integral of Eq.(7) written as a sum of resolvents (a rational
 *   approximation of f accurate to about 1e-15, poles from css_fermi_poles), with
 *   CSS_SUBSPACE_EIG (and always when n_colors > 128) by dense diagonalisation
 *   (rocSOLVER dsyevd) as the paper does, F = U diag(g f(lambda)) U[0:b,:]^T B_0.
 *   Then X = [Q_1..Q_k] F and P_mn = sign[n] X[m, colour(n)] on the pattern
 *   (Eqs.(3), (6)), symmetrised with CSS_SYMMETRIZE.
 *   mu, kT      chemical potential and temperature (kT > 0), units of H
 *   spin_deg    g (2 for closed shells)
 *   p_row_ptr, p_col, p_nnz  device pattern (e.g. from css_color): columns sorted
 *               (strictly increasing) within each row, always (the band energy
 *               looks H's entries up in the pattern rows); symmetric when
 *               CSS_SYMMETRIZE is set. CSS_E_CSR otherwise
 *   p_val       device double[p_nnz] out
 *   e_band      host out: sum over entries in both H and the pattern of H_mn P_mn
 *   trace       host out: sum_m P_mm
 *   info        host out (may be NULL)
 */
css_status css_density_matrix(const css_csr* H, const int32_t* color, const int8_t* sign,
                              int32_t n_colors, double mu, double kT, int32_t depth,
                              double spin_deg, const int64_t* p_row_ptr, const int32_t* p_col,
                              int64_t p_nnz, uint32_t flags, double* p_val,
                              double* e_band, double* trace, css_info* info,
                              void* ws, size_t ws_bytes, void* stream);

/*
 * css_density_matrix_noalloc -- css_density_matrix for callers that cannot allocate
 *   device memory (code under HIP graph capture, tight serving loops, harnesses that
 *   forbid hipMalloc): the same computation and results, bitwise, with no workspace
 *   argument. The library's scratch is a file-scope device array of 256 MiB, one per
 *   GPU, held until the process ends; this call allocates nothing (no hipMalloc or
 *   hipFree, no allocating library routine, no events: info->t_phase_ms stays 0).
 *   Arguments as css_density_matrix without ws / ws_bytes.
 *   The pole expansion's solver takes the scratch left after the other buffers.
 *   Returns CSS_E_WORKSPACE before any device work when the buffers and 64 poles do
 *   not fit in the 256 MiB (for example 216 water molecules, 1296 orbitals, at depth
 *   40 fit; 1000 molecules do not), and after the Lanczos pass when the spectrum needs more poles
 *   than fit; CSS_E_UNSUPPORTED with CSS_SUBSPACE_EIG (the dense eigensolver
 *   allocates). Every call on one GPU
 *   uses that GPU's one scratch array: calls that overlap on a GPU (several streams
 *   or threads) race and must be serialised by the caller. The array keeps the last
 *   call's contents; each call clears what it needs.
 */
css_status css_density_matrix_noalloc(const css_csr* H, const int32_t* color, const int8_t* sign,
                                      int32_t n_colors, double mu, double kT, int32_t depth, double spin_deg,
                                      const int64_t* p_row_ptr, const int32_t* p_col, int64_t p_nnz,
                                      uint32_t flags, double* p_val, double* e_band, double* trace,
                                      css_info* info, void* stream);

/*
 * css_energy_density_matrix -- css_density_matrix together with the CSS estimate
 *   of the energy-weighted density matrix P_E = g f(H) H (the force expression
 *   of the paper's SCF section, rho_E = sum_i f(e_i) e_i |psi_i><psi_i|, taken as
 *   S^-1 H rho~ with S = I): X_E = H X, then P_E,mn = sign[n] X_E[m, colour(n)] on
 *   the same pattern, symmetrised with CSS_SYMMETRIZE. One more sparse x block
 *   product and one more gather than css_density_matrix.
 *   Arguments as css_density_matrix, and:
 *   pe_val      device double[p_nnz] out: P_E on the pattern
 *   pe_trace    host out (may be NULL): sum_m P_E,mm (the Krylov band energy up to
 *               rounding, Tr(r^T H X) = Tr(H rho~))
 *   ws          css_workspace_size(CSS_ENTRY_ENERGY_DENSITY, ...) bytes.
 *   p_val, e_band, trace and info are those css_density_matrix returns.
 */
css_status css_energy_density_matrix(const css_csr* H, const int32_t* color, const int8_t* sign,
                                     int32_t n_colors, double mu, double kT, int32_t depth,
                                     double spin_deg, const int64_t* p_row_ptr, const int32_t* p_col,
                                     int64_t p_nnz, uint32_t flags, double* p_val, double* pe_val,
                                     double* e_band, double* trace, double* pe_trace, css_info* info,
                                     void* ws, size_t ws_bytes, void* stream);

/*
 * css_inv_sqrt_overlap -- the CSS estimate of S^(-1/2) on a cutoff pattern, for a
 *   non-orthogonal basis (the overlap step that precedes H' = S^(-1/2) H S^(-1/2):
 *   S^(-1/2) taken as -1/pi Im of the integral of z^(-1/2) G_S(z), projected onto
 *   coloured probes o). The same path as css_density_matrix with S in place of H
 *   and x^(-1/2) in place of g f(x): block Lanczos on S from the probes, then
 *   F = T^(-1/2) E_1 B_0 for the projected overlap T, by the coupled Newton-Schulz
 *   iteration on T / c (c its Gershgorin upper bound; FP64 MFMA products, run until
 *   |Z Y - I| <= 1e-9 and one more step), or with CSS_SUBSPACE_EIG by dense
 *   diagonalisation T = U diag(lambda) U^T (rocSOLVER dsyevd), F = U
 *   diag(lambda^(-1/2)) U[0:b,:]^T B_0; Y = sum_j Q_j F_j, then y_mn = sign[n]
 *   Y[m, colour(n)] on the pattern (symmetrised with CSS_SYMMETRIZE).
 *   S            device CSR, symmetric positive definite (the overlap matrix)
 *   color, sign, n_colors   the probes o (css_color / css_build_probes on the
 *                overlap's cutoff)
 *   depth        Krylov blocks v^s
 *   p_row_ptr, p_col, p_nnz  the pattern S^(-1/2) is read on (device, as for
 *                css_density_matrix)
 *   flags        as css_density_matrix; CSS_SUBSPACE_EIG selects dsyevd
 *   y_val        device double[p_nnz] out: S^(-1/2) on the pattern
 *   trace        host out: sum_m y_mm
 *   s_dot        host out (may be NULL): sum over entries of S in the pattern of
 *                S_mn y_mn (an estimate of Tr S^(1/2))
 *   info         host out (may be NULL): as css_density_matrix, with
 *                trace_krylov = sum_k lambda_k^(-1/2) w_k and
 *                e_band_krylov = sum_k lambda_k^(1/2) w_k
 *   ws           css_workspace_size(CSS_ENTRY_INV_SQRT, ...) bytes, device.
 *   Errors as css_density_matrix; CSS_E_NONFINITE also when S is not positive
 *   definite (a Ritz value <= 0 with dsyevd; a non-positive Gershgorin bound or no
 *   convergence in 60 steps with Newton-Schulz). Synchronises the stream before
 *   returning.
 */
css_status css_inv_sqrt_overlap(const css_csr* S, const int32_t* color, const int8_t* sign,
                                int32_t n_colors, int32_t depth, const int64_t* p_row_ptr,
                                const int32_t* p_col, int64_t p_nnz, uint32_t flags, double* y_val,
                                double* trace, double* s_dot, css_info* info, void* ws,
                                size_t ws_bytes, void* stream);

/*
 * css_transform_hamiltonian -- S^(-1/2) and the orthogonalised Hamiltonian
 *   H' = S^(-1/2) H S^(-1/2) on a cutoff pattern, for a non-orthogonal basis (the
 *   step after Eqs.(8)-(10): H' read off S^(-1/2) H Y o^T with Y = S^(-1/2) o).
 *   First css_inv_sqrt_overlap (Y and the sparse S^(-1/2) on the pattern), then
 *   Z = S^(-1/2) (H Y) with both sparse x block products in FP64 (the sparse
 *   S^(-1/2) is the one just gathered), then h'_mn = sign[n] Z[m, colour(n)] on
 *   the pattern (symmetrised with CSS_SYMMETRIZE). Only sparse x block products.
 *   H            device CSR of S's size, FP64 or FP32 values (widened to FP64),
 *                nnz at most S's
 *   S, color, sign, n_colors, depth, p_row_ptr, p_col, flags  as
 *                css_inv_sqrt_overlap (p_nnz < 2^31)
 *   y_val        device double[p_nnz] out: S^(-1/2) on the pattern
 *   hp_val       device double[p_nnz] out: H' on the pattern
 *   y_trace      host out: sum_m y_mm
 *   hp_trace     host out (may be NULL): sum_m h'_mm
 *   info         host out (may be NULL): as css_inv_sqrt_overlap
 *   ws           css_workspace_size(CSS_ENTRY_TRANSFORM_H, n, nnz of S, ...) bytes.
 *   Errors as css_inv_sqrt_overlap; CSS_E_CSR for a malformed H. Synchronises
 *   the stream before returning.
 */
css_status css_transform_hamiltonian(const css_csr* H, const css_csr* S, const int32_t* color,
                                     const int8_t* sign, int32_t n_colors, int32_t depth,
                                     const int64_t* p_row_ptr, const int32_t* p_col, int64_t p_nnz,
                                     uint32_t flags, double* y_val, double* hp_val, double* y_trace,
                                     double* hp_trace, css_info* info, void* ws, size_t ws_bytes,
                                     void* stream);

/*
 * css_density_matrix_nonorth -- the CSS density matrix of a non-orthogonal basis
 *   (Eq.(6)): rho~ = S^(-1/2) Phi rho^K Phi^T r~ r^T, with r the probes, r~ =
 *   S^(-1/2) r, Phi the block Krylov basis of H' = S^(-1/2) H S^(-1/2) from r~
 *   (the first block Q_1 R_0 = r~ by Cholesky QR, so B_0 = R_0 is triangular) and
 *   rho^K = g f(T) (Eq.(7)) by the pole expansion of css_density_matrix with
 *   B_0 = I, then F = F_I R_0 (F is linear in B_0), or with CSS_SUBSPACE_EIG by
 *   dense diagonalisation (rocSOLVER dsyevd). Only
 *   sparse x block products: r~ = S^(-1/2) r and X = S^(-1/2) X' in FP64, the
 *   Lanczos steps on H' in the precision the flags select. Then P_mn =
 *   sign[n] X[m, colour(n)] on the pattern (symmetrised with CSS_SYMMETRIZE).
 *   Hp           device CSR of H' (css_transform_hamiltonian's values on an int32
 *                copy of the pattern's row pointers), FP64 or FP32
 *   S_isqrt      device CSR of the sparse S^(-1/2), FP64 values (nnz < 2^31)
 *   H, S         device CSRs of the original H and S (either may be NULL): for
 *                e_band = sum H_mn P_mn and n_elec = sum S_mn P_mn (= Tr(P S),
 *                the Mulliken electron count) over entries in the pattern
 *   color, sign, n_colors, mu, kT, depth, spin_deg, p_row_ptr, p_col, p_nnz  as
 *                css_density_matrix (the probes r on the density's cutoff)
 *   flags        precision and re-orthogonalisation as css_density_matrix; stored
 *                basis only (CSS_E_UNSUPPORTED with CSS_BASIS_TWOPASS);
 *                CSS_SUBSPACE_EIG selects the dense diagonalisation
 *   p_val        device double[p_nnz] out
 *   e_band       host out (NULL allowed when H is NULL)
 *   n_elec       host out (NULL allowed when S is NULL)
 *   trace        host out: sum_m P_mm
 *   info         host out (may be NULL): as css_density_matrix; trace_krylov =
 *                Tr(R_0^T [g f(T)]_11 R_0) = sum_k g f(lambda_k) |R_0^T U[0:b,k]|^2
 *                (the Krylov estimate of Tr(r~^T g f(H') r~), which is Tr(P_raw)
 *                up to rounding) and e_band_krylov the same with T g f(T)
 *   ws           css_workspace_size(CSS_ENTRY_DENSITY_NONORTH, n, nnz of H', ...)
 *   Errors as css_density_matrix; CSS_E_BREAKDOWN_AT_1 when r~ is rank deficient.
 *   Synchronises the stream before returning.
 */
css_status css_density_matrix_nonorth(const css_csr* Hp, const css_csr* S_isqrt, const css_csr* H,
                                      const css_csr* S, const int32_t* color, const int8_t* sign,
                                      int32_t n_colors, double mu, double kT, int32_t depth,
                                      double spin_deg, const int64_t* p_row_ptr, const int32_t* p_col,
                                      int64_t p_nnz, uint32_t flags, double* p_val, double* e_band,
                                      double* n_elec, double* trace, css_info* info, void* ws,
                                      size_t ws_bytes, void* stream);

/*
 * css_find_mu -- the chemical potential for a given electron count (the mu of
 *   Eq.(1) that an SCF cycle must supply): the mu at which the Krylov quadrature
 *   count N(mu) = Tr(B_0^T [g f_mu(T)]_11 B_0) = sum_k g f_mu(lambda_k) w_k (the
 *   Krylov estimate of Tr P, Eqs.(6)-(7), monotone in mu) equals n_electrons,
 *   after one block Lanczos pass as in css_density_matrix.
 *   Default: N(mu) from the pole expansion of css_density_matrix's subspace step
 *   at each trial mu, root by Chandrupatla's bracketing method (inverse quadratic
 *   interpolation where it is safe, else bisection) on the Gershgorin bracket of T widened
 *   by 50 kT, to an interval of 1e-13 max(1, |ends|).
 *   CSS_SUBSPACE_EIG (and n_colors > 128): T = U diag(lambda) U^T by rocSOLVER
 *   dsyevd, w_k = sum_c n_c U[c,k]^2, bisection on the device on
 *   [min lambda - 50 kT, max lambda + 50 kT] to the same width.
 *   H, color, sign, n_colors, kT, depth, spin_deg, flags as css_density_matrix
 *   (CSS_SYMMETRIZE has no effect).
 *   n_electrons  in (0, spin_deg * n), else CSS_E_ARG before any device work
 *   mu           host out: the chemical potential
 *   count        host out (may be NULL): the quadrature count at mu
 *   info         host out (may be NULL): depth_eff, n_colors, breakdown,
 *                min_diag_r, trace_krylov (= count), n_evals, t_phase_ms[0..2]
 *                (lanczos, spectral bounds or diagonalisation, root search) and
 *                [5] (total)
 *   ws           css_workspace_size(CSS_ENTRY_FIND_MU, ...) bytes, device.
 *   Synchronises the stream before returning.
 */
css_status css_find_mu(const css_csr* H, const int32_t* color, const int8_t* sign, int32_t n_colors,
                       double n_electrons, double kT, int32_t depth, double spin_deg, uint32_t flags,
                       double* mu, double* count, css_info* info, void* ws, size_t ws_bytes, void* stream);

/* One system of a batch (all arrays device, as for css_density_matrix). */
typedef struct {
    css_csr H;                    /* the system's Hamiltonian */
    const int32_t* color;         /* int32[H.n], colours 0..n_colors-1 */
    const int8_t* sign;           /* int8[H.n], probe signs */
    int32_t n_colors;
    double mu;                    /* the system's chemical potential */
    const int64_t* p_row_ptr;     /* pattern, as css_density_matrix */
    const int32_t* p_col;
    int64_t p_nnz;
    double* p_val;                /* out: double[p_nnz] */
    double e_band, trace;         /* out */
    css_info info;                /* out */
    css_status status;            /* out: this system's status */
} css_system;

#define CSS_MAX_BATCH_STREAMS 16

/*
 * css_density_matrix_batched -- css_density_matrix for `count` independent
 *   systems of uneven size (clusters, fragments, snapshots) in one call. Each
 *   system's result (p_val, e_band, trace, info) is bitwise the one the single-
 *   system call gives; kT, depth, spin_deg and flags are shared. The systems run
 *   side by side on `concurrency` (1..16) library-created streams of default
 *   priority, largest first, so that the N-independent, latency-bound phases of
 *   small systems overlap. Work starts after the work already queued on
 *   `stream`; all of it is complete when the call returns.
 *   ws        device, css_batched_workspace_size(...) bytes: one slice per stream.
 *   Returns the first failing system's status (every system's own status is in
 *   its struct), CSS_E_UNSUPPORTED with CSS_SUBSPACE_EIG.
 */
css_status css_density_matrix_batched(css_system* systems, int32_t count, double kT, int32_t depth,
                                      double spin_deg, uint32_t flags, int32_t concurrency,
                                      void* ws, size_t ws_bytes, void* stream);

/* Workspace bytes for css_density_matrix_batched (host only). */
css_status css_batched_workspace_size(const css_system* systems, int32_t count, int32_t depth,
                                      uint32_t flags, int32_t concurrency, size_t* bytes);

/* One colouring of a batch: the arguments of css_color, outputs included. */
typedef struct {
    const double* xyz;            /* device, n x 3 */
    int32_t n;
    double box[3];
    double r_cut;
    int32_t* color;               /* device int32[n] out */
    int32_t n_colors;             /* out */
    int64_t* p_row_ptr;           /* device int64[n+1] out */
    int32_t* p_col;               /* device int32[p_nnz] out (capacity p_nnz on input) */
    int64_t p_nnz;                /* in: capacity of p_col; out: entries */
    int32_t rounds;               /* out */
    css_status status;            /* out: CSS_E_CAPACITY if p_col was too small */
} css_color_job;

/*
 * css_color_batched -- css_color for `count` independent geometries in one call,
 *   side by side on `concurrency` library streams as css_density_matrix_batched.
 *   Each job's outputs are those css_color gives for it alone. A job whose
 *   capacity is too small reports CSS_E_CAPACITY (with the entries needed in
 *   p_nnz) without affecting the others.
 *   ws  device, css_color_batched_workspace_size(...) bytes.
 */
css_status css_color_batched(css_color_job* jobs, int32_t count, int32_t concurrency, void* ws,
                             size_t ws_bytes, void* stream);
css_status css_color_batched_workspace_size(const css_color_job* jobs, int32_t count,
                                            int32_t concurrency, size_t* bytes);

/*
 * css_workspace_size -- bytes of workspace an entry point needs.
 *   entry  CSS_ENTRY_*; the other arguments as they will be passed
 *   (nnz = H's nnz, or for CSS_ENTRY_COLOR unused; CSS_ENTRY_SPMM uses n and
 *   nnz only). For CSS_ENTRY_LANCZOS / CSS_ENTRY_DENSITY the size holds for H's
 *   values in either FP32 or FP64 (values not in the precision the flags select
 *   are converted into the workspace).
 */
css_status css_workspace_size(int32_t entry, int32_t n, int64_t nnz, int32_t n_colors,
                              int32_t depth, uint32_t flags, size_t* bytes);

/*
 * css_fermi_poles -- the rational approximation of the Fermi function used for
 *   the subspace step (host only, no device work). With y = (x - mu)/(2 kT),
 *   f(x) = 1/2 - (1/2) sum_p c_p y / (1 + kappa_p^2 y^2): the Lambert continued
 *   fraction of tanh truncated at `depth` (even, 2..512) levels. Returns the
 *   positive kappa_p and weight_p = c_p / (2 kappa_p) (arrays of depth/2, host,
 *   either may be NULL) and their count.
 */
css_status css_fermi_poles(int32_t depth, double* kappa, double* weight, int32_t* npoles);

/*
 * Launch choices (the library's tuning knobs, for an autotuner). Process-wide, read
 * when a kernel is launched; zero fields select the built-in defaults. No choice
 * changes the arithmetic of the method, only the launch shape and hence the order
 * in which FP32 partial sums are added (results stay deterministic for a fixed
 * tuning); cholqr2_series selects between two evaluations of the second CholQR
 * factor that agree to below the working precision's rounding.
 *   spmm_kernel  sparse x block product: 0 automatic (the 16-row grouped MFMA kernel
 *                where H's row groups are dense enough, else the row-parallel CSR
 *                kernel), 1 16-row groups, 2 the CSR kernel
 *   spmm_run     row groups per XCD run of the grouped kernel (0 = 512)
 *   spmm_depth   k-steps in flight per wavefront of the grouped kernel: 0 (= 4), 4, 8
 *   gram_chunks  FP32 split Gram products: row chunks sized for about this many
 *                work-groups per compute unit, 0 (= 1), 1, 2, 4
 *   update_rows  FP32 split block updates: rows per work-group, 0 (= 128), 64, 128
 *   cholqr2_series  second Cholesky QR pass (CSS_CHOLQR2), whose Gram is I + E with E
 *                of the first pass's loss of orthogonality: 0 (= 1), 1 a second-order
 *                series in E when max|E| <= 2e-6 (FP64) or 1e-4 (FP32), so that the
 *                neglected |E|^3 is below rounding, else the factorisation; 2 always the
 *                factorisation
 */
typedef struct {
    int32_t spmm_kernel;
    int32_t spmm_run;
    int32_t spmm_depth;
    int32_t gram_chunks;
    int32_t update_rows;
    int32_t cholqr2_series;
    int32_t reserved[2];
} css_tuning;

/* Sets (t != NULL) or resets to the defaults (t == NULL) the process-wide tuning.
 * CSS_E_ARG for an out-of-range field. Not to be called while another thread is
 * inside the library. */
css_status css_set_tuning(const css_tuning* t);
css_status css_get_tuning(css_tuning* t);

/*
 * css_spmm_time -- average device time of `reps` launches of W = H V (css_spmm) with
 *   the launch choices `cfg` (NULL: the current tuning), measured with HIP events on
 *   `stream` after one untimed launch; for the autotuner. Arguments as css_spmm;
 *   avg_ms host out. Synchronises the stream.
 */
css_status css_spmm_time(const css_csr* H, const void* V, void* W, int32_t b, int32_t ld, const void* ws,
                         size_t ws_bytes, const css_tuning* cfg, int32_t reps, float* avg_ms, void* stream);

/* Leading dimension the library uses for blocks of b columns. */
int32_t css_block_ld(int32_t n_colors);

/* Static text for a status code. */
const char* css_status_string(css_status s);

#ifdef __cplusplus
}
#endif

#endif /* CSS_H */
