"""Oracle: reconstruction, extraction and the whole density-matrix pipeline.

Test infrastructure only: see the package docstring.

Definitions followed:
* Eq.(3): rho~ = X r^T, so the estimate of P_mn is X[m, :] r[n, :]^T =
  s_n X[m, c(n)] (only the probe of n's colour is nonzero at n);
* Eq.(6): X = Phi F = sum_j Q_j F_j, F_j the j-th block of rows of F;
* the text around Eq.(2) and Fig.1(a): P is read off only on the pairs closer
  than the cutoff (the colouring's conflict graph plus the diagonal);
* the orbital energy sum E = Tr(H rho) quoted with Fig.2(a).

Readings:
* the raw estimate is not symmetric; by default P <- (P + P^T)/2 on the
  (symmetric) pattern. The largest raw asymmetry is reported;
* E_band = sum over entries (m, n) present in both H and the pattern of
  H_mn P_mn; trace = sum_m P_mm; no value is dropped by a threshold.
"""
from __future__ import annotations

import numpy as np

from .lanczos import REORTH_FULL, assemble_T, block_lanczos
from .subspace import contraction, eig_subspace, fermi, inv_sqrt_contraction


def reconstruct_X(Q: list, F: np.ndarray) -> np.ndarray:
    b = Q[0].shape[1]
    X = np.zeros_like(Q[0])
    for j, Qj in enumerate(Q):
        X += Qj @ F[j * b:(j + 1) * b, :]
    return X


def pattern_rows(p_row_ptr: np.ndarray) -> np.ndarray:
    n = p_row_ptr.shape[0] - 1
    return np.repeat(np.arange(n), np.diff(p_row_ptr))


def gather_raw(X: np.ndarray, color, sign, p_row_ptr, p_col) -> np.ndarray:
    rows = pattern_rows(p_row_ptr)
    cols = p_col.astype(np.int64)
    return sign[cols].astype(np.float64) * X[rows, color[cols]]


def symmetrize(p_raw: np.ndarray, p_row_ptr, p_col) -> np.ndarray:
    """(P + P^T)/2 on a symmetric pattern (looked up by binary search)."""
    rows = pattern_rows(p_row_ptr)
    cols = p_col.astype(np.int64)
    n = p_row_ptr.shape[0] - 1
    key = rows * n + cols
    tkey = cols * n + rows
    pos = np.searchsorted(key, tkey)       # rows sorted, cols sorted within rows
    if np.any(pos >= key.size) or np.any(key[np.minimum(pos, key.size - 1)] != tkey):
        raise ValueError("pattern is not symmetric")
    return 0.5 * (p_raw + p_raw[pos])


def trace_of(p_val, p_row_ptr, p_col) -> float:
    rows = pattern_rows(p_row_ptr)
    return float(np.sum(p_val[rows == p_col]))


def band_energy(H, p_val, p_row_ptr, p_col) -> float:
    """sum over (m,n) in both patterns of H_mn P_mn."""
    Hc = H.tocsr()
    rows = pattern_rows(p_row_ptr)
    h = np.asarray(Hc[rows, p_col.astype(np.int64)]).ravel()
    return float(np.sum(h * p_val))


def idempotency_defect(p_val, p_row_ptr, p_col, spin_deg=2.0) -> float:
    """Tr P - ||P||_F^2 / g over the pattern. For symmetric P this is Tr P - Tr(P^2)/g;
    for the Fermi-Dirac operator P = g f(H) of Eq.(1) it equals g sum_k f_k (1 - f_k),
    zero when P/g is a projector (an insulator at zero temperature) and small at
    small kT in a gapped system."""
    return trace_of(p_val, p_row_ptr, p_col) - float(np.sum(np.asarray(p_val) ** 2)) / spin_deg


def density_matrix(H, color, sign, n_colors, mu, kT, depth, p_row_ptr, p_col,
                   spin_deg=2.0, reorth=REORTH_FULL, cholqr2=True, symmetrize_p=True,
                   eig_driver="evd"):
    """The whole CSS estimate of P on the pattern; returns a dict of results."""
    color = np.asarray(color)
    sign = np.asarray(sign)
    lz = block_lanczos(H, color, sign, n_colors, depth, reorth=reorth, cholqr2=cholqr2)
    T = assemble_T(lz.A, lz.B)
    lam, U = eig_subspace(T, driver=eig_driver)
    F, trace_k, e_k = contraction(lam, U, lz.b0, mu, kT, spin_deg)
    X = reconstruct_X(lz.Q, F)
    p_raw = gather_raw(X, color, sign, p_row_ptr, p_col)
    p_sym = symmetrize(p_raw, p_row_ptr, p_col)
    p_val = p_sym if symmetrize_p else p_raw
    return {
        "p_val": p_val, "p_raw": p_raw, "X": X, "F": F, "lam": lam, "T": T,
        "lanczos": lz, "v_eff": lz.v_eff, "breakdown": lz.breakdown,
        "trace": trace_of(p_val, p_row_ptr, p_col),
        "e_band": band_energy(H, p_val, p_row_ptr, p_col),
        "idem": idempotency_defect(p_val, p_row_ptr, p_col, spin_deg),
        "trace_krylov": trace_k, "e_band_krylov": e_k,
        "asym_max": float(np.max(np.abs(p_raw - p_sym))) if p_raw.size else 0.0,
    }


def energy_density_matrix(H, res: dict, color, sign, p_row_ptr, p_col, symmetrize_p=True) -> dict:
    """The CSS estimate of the energy-weighted density matrix, rho~_E = S^-1 H rho~
    (the force expression of the paper's SCF section) with S = I: X_E = H X from the
    X of `density_matrix` (its result dict `res`), read off the pattern as P is."""
    XE = H @ res["X"]
    pe_raw = gather_raw(XE, np.asarray(color), np.asarray(sign), p_row_ptr, p_col)
    pe_val = symmetrize(pe_raw, p_row_ptr, p_col) if symmetrize_p else pe_raw
    return {"pe_val": pe_val, "pe_raw": pe_raw, "XE": XE, "pe_trace": trace_of(pe_val, p_row_ptr, p_col)}


# ---- references used to separate the method error from the parity error ----

def dense_fermi_dm(H, mu, kT, spin_deg=2.0) -> np.ndarray:
    """g f(H) from dense diagonalisation (Eq.(1) with S = I)."""
    Hd = H.toarray() if hasattr(H, "toarray") else np.asarray(H)
    lam, U = np.linalg.eigh(Hd)
    return (U * (spin_deg * fermi(lam, mu, kT))[None, :]) @ U.T


def dense_energy_fermi_dm(H, mu, kT, spin_deg=2.0) -> np.ndarray:
    """sum_i g f(e_i) e_i psi_i psi_i^T from dense diagonalisation (S = I)."""
    Hd = H.toarray() if hasattr(H, "toarray") else np.asarray(H)
    lam, U = np.linalg.eigh(Hd)
    return (U * (spin_deg * fermi(lam, mu, kT) * lam)[None, :]) @ U.T


def css_exact_X(P_dense: np.ndarray, color, sign, n_colors) -> np.ndarray:
    """X = g f(H) r with no Krylov truncation (Eq.(2)-(3) alone)."""
    from .probes import probe_block
    return P_dense @ probe_block(np.asarray(color), np.asarray(sign), n_colors)


def mu_midgap_dense(H, n_electrons: int, spin_deg=2.0) -> float:
    Hd = H.toarray() if hasattr(H, "toarray") else np.asarray(H)
    eps = np.linalg.eigvalsh(Hd)
    K = int(round(n_electrons / spin_deg))
    return 0.5 * (eps[K - 1] + eps[K])


def krylov_weights(U: np.ndarray, b0: np.ndarray) -> np.ndarray:
    b = b0.shape[0]
    return (b0[:, None] ** 2 * U[:b, :] ** 2).sum(axis=0)


def mu_krylov_bisection(lam: np.ndarray, w: np.ndarray, n_electrons: float, kT: float,
                        spin_deg=2.0, tol=1e-13) -> float:
    """mu at which the Krylov quadrature trace sum_k g f(lambda_k) w_k equals N_e.

    Used to choose mu for systems too large for dense diagonalisation; the
    trace is monotone in mu, so plain bisection on [min lambda - 50 kT,
    max lambda + 50 kT] converges.
    """
    lo, hi = float(lam.min()) - 50 * kT, float(lam.max()) + 50 * kT
    while hi - lo > tol * max(1.0, abs(lo), abs(hi)):
        mid = 0.5 * (lo + hi)
        if np.sum(spin_deg * fermi(lam, mid, kT) * w) < n_electrons:
            lo = mid
        else:
            hi = mid
    return 0.5 * (lo + hi)


def find_mu(H, color, sign, n_colors, n_electrons, kT, depth, spin_deg=2.0, reorth=REORTH_FULL,
            cholqr2=True) -> dict:
    """The mu of Eq.(1) for a given electron count, from the Krylov quadrature of
    Tr P (Eqs.(6)-(7)): block Lanczos, the eigenpairs of T, the weights
    w_k = sum_c n_c U[c,k]^2, then bisection on sum_k g f_mu(lambda_k) w_k."""
    lz = block_lanczos(H, np.asarray(color), np.asarray(sign), n_colors, depth, reorth=reorth, cholqr2=cholqr2)
    lam, U = eig_subspace(assemble_T(lz.A, lz.B))
    w = krylov_weights(U, lz.b0)
    mu = mu_krylov_bisection(lam, w, n_electrons, kT, spin_deg)
    return {"mu": mu, "lam": lam, "w": w, "v_eff": lz.v_eff,
            "count": float(np.sum(spin_deg * fermi(lam, mu, kT) * w))}


def krylov_count(lam, w, mu, kT, spin_deg=2.0) -> float:
    """sum_k g f_mu(lambda_k) w_k."""
    return float(np.sum(spin_deg * fermi(lam, mu, kT) * w))


def krylov_count_slope(lam, w, mu, kT, spin_deg=2.0) -> float:
    """d/dmu of the quadrature count: (g/kT) sum_k f (1 - f) w_k."""
    f = fermi(lam, mu, kT)
    return float(np.sum(spin_deg * f * (1.0 - f) * w) / kT)


def inv_sqrt_matrix(S, color, sign, n_colors, depth, p_row_ptr, p_col, reorth=REORTH_FULL, cholqr2=True,
                    symmetrize_p=True) -> dict:
    """The CSS estimate of S^(-1/2) on the pattern (the overlap step of the
    non-orthogonal case): block Lanczos on S from the probes o, the projected
    overlap T = U diag(lambda) U^T, Y = Psi U diag(lambda^(-1/2)) U^T Psi^T o,
    read off as P is: S^(-1/2)_mn = o_n-component of Y[m]."""
    color = np.asarray(color)
    sign = np.asarray(sign)
    lz = block_lanczos(S, color, sign, n_colors, depth, reorth=reorth, cholqr2=cholqr2)
    T = assemble_T(lz.A, lz.B)
    lam, U = eig_subspace(T)
    F, trace_k, half_k = inv_sqrt_contraction(lam, U, lz.b0)
    Y = reconstruct_X(lz.Q, F)
    y_raw = gather_raw(Y, color, sign, p_row_ptr, p_col)
    y_sym = symmetrize(y_raw, p_row_ptr, p_col)
    y_val = y_sym if symmetrize_p else y_raw
    return {"y_val": y_val, "y_raw": y_raw, "Y": Y, "lam": lam, "v_eff": lz.v_eff, "lanczos": lz,
            "trace": trace_of(y_val, p_row_ptr, p_col), "trace_krylov": trace_k,
            "s_dot": band_energy(S, y_val, p_row_ptr, p_col), "half_krylov": half_k}


def transform_hamiltonian(H, S, color, sign, n_colors, depth, p_row_ptr, p_col, reorth=REORTH_FULL,
                          cholqr2=True, symmetrize_p=True) -> dict:
    """H' = S^(-1/2) H S^(-1/2) on the pattern, read off S^(-1/2) H Y o^T with
    Y = S^(-1/2) o from `inv_sqrt_matrix` and the left S^(-1/2) the sparse estimate
    on the pattern (the non-orthogonal step after Eqs.(8)-(10))."""
    import scipy.sparse as sp
    r = inv_sqrt_matrix(S, color, sign, n_colors, depth, p_row_ptr, p_col, reorth=reorth, cholqr2=cholqr2,
                        symmetrize_p=symmetrize_p)
    n = len(p_row_ptr) - 1
    S_half = sp.csr_matrix((r["y_val"], np.asarray(p_col, dtype=np.int64), np.asarray(p_row_ptr, dtype=np.int64)),
                           shape=(n, n))
    Z = S_half @ (H @ r["Y"])
    h_raw = gather_raw(Z, color, sign, p_row_ptr, p_col)
    h_sym = symmetrize(h_raw, p_row_ptr, p_col)
    h_val = h_sym if symmetrize_p else h_raw
    return {"y_val": r["y_val"], "hp_val": h_val, "hp_raw": h_raw, "Z": Z, "v_eff": r["v_eff"],
            "y_trace": r["trace"], "hp_trace": trace_of(h_val, p_row_ptr, p_col)}


def density_matrix_nonorth(Hp, S_isqrt, color, sign, n_colors, mu, kT, depth, p_row_ptr, p_col, spin_deg=2.0,
                           H=None, S=None, reorth=REORTH_FULL, cholqr2=True, symmetrize_p=True) -> dict:
    """The CSS density matrix of a non-orthogonal basis (Eq.(6)):
    rho~ = S^(-1/2) Phi rho^K Phi^T r~ r^T, r~ = S^(-1/2) r, Phi the block Krylov
    basis of H' from r~ (Q_1 R_0 = r~), rho^K = g f(T) from the eigenpairs of T
    (Eq.(7)). Hp and S_isqrt are the sparse H' and S^(-1/2)."""
    from .probes import probe_block
    color = np.asarray(color)
    sign = np.asarray(sign)
    r = probe_block(color, sign, n_colors)
    r_t = S_isqrt @ r
    lz = block_lanczos(Hp, color, sign, n_colors, depth, reorth=reorth, cholqr2=cholqr2, start=r_t)
    T = assemble_T(lz.A, lz.B)
    lam, U = eig_subspace(T)
    b = n_colors
    occ = spin_deg * fermi(lam, mu, kT)
    UR = U[:b, :].T @ lz.r0                      # U[0:b,:]^T R_0  (n_T x b)
    F = (U * occ[None, :]) @ UR                  # U g f(Lambda) U[0:b,:]^T R_0
    w = (UR ** 2).sum(axis=1)
    Xp = reconstruct_X(lz.Q, F)
    X = S_isqrt @ Xp
    p_raw = gather_raw(X, color, sign, p_row_ptr, p_col)
    p_sym = symmetrize(p_raw, p_row_ptr, p_col)
    p_val = p_sym if symmetrize_p else p_raw
    out = {"p_val": p_val, "p_raw": p_raw, "X": X, "lam": lam, "v_eff": lz.v_eff, "lanczos": lz,
           "trace": trace_of(p_val, p_row_ptr, p_col), "trace_krylov": float(np.sum(occ * w)),
           "e_band_krylov": float(np.sum(lam * occ * w))}
    if H is not None:
        out["e_band"] = band_energy(H, p_val, p_row_ptr, p_col)
    if S is not None:
        out["n_elec"] = band_energy(S, p_val, p_row_ptr, p_col)
    return out


def dense_fermi_dm_generalized(H, S, mu, kT, spin_deg=2.0) -> np.ndarray:
    """g f of the generalised problem H c = e S c with S-orthonormal c:
    rho = sum_i g f(e_i) c_i c_i^T (scipy's generalised symmetric eigensolver)."""
    import scipy.linalg as sla
    Hd = H.toarray() if hasattr(H, "toarray") else np.asarray(H)
    Sd = S.toarray() if hasattr(S, "toarray") else np.asarray(S)
    e, C = sla.eigh(Hd, Sd)
    return (C * (spin_deg * fermi(e, mu, kT))[None, :]) @ C.T

