"""Oracle: the Fermi-Dirac density matrix inside the Krylov subspace.

Test infrastructure only: see the package docstring.

Definitions followed:
* Eq.(1): f(z) = 1 / (exp(beta (z - mu)) + 1), beta = 1/kT; the contour
  integral of f times the resolvent of a Hermitian matrix equals the matrix
  function f of it.
* Eq.(6)-(7): rho^K is that integral with H^K in place of H, computed (as the
  paper does) by exact diagonalisation H^K = U diag(lambda) U^T, so
  rho^K = U diag(f(lambda)) U^T.
* Eq.(6): the estimate needs rho^K only applied to Phi^T r = E_1 B_0 (the
  probes live in the first block), so F = g * U diag(f(lambda)) U[0:b,:]^T B_0.

Readings:
* spin degeneracy g = 2 (closed shell; 8 electrons on 6 orbitals per water);
* f is evaluated without overflow: for x = (lambda - mu)/kT > 0 as
  e^-x / (1 + e^-x), otherwise 1 / (1 + e^x);
* Krylov quadrature (Gauss-type) estimates of the trace and band energy:
  w_k = sum_c n_c U[c,k]^2, trace_K = sum_k g f(lambda_k) w_k,
  E_K = sum_k lambda_k g f(lambda_k) w_k. In exact arithmetic they equal
  Tr(P_raw) and Tr(H P_raw) of the unsymmetrised estimate.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla


def fermi(x: np.ndarray, mu: float, kT: float) -> np.ndarray:
    t = (np.asarray(x, dtype=np.float64) - mu) / kT
    out = np.empty_like(t)
    pos = t > 0
    e = np.exp(-t[pos])
    out[pos] = e / (1.0 + e)
    out[~pos] = 1.0 / (1.0 + np.exp(t[~pos]))
    return out


def eig_subspace(T: np.ndarray, driver: str = "evd"):
    return sla.eigh(T, driver=driver)


def contraction(lam: np.ndarray, U: np.ndarray, b0: np.ndarray, mu: float, kT: float,
                spin_deg: float = 2.0):
    """F (n_T x b), trace_K, E_K."""
    b = b0.shape[0]
    occ = spin_deg * fermi(lam, mu, kT)
    Utop = U[:b, :]
    F = (U * occ[None, :]) @ Utop.T
    F = F * b0[None, :]
    w = (b0[:, None] ** 2 * Utop ** 2).sum(axis=0)
    trace_k = float(np.sum(occ * w))
    e_k = float(np.sum(lam * occ * w))
    return F, trace_k, e_k


def inv_sqrt_contraction(lam: np.ndarray, U: np.ndarray, b0: np.ndarray):
    """The same contraction for f(x) = x^(-1/2) (the Krylov estimate of S^(-1/2) applied
    to the probes, from the eigenpairs of the projected overlap): F (n_T x b),
    the quadrature trace sum_k lambda_k^(-1/2) w_k and sum_k lambda_k^(1/2) w_k.
    The projected matrix must be positive definite."""
    if np.any(lam <= 0.0):
        raise ValueError("projected overlap is not positive definite")
    b = b0.shape[0]
    occ = 1.0 / np.sqrt(lam)
    Utop = U[:b, :]
    F = (U * occ[None, :]) @ Utop.T
    F = F * b0[None, :]
    w = (b0[:, None] ** 2 * Utop ** 2).sum(axis=0)
    return F, float(np.sum(occ * w)), float(np.sum(np.sqrt(lam) * w))

