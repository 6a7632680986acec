"""Oracle: block Lanczos projection of H onto the block Krylov space of the probes.

Test infrastructure only: see the package docstring.

Definition followed: after Eq.(4) the paper builds, with the block Lanczos
process of Golub and Underwood, an orthonormal basis Phi of the block Krylov
space K^v(H, r) = span{r, H r, ..., H^(v-1) r} and projects H onto it,
H^K = Phi^T H Phi. With an orthogonal basis (S = I) H' = H and r~ = r.

The block three-term recurrence (exact arithmetic):
    H Q_j = Q_{j-1} B_{j-1}^T + Q_j A_j + Q_{j+1} B_j,   Q_0 = 0,
so Phi = [Q_1 .. Q_k] and H^K is block tridiagonal with A_j on the diagonal,
B_j below it and B_j^T above it.

Readings (the paper gives no detail of its block Lanczos):
* depth v counts block powers (v blocks of b columns); the number of blocks
  actually built is v_eff = min(v, floor(N / b)), fixed before any floating
  point, and smaller only on breakdown;
* one step: W = H Q_j - Q_{j-1} B_{j-1}^T; A_j = Q_j^T W symmetrised as
  (A + A^T)/2; W <- W - Q_j A_j;
* re-orthogonalisation: "full" repeats classical Gram-Schmidt once against
  Q_1..Q_j, "local" against Q_{j-1}, Q_j only, "alternate" does the full pass
  on the steps j = 0, 2, 4, ... (counting from 0) and the local pass on the
  others, "none" skips it; the symmetrised coefficient against Q_j is added to
  A_j, the others are dropped;
* W = Q_{j+1} B_j by Cholesky QR: G = W^T W = R^T R (R upper, positive
  diagonal), Q_{j+1} = W R^-1, B_j = R; with CholQR2 the factorisation is
  repeated once on Q_{j+1} and B_j = R_2 R;
* breakdown: the Cholesky factorisation fails or min diag R <= 1e-10 ||H||_inf;
  the recurrence then stops with v_eff = j.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import scipy.linalg as sla

from .probes import first_block

REORTH_NONE, REORTH_LOCAL, REORTH_FULL, REORTH_ALTERNATE = "none", "local", "full", "alternate"
BREAKDOWN_REL = 1e-10


@dataclass
class LanczosResult:
    A: list            # v_eff blocks, b x b
    B: list            # v_eff - 1 blocks, b x b, upper triangular
    Q: list            # v_eff blocks, N x b
    b0: np.ndarray     # diag of B_0 (probes as the first block), else None
    v_eff: int
    breakdown: bool
    min_diag_r: float  # smallest diag of the first Cholesky factor over all steps
    r0: np.ndarray = None   # B_0 = R_0, upper triangular, when a start block is given


def inf_norm(H) -> float:
    return float(np.max(np.abs(H).sum(axis=1))) if H.shape[0] else 0.0


def _cholesky_upper(G: np.ndarray):
    """R upper with G = R^T R, or None when G is not numerically positive definite."""
    try:
        return sla.cholesky(G, lower=False)
    except np.linalg.LinAlgError:
        return None


def block_lanczos(H, color, sign, n_colors: int, depth: int,
                  reorth: str = REORTH_FULL, cholqr2: bool = True, start=None) -> LanczosResult:
    """start: an N x b first block (the non-orthogonal case's r~ = S^(-1/2) r); its
    QR with a positive-diagonal R_0 (numpy's Householder QR, signs fixed) gives Q_1
    and B_0 = R_0. Otherwise the first block is the normalised probes."""
    N = H.shape[0]
    b = n_colors
    v_max = min(depth, N // b)
    if v_max < 1:
        raise ValueError("depth must be >= 1 and n_colors <= N")
    r0 = None
    if start is None:
        Q1, b0 = first_block(np.asarray(color), np.asarray(sign), b)
    else:
        Q1, r0 = np.linalg.qr(np.asarray(start, dtype=np.float64))
        d = np.sign(np.diag(r0))
        d[d == 0] = 1.0
        Q1, r0, b0 = Q1 * d[None, :], r0 * d[:, None], None
    tau = BREAKDOWN_REL * inf_norm(H)

    Qs, As, Bs = [Q1], [], []
    breakdown = False
    min_diag = np.inf
    for j in range(v_max):
        Qj = Qs[j]
        W = H @ Qj
        if j > 0:
            W = W - Qs[j - 1] @ Bs[j - 1].T
        A = Qj.T @ W
        A = 0.5 * (A + A.T)
        W = W - Qj @ A
        if reorth not in (REORTH_NONE, REORTH_FULL, REORTH_LOCAL, REORTH_ALTERNATE):
            raise ValueError(f"unknown re-orthogonalisation {reorth!r}")
        if reorth != REORTH_NONE:
            full = reorth == REORTH_FULL or (reorth == REORTH_ALTERNATE and j % 2 == 0)
            basis = Qs if full else Qs[max(0, j - 1):]
            coeff = [Qi.T @ W for Qi in basis]
            for Qi, C in zip(basis, coeff):
                W = W - Qi @ C
            A = A + 0.5 * (coeff[-1] + coeff[-1].T)
        As.append(A)
        if j == v_max - 1:
            break
        R = _cholesky_upper(W.T @ W)
        if R is not None:
            d = float(np.min(np.diag(R)))
            min_diag = min(min_diag, d)
        if R is None or d <= tau:
            breakdown = True
            break
        Qn = sla.solve_triangular(R, W.T, trans="T", lower=False).T     # W R^-1
        if cholqr2:
            R2 = _cholesky_upper(Qn.T @ Qn)
            if R2 is None:
                breakdown = True
                break
            Qn = sla.solve_triangular(R2, Qn.T, trans="T", lower=False).T
            R = R2 @ R
        Bs.append(R)
        Qs.append(Qn)
    v_eff = len(As)
    return LanczosResult(As, Bs, Qs[:v_eff], b0, v_eff, breakdown,
                         float(min_diag) if np.isfinite(min_diag) else float("nan"), r0)


def assemble_T(A: list, B: list) -> np.ndarray:
    """Block tridiagonal H^K: A_j on the diagonal, B_j below, B_j^T above."""
    k = len(A)
    b = A[0].shape[0]
    T = np.zeros((k * b, k * b))
    for j in range(k):
        T[j * b:(j + 1) * b, j * b:(j + 1) * b] = A[j]
    for j in range(k - 1):
        T[(j + 1) * b:(j + 2) * b, j * b:(j + 1) * b] = B[j]
        T[j * b:(j + 1) * b, (j + 1) * b:(j + 2) * b] = B[j].T
    return T
