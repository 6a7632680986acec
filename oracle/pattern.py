"""Oracle: the conflict graph of the colouring (also the sparsity pattern of P).

Test infrastructure only: see the package docstring.

Definition followed (the text around Eq.(2), which introduces the colouring):
two orbitals m, n must receive different colours when the spatial distance
d_mn between them is within the cutoff d_cut. The density matrix is extracted
on exactly those pairs, so the same graph, with the diagonal added, is the
sparsity pattern of P.

Readings (the paper leaves these open):
* distance is measured between the orbitals' centres (their atoms), with the
  minimum-image convention in periodic directions,
  dx <- dx - L * rint(dx / L) with rint rounding half to even;
* d^2 = (dx*dx + dy*dy) + dz*dz, each product and sum rounded separately
  (no fused multiply-add), compared as d^2 <= r_cut*r_cut ("within");
* orbitals at the same centre are always in conflict (distance 0).
"""
from __future__ import annotations

import numpy as np


def pair_d2(xyz_m: np.ndarray, xyz_n: np.ndarray, box: np.ndarray) -> np.ndarray:
    """Squared minimum-image distance between points m (k,3) and n (k,3)."""
    d = xyz_n - xyz_m
    for k in range(3):
        if box[k] > 0:
            d[:, k] = d[:, k] - box[k] * np.rint(d[:, k] / box[k])
    return d[:, 0] * d[:, 0] + d[:, 1] * d[:, 1] + d[:, 2] * d[:, 2]


def _candidate_pairs(xyz: np.ndarray, box: np.ndarray, r_cut: float):
    """A superset of all conflicting pairs (m < n), from a k-d tree.

    The k-d tree only proposes candidates with a slightly enlarged radius; the
    decision is taken by `pair_d2` on the original coordinates.
    """
    from scipy.spatial import cKDTree
    n = xyz.shape[0]
    periodic = np.all(box > 0)
    r_search = r_cut * (1.0 + 1e-9) + 1e-9
    if periodic:
        L = box.astype(np.float64)
        wrapped = np.mod(xyz, L)
        wrapped[wrapped >= L] = 0.0
        tree = cKDTree(wrapped, boxsize=L)
    elif np.any(box > 0):
        # mixed periodic / open: fall back to all pairs
        mi, ni = np.triu_indices(n, 1)
        return mi.astype(np.int64), ni.astype(np.int64)
    else:
        tree = cKDTree(xyz)
    pairs = tree.query_pairs(r_search, output_type="ndarray")
    if pairs.size == 0:
        return np.zeros(0, np.int64), np.zeros(0, np.int64)
    return pairs[:, 0].astype(np.int64), pairs[:, 1].astype(np.int64)


def conflict_pattern(xyz: np.ndarray, box, r_cut: float):
    """Pattern of P: rows sorted, diagonal included.

    Returns (row_ptr int64[n+1], col int32[nnz], deg int32[n]) where deg counts
    conflicting partners excluding the orbital itself.
    """
    xyz = np.asarray(xyz, dtype=np.float64)
    box = np.asarray(box, dtype=np.float64)
    n = xyz.shape[0]
    if n == 0:
        return np.zeros(1, np.int64), np.zeros(0, np.int32), np.zeros(0, np.int32)
    m_idx, n_idx = _candidate_pairs(xyz, box, r_cut)
    if m_idx.size:
        keep = pair_d2(xyz[m_idx], xyz[n_idx], box) <= r_cut * r_cut
        m_idx, n_idx = m_idx[keep], n_idx[keep]
    rows = np.concatenate([m_idx, n_idx, np.arange(n)])
    cols = np.concatenate([n_idx, m_idx, np.arange(n)])
    order = np.lexsort((cols, rows))
    rows, cols = rows[order], cols[order]
    counts = np.bincount(rows, minlength=n)
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    return row_ptr, cols.astype(np.int32), (counts - 1).astype(np.int32)
