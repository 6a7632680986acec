"""Seeded synthetic inputs: water-like boxes and an orthogonal tight-binding H.

This module makes the workloads the density-matrix path is run on. It holds
no step of the method itself (no distance predicate for the colouring, no
colouring, no probes, no Krylov arithmetic): it only lays out molecules and
fills a sparse symmetric Hamiltonian. Both the oracle's tests and the GPU path
take their inputs from here, and nothing else is shared between them.

The paper runs DFTB-2 water with 6 atomic orbitals per molecule in periodic
supercells at liquid density. Its parameter sets are not available, so a
stand-in with the same shapes is generated:

* geometry: M molecules on the first M sites of a seeded permutation of a
  ceil(M^(1/3))^3 grid in a periodic cube of edge 31.0*(M/1000)^(1/3) Angstrom
  (about 1 g/cm^3), uniform random rotation (unit quaternion from four
  normals), uniform jitter of +-0.2 Angstrom per axis; O-H 0.9572 Angstrom,
  H-O-H 104.52 degrees;
* orbitals, molecule-major in grid order: O s, O px, O py, O pz, H1 s, H2 s;
* onsite energies O_s -1.0, O_p -0.5, H_s -0.3 Ha plus Gaussian noise of
  standard deviation 0.01 Ha on each diagonal element;
* hopping between orbitals on different atoms A, B closer than 5 Angstrom
  (minimum image): t(r) * g_a(u) * g_b(-u), t(r) = -0.4 exp(-r / 1 Angstrom),
  u the unit vector from A to B, g_s = 1 and g_p = the p orbital's direction
  cosine along its argument (sigma-only Slater-Koster); same-atom
  off-diagonal entries are stored as explicit zeros so that the sparsity
  pattern is purely geometric.

H is returned as CSR with int32 column indices sorted within each row.

For the non-orthogonal case an overlap matrix S of the same pattern is
generated too (`overlap_s`, `water_overlap`): 1 on the diagonal and a
positive two-centre term with the same angular factors as the hopping.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

OH_BOND = 0.9572          # Angstrom
HOH_ANGLE_DEG = 104.52    # degrees
EDGE_PER_1000 = 31.0      # Angstrom, cube edge holding 1000 molecules
JITTER = 0.2              # Angstrom, per axis
ONSITE_O_S = -1.0         # Ha
ONSITE_O_P = -0.5
ONSITE_H_S = -0.3
ONSITE_NOISE = 0.01       # Ha, standard deviation
HOP_T0 = -0.4             # Ha
HOP_DECAY = 1.0           # Angstrom
HOP_CUT = 5.0             # Angstrom
OVL_S0 = 0.4              # overlap amplitude (dimensionless)
OVL_DECAY = 1.0           # Angstrom
ORB_PER_MOL = 6
ELECTRONS_PER_MOL = 8
KT_DEFAULT = 0.01         # Ha
R_CUT_DEFAULT = 6.0       # Angstrom, colouring / density-matrix cutoff


@dataclass
class CSR:
    """Plain CSR arrays (host)."""
    n: int
    row_ptr: np.ndarray    # int32 [n+1]
    col: np.ndarray        # int32 [nnz], sorted within each row
    val: np.ndarray        # float64 [nnz]

    @property
    def nnz(self) -> int:
        return int(self.row_ptr[-1])

    def to_scipy(self):
        import scipy.sparse as sp
        return sp.csr_matrix((self.val, self.col, self.row_ptr), shape=(self.n, self.n))


@dataclass
class WaterSystem:
    n_mol: int
    box: np.ndarray          # float64 [3] (0 = open)
    atom_xyz: np.ndarray     # float64 [3M, 3]
    orb_xyz: np.ndarray      # float64 [6M, 3], the owning atom's centre
    orb_atom: np.ndarray     # int32 [6M]
    H: CSR
    seed: int
    meta: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return self.H.n

    @property
    def n_electrons(self) -> int:
        return ELECTRONS_PER_MOL * self.n_mol


def box_edge(n_mol: int) -> float:
    return EDGE_PER_1000 * (n_mol / 1000.0) ** (1.0 / 3.0)


def _grid_size(n_mol: int) -> int:
    g = max(1, int(round(n_mol ** (1.0 / 3.0))))
    while g ** 3 < n_mol:
        g += 1
    while g > 1 and (g - 1) ** 3 >= n_mol:
        g -= 1
    return g


def _quat_to_rot(q: np.ndarray) -> np.ndarray:
    """Rotation matrices from unit quaternions (w, x, y, z); q is [k, 4]."""
    w, x, y, z = q[:, 0], q[:, 1], q[:, 2], q[:, 3]
    R = np.empty((q.shape[0], 3, 3))
    R[:, 0, 0] = 1 - 2 * (y * y + z * z)
    R[:, 0, 1] = 2 * (x * y - z * w)
    R[:, 0, 2] = 2 * (x * z + y * w)
    R[:, 1, 0] = 2 * (x * y + z * w)
    R[:, 1, 1] = 1 - 2 * (x * x + z * z)
    R[:, 1, 2] = 2 * (y * z - x * w)
    R[:, 2, 0] = 2 * (x * z - y * w)
    R[:, 2, 1] = 2 * (y * z + x * w)
    R[:, 2, 2] = 1 - 2 * (x * x + y * y)
    return R


def water_geometry(n_mol: int, seed: int, edge: float | None = None):
    """Atom positions [3M, 3] (O, H1, H2 per molecule) wrapped into [0, L)^3."""
    rng = np.random.default_rng(seed)
    L = box_edge(n_mol) if edge is None else float(edge)
    g = _grid_size(n_mol)
    a = L / g
    sites = np.sort(rng.permutation(g ** 3)[:n_mol])
    ijk = np.stack([sites // (g * g), (sites // g) % g, sites % g], axis=1).astype(np.float64)
    centre = (ijk + 0.5) * a
    q = rng.normal(size=(n_mol, 4))
    q /= np.sqrt((q * q).sum(axis=1))[:, None]
    R = _quat_to_rot(q)
    half = math.radians(HOH_ANGLE_DEG) / 2.0
    body = np.array([[0.0, 0.0, 0.0],
                     [OH_BOND * math.sin(half), OH_BOND * math.cos(half), 0.0],
                     [-OH_BOND * math.sin(half), OH_BOND * math.cos(half), 0.0]])
    jitter = rng.uniform(-JITTER, JITTER, size=(n_mol, 3))
    atoms = np.einsum("mij,aj->mai", R, body) + (centre + jitter)[:, None, :]
    atoms = atoms.reshape(3 * n_mol, 3)
    atoms = np.mod(atoms, L)
    atoms[atoms >= L] -= L     # np.mod can return L for tiny negatives
    return atoms, np.array([L, L, L]), rng


def _atom_pairs(atoms: np.ndarray, L: float, cut: float):
    """All unordered atom pairs (i < j) with minimum-image distance <= cut."""
    from scipy.spatial import cKDTree
    tree = cKDTree(atoms, boxsize=L)
    pairs = tree.query_pairs(cut, output_type="ndarray")
    if pairs.size == 0:
        return np.zeros((0, 2), dtype=np.int64)
    return pairs.astype(np.int64)


def tight_binding_h(atoms: np.ndarray, L: float, rng, n_mol: int, progress=None) -> CSR:
    is_o = (np.arange(atoms.shape[0]) % 3) == 0
    first_orb, N = _orbital_offsets(is_o)
    # onsite energies with their noise (the only random draw of H)
    onsite = np.empty(N)
    o_first = first_orb[is_o]
    h_first = first_orb[~is_o]
    onsite[o_first] = ONSITE_O_S
    for k in range(1, 4):
        onsite[o_first + k] = ONSITE_O_P
    onsite[h_first] = ONSITE_H_S
    onsite = onsite + rng.normal(0.0, ONSITE_NOISE, size=N)
    return _two_centre_matrix(atoms, L, onsite, HOP_T0, HOP_DECAY, HOP_CUT, "H", progress)


def overlap_s(atoms: np.ndarray, L: float, progress=None) -> CSR:
    """A non-orthogonal basis' overlap matrix on the same atoms: 1 on the diagonal
    and s(r) g_a(u) g_b(-u), s(r) = 0.4 exp(-r / 1 Angstrom), between orbitals
    of different atoms closer than 5 Angstrom (the same angular factors and
    pattern as H). On water boxes its spectrum lies in about [0.76, 1.84]."""
    is_o = (np.arange(atoms.shape[0]) % 3) == 0
    _, N = _orbital_offsets(is_o)
    return _two_centre_matrix(atoms, L, np.ones(N), OVL_S0, OVL_DECAY, HOP_CUT, "S", progress)


def _orbital_offsets(is_o: np.ndarray):
    n_orb_atom = np.where(is_o, 4, 1)
    first_orb = np.zeros(is_o.size, dtype=np.int64)
    first_orb[1:] = np.cumsum(n_orb_atom)[:-1]
    return first_orb, int(n_orb_atom.sum())


def _two_centre_matrix(atoms: np.ndarray, L: float, diag: np.ndarray, t0: float, decay: float, cut: float,
                       name: str, progress=None) -> CSR:
    """diag on the diagonal, explicit zeros between different orbitals of one atom,
    t0 exp(-r / decay) g_a(u) g_b(-u) between orbitals of atoms closer than cut."""
    n_atoms = atoms.shape[0]
    is_o = (np.arange(n_atoms) % 3) == 0
    first_orb, N = _orbital_offsets(is_o)

    rows, cols, vals = [], [], []

    # same-atom blocks: diag on the diagonal, explicit zeros off it
    o_first = first_orb[is_o]
    h_first = first_orb[~is_o]
    for a in range(4):
        for b in range(4):
            rows.append(o_first + a)
            cols.append(o_first + b)
            vals.append(diag[o_first + a] if a == b else np.zeros(o_first.size))
    rows.append(h_first)
    cols.append(h_first)
    vals.append(diag[h_first])

    # inter-atomic terms, each pair computed once and mirrored
    pairs = _atom_pairs(atoms, L, cut)
    if progress:
        progress(f"{pairs.shape[0]} atom pairs within {cut} A")
    A, B = pairs[:, 0], pairs[:, 1]
    d = atoms[B] - atoms[A]
    d -= L * np.rint(d / L)
    r = np.sqrt((d * d).sum(axis=1))
    u = d / r[:, None]
    t = t0 * np.exp(-r / decay)

    def gvec(is_oxygen, uvec):
        # angular factors per orbital of an atom: [s, px, py, pz] (O) or [s] (H)
        return [np.ones(uvec.shape[0])] + ([uvec[:, 0], uvec[:, 1], uvec[:, 2]] if is_oxygen else [])

    for oa in (True, False):
        if progress:
            progress(f"{name} blocks from {'O' if oa else 'H'} atoms")
        for ob in (True, False):
            sel = (is_o[A] == oa) & (is_o[B] == ob)
            if not np.any(sel):
                continue
            Ai, Bi, ts, us = A[sel], B[sel], t[sel], u[sel]
            ga, gb = gvec(oa, us), gvec(ob, -us)
            for ia, fa in enumerate(ga):
                for ib, fb in enumerate(gb):
                    v = ts * fa * fb
                    m = first_orb[Ai] + ia
                    n = first_orb[Bi] + ib
                    rows += [m, n]
                    cols += [n, m]
                    vals += [v, v]

    row = np.concatenate(rows).astype(np.int32)
    col = np.concatenate(cols).astype(np.int32)
    val = np.concatenate(vals).astype(np.float64)
    if row.size >= 2 ** 31:
        raise ValueError(f"{name} has too many nonzeros for int32 row pointers")
    # CSR with sorted columns; every (row, col) occurs once, so nothing is summed
    import scipy.sparse as sp
    if progress:
        progress(f"CSR of {row.size} entries")
    m = sp.csr_matrix((val, (row, col)), shape=(N, N))
    m.sort_indices()
    if m.nnz != row.size:
        raise AssertionError(f"duplicate orbital pair in {name}")
    return CSR(N, m.indptr.astype(np.int32), m.indices.astype(np.int32), m.data.astype(np.float64))


def water_system(n_mol: int, seed: int, edge: float | None = None, progress=None) -> WaterSystem:
    """A periodic water-like box of n_mol molecules with its tight-binding H.

    progress: optional callable taking a short text, called between the stages
    of a long generation (it does not change the result)."""
    atoms, box, rng = water_geometry(n_mol, seed, edge)
    if progress:
        progress(f"{3 * n_mol} atoms placed")
    H = tight_binding_h(atoms, float(box[0]), rng, n_mol, progress)
    orb_atom = np.repeat(np.arange(3 * n_mol), np.tile([4, 1, 1], n_mol)).astype(np.int32)
    orb_xyz = atoms[orb_atom]
    return WaterSystem(n_mol, box, atoms, np.ascontiguousarray(orb_xyz), orb_atom, H, seed,
                       meta={"edge": float(box[0]), "grid": _grid_size(n_mol)})


def water_overlap(ws: WaterSystem, progress=None) -> CSR:
    """The overlap matrix S of a water box (see `overlap_s`); it draws no random numbers."""
    return overlap_s(ws.atom_xyz, float(ws.box[0]), progress)


def chain_1d(n_sites: int, spacing: float = 1.0):
    """Orbital centres of a periodic 1D chain along x (one orbital per site)."""
    xyz = np.zeros((n_sites, 3))
    xyz[:, 0] = spacing * np.arange(n_sites)
    return xyz, np.array([n_sites * spacing, 0.0, 0.0])


def random_symmetric_csr(xyz: np.ndarray, box: np.ndarray, cut: float, seed: int,
                         diag_scale: float = 1.0, off_scale: float = 0.1) -> CSR:
    """A random symmetric H whose pattern is every pair closer than `cut`.

    Used for small property tests away from the water geometry (chains, open
    clusters). Distances use the minimum image in periodic dimensions.
    """
    rng = np.random.default_rng(seed)
    n = xyz.shape[0]
    d = xyz[None, :, :] - xyz[:, None, :]
    for k in range(3):
        if box[k] > 0:
            d[..., k] -= box[k] * np.rint(d[..., k] / box[k])
    r2 = (d * d).sum(axis=-1)
    mask = r2 <= cut * cut
    vals = rng.normal(size=(n, n)) * off_scale
    vals = np.triu(vals, 1)
    vals = vals + vals.T
    vals[np.arange(n), np.arange(n)] = rng.normal(size=n) * diag_scale
    vals = np.where(mask, vals, 0.0)
    rows, cols = np.nonzero(mask)
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(mask.sum(axis=1), out=row_ptr[1:])
    return CSR(n, row_ptr.astype(np.int32), cols.astype(np.int32), vals[rows, cols].astype(np.float64))
