"""Oracle: chromatic superposition states (CSS probe vectors).

Test infrastructure only: see the package docstring.

Definition followed (text around Eq.(2) and Fig.1(c)): for each colour i the
probe r_i holds +-1 on the orbitals of colour i and 0 elsewhere; the paper
notes the signs may be drawn at random so that errors cancel stochastically.
Because different probes have disjoint supports they are mutually
orthogonal, and the block r = [r_1 .. r_b] factors exactly as r = Q_1 B_0 with
Q_1 = r diag(1/sqrt(n_c)) (orthonormal columns) and B_0 = diag(sqrt(n_c)),
n_c the number of orbitals of colour c.

Reading (sign source): s_m = +1 when the top bit of the SplitMix64 output for
counter m is 0, else -1. SplitMix64 (Steele, Lea and Flood, OOPSLA 2014) with
state seed produces, as its (m+1)-th output, mix(seed + (m+1)*0x9E3779B97F4A7C15)
where mix(z) = z1 ^ (z1 >> 31), z1 = (z0 ^ (z0 >> 27)) * 0x94D049BB133111EB,
z0 = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9, all modulo 2^64. A flag selects all
signs +1 instead.
"""
from __future__ import annotations

import numpy as np

GOLDEN_GAMMA = np.uint64(0x9E3779B97F4A7C15)
MIX1 = np.uint64(0xBF58476D1CE4E5B9)
MIX2 = np.uint64(0x94D049BB133111EB)


def splitmix64(seed: int, counter: np.ndarray) -> np.ndarray:
    """Output number counter+1 of SplitMix64 started at state `seed`."""
    with np.errstate(over="ignore"):
        z = np.uint64(seed) + (np.asarray(counter, dtype=np.uint64) + np.uint64(1)) * GOLDEN_GAMMA
        z = (z ^ (z >> np.uint64(30))) * MIX1
        z = (z ^ (z >> np.uint64(27))) * MIX2
        return z ^ (z >> np.uint64(31))


def probe_signs(n: int, seed: int, all_ones: bool = False) -> np.ndarray:
    if all_ones:
        return np.ones(n, dtype=np.int8)
    top = splitmix64(seed, np.arange(n, dtype=np.uint64)) >> np.uint64(63)
    return np.where(top == 0, 1, -1).astype(np.int8)


def color_counts(color: np.ndarray, n_colors: int) -> np.ndarray:
    return np.bincount(color, minlength=n_colors).astype(np.int32)


def probe_block(color: np.ndarray, sign: np.ndarray, n_colors: int) -> np.ndarray:
    """Dense r (N x b): r[m, color[m]] = sign[m]."""
    n = color.shape[0]
    r = np.zeros((n, n_colors))
    r[np.arange(n), color] = sign
    return r


def first_block(color: np.ndarray, sign: np.ndarray, n_colors: int):
    """Q_1 (N x b, orthonormal columns) and the diagonal of B_0, with r = Q_1 B_0."""
    n_c = color_counts(color, n_colors).astype(np.float64)
    if np.any(n_c == 0):
        raise ValueError("every colour must own at least one orbital")
    b0 = np.sqrt(n_c)
    Q1 = probe_block(color, sign, n_colors) / b0[None, :]
    return Q1, b0
