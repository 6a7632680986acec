"""Pins of the oracle's conflict pattern and greedy colouring (CPU only)."""
import json
import os
from fractions import Fraction

import numpy as np
import pytest

from oracle.coloring import greedy_color, welsh_powell_order
from oracle.pattern import conflict_pattern
from paper_2605_20918_amd import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def cubic_lattice(g, spacing=1.0):
    idx = np.arange(g ** 3)
    xyz = np.stack([idx // (g * g), (idx // g) % g, idx % g], axis=1).astype(np.float64) * spacing
    return xyz, np.array([g * spacing] * 3, dtype=np.float64)


@pytest.mark.parametrize("r_cut,deg", [(1.0, 6), (1.5, 18), (1.8, 26), (2.0, 32)])
def test_cubic_lattice_shell_counts(r_cut, deg):
    # closed form: shells of the simple cubic lattice hold 6 (d=1), 12 (sqrt2), 8 (sqrt3), 6 (d=2)
    # r_cut = 1.0 lands exactly on the first shell: "within" includes it
    xyz, box = cubic_lattice(6)
    rp, col, d = conflict_pattern(xyz, box, r_cut)
    assert np.all(d == deg)
    assert np.all(np.diff(rp) == deg + 1)


def test_pattern_symmetric_sorted_with_diagonal():
    ws = synth.water_system(27, seed=5)
    rp, col, deg = conflict_pattern(ws.orb_xyz, ws.box, 6.0)
    n = ws.n
    rows = np.repeat(np.arange(n), np.diff(rp))
    assert np.all(np.diff(col.astype(np.int64) + rows * n) > 0)      # strictly sorted rows
    key = set(zip(rows.tolist(), col.tolist()))
    assert all((c, r) in key for r, c in key)
    assert all((i, i) in key for i in range(n))
    # same-atom orbitals always conflict
    for a in range(ws.n_mol):
        o = 6 * a
        assert {(o, o + 1), (o, o + 2), (o, o + 3)} <= key


def test_pattern_against_exact_arithmetic_brute_force():
    # exact rational distances on a tiny periodic set; pairs within 1e-9 of the
    # cutoff are excluded from the comparison (measure-zero rounding cases)
    rng = np.random.default_rng(7)
    L = 9.0
    xyz = np.round(rng.uniform(0, L, size=(60, 3)), 3)
    box = np.array([L, L, L])
    r_cut = 3.1
    rp, col, _ = conflict_pattern(xyz, box, r_cut)
    got = set(zip(np.repeat(np.arange(60), np.diff(rp)).tolist(), col.tolist()))
    Lf = Fraction(L)
    for m in range(60):
        for n in range(60):
            d2 = Fraction(0)
            for k in range(3):
                d = Fraction(float(xyz[n, k])) - Fraction(float(xyz[m, k]))
                while d > Lf / 2:
                    d -= Lf
                while d < -Lf / 2:
                    d += Lf
                d2 += d * d
            if abs(float(d2) - r_cut ** 2) < 1e-9:
                continue
            assert ((m, n) in got) == (d2 <= Fraction(r_cut) ** 2), (m, n)


def test_minimum_image_across_boundary():
    xyz = np.array([[0.1, 5.0, 5.0], [9.9, 5.0, 5.0], [5.0, 5.0, 5.0]])
    rp, col, deg = conflict_pattern(xyz, np.array([10.0, 10.0, 10.0]), 0.5)
    assert deg.tolist() == [1, 1, 0]
    rp, col, deg = conflict_pattern(xyz, np.array([0.0, 0.0, 0.0]), 0.5)    # open box
    assert deg.tolist() == [0, 0, 0]


@pytest.mark.parametrize("n,spacing,r_cut", [(12, 1.0, 2.5), (30, 0.7, 1.45), (20, 1.0, 4.0), (10, 2.0, 2.0)])
def test_chain_closed_form(n, spacing, r_cut):
    # Fig.1(b): periodic 1D chain, k*a <= r_cut < (k+1)*a and (k+1) | n
    # => every degree is 2k, WP order = index order, colour(i) = i mod (k+1)
    k = int(np.floor(r_cut / spacing + 1e-12))
    assert n % (k + 1) == 0
    xyz, box = synth.chain_1d(n, spacing)
    rp, col, deg = conflict_pattern(xyz, box, r_cut)
    assert np.all(deg == 2 * k)
    color, b = greedy_color(rp, col, deg)
    assert b == k + 1
    assert np.array_equal(color, np.arange(n) % (k + 1))


def test_complete_graph_gives_identity_colouring():
    rng = np.random.default_rng(3)
    xyz = rng.uniform(0, 1, size=(25, 3))
    rp, col, deg = conflict_pattern(xyz, np.zeros(3), 10.0)
    color, b = greedy_color(rp, col, deg)
    assert b == 25 and np.array_equal(color, np.arange(25))


def test_bipartite_lattice_parity_colouring():
    # periodic even cubic lattice, nearest neighbours only: all degrees 6, so the
    # WP order is the index order and first fit gives the checkerboard
    g = 4
    xyz, box = cubic_lattice(g)
    rp, col, deg = conflict_pattern(xyz, box, 1.0)
    color, b = greedy_color(rp, col, deg)
    idx = np.arange(g ** 3)
    assert b == 2
    assert np.array_equal(color, ((idx // 16) + (idx // 4) % 4 + idx % 4) % 2)


def test_welsh_powell_hand_example():
    with open(os.path.join(GOLDEN, "wp_line.json")) as f:
        g = json.load(f)
    xyz = np.zeros((len(g["x"]), 3))
    xyz[:, 0] = g["x"]
    rp, col, deg = conflict_pattern(xyz, np.zeros(3), g["r_cut"])
    assert deg.tolist() == g["degree"]
    color, b = greedy_color(rp, col, deg)
    assert color.tolist() == g["color"] and b == g["n_colors"]


def test_wp_order_ties_by_index():
    deg = np.array([3, 5, 5, 1, 3])
    assert welsh_powell_order(deg).tolist() == [1, 2, 0, 4, 3]


def test_water_colouring_valid_and_bounded():
    ws = synth.water_system(64, seed=20919)
    rp, col, deg = conflict_pattern(ws.orb_xyz, ws.box, 6.0)
    color, b = greedy_color(rp, col, deg)
    rows = np.repeat(np.arange(ws.n), np.diff(rp))
    off = rows != col
    assert not np.any(color[rows[off]] == color[col[off]])
    assert b <= deg.max() + 1
    assert set(np.unique(color)) == set(range(b))
    # first use order: colour c first appears before colour c+1 along the WP order
    first = [np.min(np.nonzero(color[welsh_powell_order(deg)] == c)[0]) for c in range(b)]
    assert first == sorted(first)
