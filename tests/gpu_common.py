"""Shared helpers of the GPU parity tests: seeded inputs and oracle references."""
from __future__ import annotations

import functools

import numpy as np

from oracle import density as D
from oracle.coloring import greedy_color
from oracle.pattern import conflict_pattern
from oracle.probes import probe_signs
from paper_2605_20918_amd import synth

KT = 0.01
R_CUT = 6.0


@functools.lru_cache(maxsize=None)
def water_case(M: int, seed: int):
    """Seeded water box with the oracle's pattern, colouring, signs and mu."""
    ws = synth.water_system(M, seed)
    H = ws.H.to_scipy()
    rp, col, deg = conflict_pattern(ws.orb_xyz, ws.box, R_CUT)
    color, b = greedy_color(rp, col, deg)
    sign = probe_signs(ws.n, seed)
    mu = D.mu_midgap_dense(H, ws.n_electrons) if ws.n <= 8000 else None
    return ws, H, rp, col, color, b, sign, mu


def to_dev(ws, dtype=None):
    import torch
    from paper_2605_20918_amd import css
    dt = dtype or torch.float64
    return css.DeviceCSR.from_host(ws.H.row_ptr, ws.H.col, ws.H.val, device="cuda", dtype=dt)


def dev_i32(x):
    import torch
    return torch.as_tensor(np.asarray(x), dtype=torch.int32).cuda()


def dev_i64(x):
    import torch
    return torch.as_tensor(np.asarray(x), dtype=torch.int64).cuda()


def dev_i8(x):
    import torch
    return torch.as_tensor(np.asarray(x), dtype=torch.int8).cuda()
