"""Loss of orthogonality of the Krylov basis, max |Q^T Q - I| (CSS_DIAG_ORTHO).

The measured value comes from the library's Gram products over the stored basis; it
is compared with the same quantity of the oracle's basis. Where the basis stays
orthonormal to rounding (full re-orthogonalisation, or local re-orthogonalisation
before Ritz values converge) both are at the rounding level. Past that point the loss
grows from rounding errors, whose pattern differs between the two sides, so there the
comparison is of magnitude.
"""
import os
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))

from oracle.lanczos import block_lanczos  # noqa: E402
from paper_2605_20918_amd import css  # noqa: E402

from gpu_common import KT, dev_i8, dev_i32, dev_i64, to_dev, water_case  # noqa: E402

BASE = css.CHOLQR2 | css.SYMMETRIZE


def setup_module(module):
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    css.load()


def _oracle_loss(H, color, sign, b, depth, reorth):
    lz = block_lanczos(H, color, sign, b, depth=depth, reorth=reorth)
    Phi = np.hstack(lz.Q)
    return lz.v_eff, float(np.max(np.abs(Phi.T @ Phi - np.eye(Phi.shape[1]))))


def _gpu_loss(ws, color, sign, b, depth, flags, dtype=None):
    _, _, info = css.css_block_lanczos(to_dev(ws, dtype), dev_i32(color), dev_i8(sign), b, depth,
                                       flags | css.DIAG_ORTHO)
    return info["depth_eff"], info["ortho_err"]


@pytest.mark.parametrize("M,seed,depth,reorth", [(216, 3, 8, "local"), (216, 3, 40, "full"),
                                                 (1000, 20920, 10, "local"), (1000, 20920, 40, "full")])
def test_orthonormal_basis_fp64(M, seed, depth, reorth):
    print(f"ortho fp64 M={M} depth={depth} {reorth}", flush=True)
    ws, H, rp, col, color, b, sign, mu = water_case(M, seed)
    v_ref, e_ref = _oracle_loss(H, color, sign, b, depth, reorth)
    flags = css.PREC_FP64 | BASE | (css.REORTH_FULL if reorth == "full" else css.REORTH_LOCAL)
    v, e = _gpu_loss(ws, color, sign, b, depth, flags)
    print(f"  gpu {e:.3e} oracle {e_ref:.3e}", flush=True)
    assert v == v_ref
    assert e_ref <= 1e-13 and 0.0 < e <= 1e-13


@pytest.mark.parametrize("M,seed,depth", [(216, 3, 12), (216, 3, 15), (1000, 20920, 20), (1000, 20920, 30),
                                          (1000, 20920, 40)])
def test_local_reorth_loss_tracks_the_oracle(M, seed, depth):
    """Local re-orthogonalisation past the first converged Ritz values: the loss grows by
    orders of magnitude with depth on both sides, and the two agree in magnitude."""
    print(f"ortho local M={M} depth={depth}", flush=True)
    ws, H, rp, col, color, b, sign, mu = water_case(M, seed)
    v_ref, e_ref = _oracle_loss(H, color, sign, b, depth, "local")
    v, e = _gpu_loss(ws, color, sign, b, depth, css.PREC_FP64 | BASE | css.REORTH_LOCAL)
    print(f"  gpu {e:.3e} oracle {e_ref:.3e}", flush=True)
    assert v == v_ref
    assert e_ref > 1e-11
    assert e_ref / 30 <= e <= 30 * e_ref


@pytest.mark.parametrize("schedule", ["full", "alternate"])
def test_mixed_path_basis_is_orthonormal_to_fp32_rounding(schedule):
    ws, H, rp, col, color, b, sign, mu = water_case(1000, 20920)
    flags = css.PREC_FP32 | BASE | css.REORTH_FULL | (css.REORTH_ALTERNATE if schedule == "alternate" else 0)
    v, e = _gpu_loss(ws, color, sign, b, 40, flags, torch.float32)
    print(f"ortho fp32 {schedule}: {e:.3e}", flush=True)
    assert v == 40
    assert 0.0 < e <= 1e-5


def test_diagnostic_leaves_the_result_unchanged_and_matches_block_lanczos():
    ws, H, rp, col, color, b, sign, mu = water_case(216, 3)
    flags = css.PREC_FP64 | BASE | css.REORTH_LOCAL
    args = (to_dev(ws), dev_i32(color), dev_i8(sign), b, mu, KT, 12, dev_i64(rp), dev_i32(col))
    p1, e1, t1, i1 = css.css_density_matrix(*args, flags)
    p1 = p1.clone()
    p2, e2, t2, i2 = css.css_density_matrix(*args, flags | css.DIAG_ORTHO)
    assert torch.equal(p1, p2) and e1 == e2 and t1 == t2
    assert np.isnan(i1["ortho_err"])
    _, e_lz = _gpu_loss(ws, color, sign, b, 12, flags)
    assert i2["ortho_err"] == e_lz


def test_two_pass_reports_nan():
    ws, H, rp, col, color, b, sign, mu = water_case(216, 3)
    flags = css.PREC_FP64 | BASE | css.REORTH_LOCAL | css.BASIS_TWOPASS | css.DIAG_ORTHO
    _, _, _, info = css.css_density_matrix(to_dev(ws), dev_i32(color), dev_i8(sign), b, mu, KT, 12, dev_i64(rp),
                                           dev_i32(col), flags)
    assert np.isnan(info["ortho_err"])
