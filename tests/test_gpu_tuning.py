"""Launch choices (css_tuning) and the autotuner on the GPU: every choice computes
the same product and density up to FP32 summation order, each is deterministic, and
the autotuner records and applies a choice."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from oracle import density as D  # noqa: E402
from paper_2605_20918_amd import autotune, css, synth  # noqa: E402

from gpu_common import KT, dev_i8, dev_i32, dev_i64, to_dev, water_case  # noqa: E402

FP32_FLAGS = css.PREC_FP32 | css.REORTH_FULL | css.CHOLQR2 | css.SYMMETRIZE

CHOICES = [dict(), dict(spmm_kernel="grouped", spmm_run=64, spmm_depth=8),
           dict(spmm_kernel="grouped", spmm_run=4096, spmm_depth=4), dict(spmm_kernel="csr"),
           dict(gram_chunks=2, update_rows=64), dict(gram_chunks=4, update_rows=128), dict(cholqr2_series=2)]


def setup_module(module):
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    css.load()


def teardown_module(module):
    css.reset_tuning()


@pytest.mark.parametrize("cfg", CHOICES)
def test_spmm_every_choice_matches_fp64_product(cfg):
    print(f"spmm tuning {cfg}", flush=True)
    ws = synth.water_system(216, 7)
    b = 88
    ld = css.block_ld(b)
    rng = np.random.default_rng(2)
    Vh = np.zeros((ws.n, ld))
    Vh[:, :b] = rng.normal(size=(ws.n, b))
    ref = ws.H.to_scipy() @ Vh
    H = css.DeviceCSR.from_host(ws.H.row_ptr, ws.H.col, ws.H.val, "cuda", torch.float32)
    spws = css.css_spmm_prepare(H)
    css.set_tuning(**cfg)
    try:
        W1 = css.css_spmm(H, torch.as_tensor(Vh, dtype=torch.float32).cuda(), b, ws=spws).double().cpu().numpy()
        W2 = css.css_spmm(H, torch.as_tensor(Vh, dtype=torch.float32).cuda(), b, ws=spws).double().cpu().numpy()
    finally:
        css.reset_tuning()
    assert np.array_equal(W1, W2)
    assert np.max(np.abs(W1 - ref)) <= 2e-6 * np.max(np.abs(ref))


@pytest.mark.parametrize("cfg", CHOICES)
def test_density_every_choice_within_mixed_tolerance(cfg):
    """The mixed density under each launch choice against the FP64 oracle (1e-5 on P,
    1e-7 relative band energy), and bitwise repeatable under that choice."""
    print(f"density tuning {cfg}", flush=True)
    ws, H, rp, col, color, b, sign, mu = water_case(216, 3)
    ref = D.density_matrix(H, color, sign, b, mu, KT, 20, rp, col, reorth="full")
    args = (to_dev(ws, torch.float32), dev_i32(color), dev_i8(sign), b, mu, KT, 20, dev_i64(rp), dev_i32(col),
            FP32_FLAGS)
    css.set_tuning(**cfg)
    try:
        p1, e1, _, _ = css.css_density_matrix(*args)
        p1 = p1.clone()
        p2, e2, _, _ = css.css_density_matrix(*args)
    finally:
        css.reset_tuning()
    assert torch.equal(p1, p2) and e1 == e2
    assert np.max(np.abs(p1.cpu().numpy() - ref["p_val"])) <= 1e-5
    assert abs(e1 - ref["e_band"]) <= 1e-7 * abs(ref["e_band"])


@pytest.mark.parametrize("M,seed,depth", [(216, 3, 40), (1000, 20920, 40)])
def test_series_second_cholqr_factor_equals_factorisation_fp64(M, seed, depth):
    """FP64: the second CholQR factor by the near-identity series (default) and by the
    blocked factorisation give the same P to rounding, both at the oracle's 1e-10."""
    print(f"cholqr2 series M={M}", flush=True)
    ws, H, rp, col, color, b, sign, mu = water_case(M, seed)
    ref = D.density_matrix(H, color, sign, b, mu, KT, depth, rp, col, reorth="full")
    args = (to_dev(ws), dev_i32(color), dev_i8(sign), b, mu, KT, depth, dev_i64(rp), dev_i32(col),
            css.PREC_FP64 | css.REORTH_FULL | css.CHOLQR2 | css.SYMMETRIZE)
    css.reset_tuning()
    p1, e1, _, i1 = css.css_density_matrix(*args)
    p1 = p1.clone()
    css.set_tuning(cholqr2_series=2)
    try:
        p2, e2, _, i2 = css.css_density_matrix(*args)
    finally:
        css.reset_tuning()
    d = torch.max(torch.abs(p1 - p2)).item()
    print(f"  series vs factorisation max|dP| {d:.3e}", flush=True)
    assert d <= 1e-13 and abs(e1 - e2) <= 1e-13 * abs(e1)
    for p in (p1, p2):
        assert np.max(np.abs(p.cpu().numpy() - ref["p_val"])) <= 1e-10


def test_twopass_replay_bitwise_under_a_tuning():
    """The two-pass mode regenerates the basis bitwise under a non-default tuning too."""
    ws, H, rp, col, color, b, sign, mu = water_case(216, 3)
    args = (to_dev(ws), dev_i32(color), dev_i8(sign), b, mu, KT, 12, dev_i64(rp), dev_i32(col))
    base = css.PREC_FP64 | css.REORTH_LOCAL | css.CHOLQR2 | css.SYMMETRIZE
    css.set_tuning(spmm_kernel="grouped", spmm_run=64, spmm_depth=8)
    try:
        p1, e1, _, _ = css.css_density_matrix(*args, base)
        p2, e2, _, _ = css.css_density_matrix(*args, base | css.BASIS_TWOPASS)
    finally:
        css.reset_tuning()
    assert torch.max(torch.abs(p1 - p2)).item() <= 1e-13


def test_autotune_records_and_applies(tmp_path):
    ws, H, rp, col, color, b, sign, mu = water_case(216, 3)
    Hd = to_dev(ws, torch.float32)
    path = str(tmp_path / "tune.json")
    out = autotune.autotune(Hd, dev_i32(color), dev_i8(sign), b, 10, FP32_FLAGS, path=path)
    now = css.get_tuning()
    assert all(now[k] == v for k, v in out["choice"].items())
    assert len(out["spmm_trials"]) == 1 + len(autotune.SPMM_RUNS) * len(autotune.SPMM_DEPTHS)
    assert len(out["lanczos_trials"]) == len(autotune.GRAM_CHUNKS) * len(autotune.UPDATE_ROWS)
    css.reset_tuning()
    got = autotune.apply_cached(Hd.n, Hd.nnz, b, "fp32", path)
    assert got == out["choice"]
    css.reset_tuning()
