"""Wide probe blocks on the GPU against the oracle: colourings at larger cutoffs give
b = 116 (pole solver with 96 < b <= 128, FP32 tiles for ld = 128), b = 131 (the
dense eigensolver, chosen automatically above 128, and the CSR SpMM for ld > 128)
and b = 307 (the paper's scale of N_c, generic Cholesky). The density (FP64
1e-10; mixed 1e-5 and 1e-7 relative band energy), the chemical potential, S^(-1/2)
and a batch holding such a system are compared with the oracle or single calls."""
import functools

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from oracle import density as D  # noqa: E402
from oracle.coloring import greedy_color  # noqa: E402
from oracle.pattern import conflict_pattern  # noqa: E402
from oracle.probes import probe_signs  # noqa: E402
from paper_2605_20918_amd import css, synth  # noqa: E402

from gpu_common import KT, dev_i8, dev_i32, dev_i64, to_dev  # noqa: E402

FP64_FLAGS = css.PREC_FP64 | css.REORTH_FULL | css.CHOLQR2 | css.SYMMETRIZE
FP32_FLAGS = css.PREC_FP32 | css.REORTH_FULL | css.CHOLQR2 | css.SYMMETRIZE
CASES = [(216, 3, 6.8, 116), (216, 3, 7.0, 131), (343, 5, 10.0, 307)]


def setup_module(module):
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    css.load()


@functools.lru_cache(maxsize=None)
def wide_case(M, seed, r_cut):
    ws = synth.water_system(M, seed)
    H = ws.H.to_scipy()
    rp, col, deg = conflict_pattern(ws.orb_xyz, ws.box, r_cut)
    color, b = greedy_color(rp, col, deg)
    sign = probe_signs(ws.n, seed)
    mu = D.mu_midgap_dense(H, ws.n_electrons)
    return ws, H, rp, col, color, b, sign, mu


@functools.lru_cache(maxsize=None)
def oracle_density(M, seed, r_cut):
    ws, H, rp, col, color, b, sign, mu = wide_case(M, seed, r_cut)
    return D.density_matrix(H, color, sign, b, mu, KT, 40, rp, col, reorth="full", cholqr2=True)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("M,seed,r_cut,b_expect", CASES)
def test_wide_density_parity(M, seed, r_cut, b_expect, prec):
    print(f"wide density {prec} M={M} r_cut={r_cut}", flush=True)
    ws, H, rp, col, color, b, sign, mu = wide_case(M, seed, r_cut)
    assert b == b_expect
    ref = oracle_density(M, seed, r_cut)
    flags = FP64_FLAGS if prec == "fp64" else FP32_FLAGS
    dt = torch.float64 if prec == "fp64" else torch.float32
    g_color, g_b, g_rp, g_col, _ = css.css_color(torch.as_tensor(ws.orb_xyz).cuda(), ws.box, r_cut)
    assert g_b == b and np.array_equal(g_color.cpu().numpy(), color)
    p, e, t, info = css.css_density_matrix(to_dev(ws, dt), g_color, dev_i8(sign), b, mu, KT, 40, g_rp, g_col, flags)
    assert info["depth_eff"] == ref["v_eff"]
    assert info["n_poles"] == (0 if b > 128 else info["n_poles"]) and (b > 128 or info["n_poles"] > 0)
    err = np.max(np.abs(p.cpu().numpy() - ref["p_val"]))
    rel_e = abs(e - ref["e_band"]) / abs(ref["e_band"])
    print(f"  b={b} v_eff={info['depth_eff']} max|dP|={err:.3e} rel dE={rel_e:.3e} poles={info['n_poles']}",
          flush=True)
    assert err <= (1e-10 if prec == "fp64" else 1e-5)
    assert rel_e <= (1e-10 if prec == "fp64" else 1e-7)


@pytest.mark.parametrize("M,seed,r_cut,b_expect", CASES)
def test_wide_find_mu_parity(M, seed, r_cut, b_expect):
    ws, H, rp, col, color, b, sign, _ = wide_case(M, seed, r_cut)
    ne = float(ws.n_electrons)
    ref = D.find_mu(H, color, sign, b, ne, KT, 40, reorth="full", cholqr2=True)
    mu, count, info = css.css_find_mu(to_dev(ws), dev_i32(color), dev_i8(sign), b, ne, KT, 40, FP64_FLAGS)
    resid = abs(D.krylov_count(ref["lam"], ref["w"], mu, KT) - ne)
    print(f"  wide mu b={b}: |dmu|={abs(mu - ref['mu']):.3e} resid={resid:.3e}", flush=True)
    assert resid <= 1e-10 * ne
    slope = D.krylov_count_slope(ref["lam"], ref["w"], ref["mu"], KT)
    assert abs(mu - ref["mu"]) <= 1e-10 * ne / slope + 1e-12


@pytest.mark.parametrize("M,seed,r_cut,b_expect", CASES)
def test_wide_inv_sqrt_parity(M, seed, r_cut, b_expect):
    ws, H, rp, col, color, b, sign, _ = wide_case(M, seed, r_cut)
    So = synth.water_overlap(ws)
    ref = D.inv_sqrt_matrix(So.to_scipy(), color, sign, b, 10, rp, col)
    Sd = css.DeviceCSR.from_host(So.row_ptr, So.col, So.val, "cuda", torch.float64)
    y, tr, _, info = css.css_inv_sqrt_overlap(Sd, dev_i32(color), dev_i8(sign), b, 10, dev_i64(rp), dev_i32(col),
                                              FP64_FLAGS)
    err = np.max(np.abs(y.cpu().numpy() - ref["y_val"]))
    print(f"  wide S^-1/2 b={b}: max|dY|={err:.3e}", flush=True)
    assert err <= 1e-10
    assert abs(tr - ref["trace"]) <= 1e-10 * abs(ref["trace"])


def test_batch_with_a_wide_system_equals_single_calls():
    """A batch holding a b = 131 system (dense eigensolver) and a b = 116 one (poles)
    gives bitwise the single-call results."""
    systems = []
    for M, seed, r_cut, _ in CASES[:2]:
        ws, H, rp, col, color, b, sign, mu = wide_case(M, seed, r_cut)
        systems.append(dict(H=to_dev(ws), color=dev_i32(color), sign=dev_i8(sign), n_colors=b, mu=mu,
                            p_row_ptr=dev_i64(rp), p_col=dev_i32(col)))
    res = css.css_density_matrix_batched(systems, KT, 40, FP64_FLAGS, concurrency=2)
    for d, r in zip(systems, res):
        p, e, t, _ = css.css_density_matrix(d["H"], d["color"], d["sign"], d["n_colors"], d["mu"], KT, 40,
                                            d["p_row_ptr"], d["p_col"], FP64_FLAGS)
        assert torch.equal(r[0], p) and r[1] == e and r[2] == t
