"""Parity at the benchmark sizes, in the launch configuration bench.py times.

10 000 molecules: the oracle runs the whole path (about a minute on the host) and the
GPU results are compared element by element. 10^6 molecules: the oracle cannot run, so
the GPU results are checked against identities that hold at any size and the mixed
path against the FP64 path.
"""
import os
import sys
import time

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402
from oracle import density as D  # noqa: E402
from oracle.coloring import greedy_color  # noqa: E402
from oracle.pattern import conflict_pattern  # noqa: E402
from oracle.probes import probe_signs  # noqa: E402
from paper_2605_20918_amd import css, synth  # noqa: E402

KT, R_CUT, MU = bench.KT, bench.R_CUT, bench.MU_WATER


def setup_module(module):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    css.load()


def _gpu_step(ws, seed, H, flags, depth=40):
    xyz = torch.as_tensor(ws.orb_xyz, dtype=torch.float64, device="cuda")
    color, b, p_rp, p_col, _ = css.css_color(xyz, [float(x) for x in ws.box], R_CUT)
    sign, _ = css.css_build_probes(color, b, seed)
    p, e, t, info = css.css_density_matrix(H, color, sign, b, MU, KT, depth, p_rp, p_col, flags)
    return color, b, p_rp, p_col, sign, p, e, t, info


def test_10k_against_the_oracle():
    wl = bench.WORKLOADS["10k"]
    ws = synth.water_system(wl["n_mol"], wl["seed"])
    print("10k: oracle pattern, colouring and density", flush=True)
    rp, col, deg = conflict_pattern(ws.orb_xyz, ws.box, R_CUT)
    color, b = greedy_color(rp, col, deg)
    sign = probe_signs(ws.n, wl["seed"])
    t0 = time.perf_counter()
    ref = D.density_matrix(ws.H.to_scipy(), color, sign, b, MU, KT, wl["depth"], rp, col, reorth="full",
                           cholqr2=True)
    print(f"10k: oracle done (b={b}, v_eff={ref['v_eff']}, density {time.perf_counter() - t0:.1f} s)", flush=True)
    # the FP64 comparator of the bench re-orthogonalises locally: its oracle does the same
    t0 = time.perf_counter()
    ref_local = D.density_matrix(ws.H.to_scipy(), color, sign, b, MU, KT, wl["depth"], rp, col, reorth="local",
                                 cholqr2=bench.BENCH_CHOLQR2)
    print(f"10k: oracle with local re-orthogonalisation {time.perf_counter() - t0:.1f} s", flush=True)
    H32 = css.DeviceCSR.from_host(ws.H.row_ptr, ws.H.col, ws.H.val, "cuda", torch.float32)
    H64 = css.DeviceCSR.from_host(ws.H.row_ptr, ws.H.col, ws.H.val, "cuda", torch.float64)
    # the mixed path of the bench re-orthogonalises against every block on alternate steps
    t0 = time.perf_counter()
    ref_alt = D.density_matrix(ws.H.to_scipy(), color, sign, b, MU, KT, wl["depth"], rp, col, reorth="alternate",
                               cholqr2=bench.BENCH_CHOLQR2)
    print(f"10k: oracle with the alternating schedule {time.perf_counter() - t0:.1f} s", flush=True)
    runs = {"mixed (bench)": (H32, bench.flags_for("fp32"), ref_alt),
            "fp64 alternate": (H64, bench.flags_for("fp64", reorth="full"), ref_alt),
            "fp64 full": (H64, css.PREC_FP64 | css.REORTH_FULL | css.CHOLQR2 | css.SYMMETRIZE, ref),
            "fp64 local (bench comparator)": (H64, bench.flags_for("fp64"), ref_local),
            "fp64 local two-pass": (H64, bench.flags_for("fp64", twopass=True), ref_local)}
    errs = {}
    for name, (H, flags, rf) in runs.items():
        g_color, g_b, g_rp, g_col, g_sign, p, e, t, info = _gpu_step(ws, wl["seed"], H, flags)
        assert g_b == b and np.array_equal(g_color.cpu().numpy(), color)
        assert np.array_equal(g_rp.cpu().numpy(), rp) and np.array_equal(g_col.cpu().numpy(), col)
        assert np.array_equal(g_sign.cpu().numpy(), sign)
        assert info["depth_eff"] == ref["v_eff"]
        dp = float(np.max(np.abs(p.cpu().numpy() - rf["p_val"])))
        de = abs(e - rf["e_band"]) / abs(rf["e_band"])
        errs[name] = (dp, de)
        print(f"10k {name}: max|dP| {dp:.3e}  rel dE {de:.3e}", flush=True)
    assert errs["mixed (bench)"][0] <= 1e-5 and errs["mixed (bench)"][1] <= 1e-7
    assert errs["fp64 full"][0] <= 1e-10 and errs["fp64 full"][1] <= 1e-10
    for name in ("fp64 local (bench comparator)", "fp64 local two-pass", "fp64 alternate"):
        assert errs[name][0] <= 1e-10 and errs[name][1] <= 1e-10
    # the energy-weighted estimate, mixed precision, element by element against the oracle
    t0 = time.perf_counter()
    eref = D.energy_density_matrix(ws.H.to_scipy(), ref, color, sign, rp, col)
    print(f"10k oracle energy-weighted (after the density): {time.perf_counter() - t0:.2f} s", flush=True)
    xyz = torch.as_tensor(ws.orb_xyz, dtype=torch.float64, device="cuda")
    g_color, g_b, g_rp, g_col, _ = css.css_color(xyz, [float(x) for x in ws.box], R_CUT)
    g_sign, _ = css.css_build_probes(g_color, g_b, wl["seed"])
    _, pe, _, _, pe_trace, _ = css.css_energy_density_matrix(H32, g_color, g_sign, g_b, MU, KT, wl["depth"], g_rp,
                                                             g_col, bench.flags_for("fp32"))
    hinf = float(np.max(np.abs(ws.H.to_scipy()).sum(axis=1)))
    dpe = float(np.max(np.abs(pe.cpu().numpy() - eref["pe_val"])))
    dtr = abs(pe_trace - eref["pe_trace"]) / abs(eref["pe_trace"])
    print(f"10k energy-weighted mixed: max|dP_E| {dpe:.3e} (||H||_inf {hinf:.2f})  rel dTr {dtr:.3e}", flush=True)
    assert dpe <= 1e-5 * hinf and dtr <= 1e-7
    # mu for N_e electrons, mixed precision, against the oracle's bisection on its own T
    from oracle.subspace import eig_subspace
    t0 = time.perf_counter()
    lam, U = eig_subspace(ref["T"])
    w = D.krylov_weights(U, ref["lanczos"].b0)
    ne = float(ws.n_electrons)
    mu_ref = D.mu_krylov_bisection(lam, w, ne, KT)
    print(f"10k oracle mu (after the Lanczos pass): {time.perf_counter() - t0:.2f} s", flush=True)
    mu, count, minfo = css.css_find_mu(H32, g_color, g_sign, g_b, ne, KT, wl["depth"], bench.flags_for("fp32"))
    resid = abs(D.krylov_count(lam, w, mu, KT) - ne)
    slope = D.krylov_count_slope(lam, w, mu_ref, KT)
    print(f"10k mu mixed: {mu:.10f} oracle {mu_ref:.10f} |dmu| {abs(mu - mu_ref):.3e} resid {resid:.3e} "
          f"slope {slope:.1f} ({minfo['t_phase_ms']['total']:.1f} ms, {minfo['n_evals']} count evaluations)",
          flush=True)
    assert minfo["depth_eff"] == ref["v_eff"]
    assert resid <= 1e-7 * ne and abs(mu - mu_ref) <= 1e-7 * ne / slope
    # S^(-1/2) of the overlap, mixed precision, v^s = 10, against the oracle
    So = synth.water_overlap(ws)
    t0 = time.perf_counter()
    yref = D.inv_sqrt_matrix(So.to_scipy(), color, sign, b, 10, rp, col)
    print(f"10k oracle S^-1/2: {time.perf_counter() - t0:.2f} s", flush=True)
    S32 = css.DeviceCSR.from_host(So.row_ptr, So.col, So.val, "cuda", torch.float32)
    y, ytr, _, yinfo = css.css_inv_sqrt_overlap(S32, g_color, g_sign, g_b, 10, g_rp, g_col, bench.flags_for("fp32"))
    dy = float(np.max(np.abs(y.cpu().numpy() - yref["y_val"])))
    dytr = abs(ytr - yref["trace"]) / abs(yref["trace"])
    print(f"10k S^-1/2 mixed: max|dY| {dy:.3e}  rel dTr {dytr:.3e} ({yinfo['t_phase_ms']['total']:.1f} ms)",
          flush=True)
    assert yinfo["depth_eff"] == yref["v_eff"] and dy <= 1e-5 and dytr <= 1e-7
    # H' = S^(-1/2) H S^(-1/2), mixed precision, against the oracle
    t0 = time.perf_counter()
    href = D.transform_hamiltonian(ws.H.to_scipy(), So.to_scipy(), color, sign, b, 10, rp, col)
    print(f"10k oracle H': {time.perf_counter() - t0:.2f} s", flush=True)
    _, hp, _, hptr, _ = css.css_transform_hamiltonian(H32, S32, g_color, g_sign, g_b, 10, g_rp, g_col,
                                                      bench.flags_for("fp32"))
    dh = float(np.max(np.abs(hp.cpu().numpy() - href["hp_val"])))
    dhtr = abs(hptr - href["hp_trace"]) / abs(href["hp_trace"])
    print(f"10k H' mixed: max|dH'| {dh:.3e}  rel dTr {dhtr:.3e}", flush=True)
    assert dh <= 1e-5 * hinf and dhtr <= 1e-7
    # density matrix of the non-orthogonal basis, mixed precision, from the oracle's sparse
    # S^(-1/2) and H' (the same inputs on both sides), against the oracle
    import scipy.sparse as sp
    Sh = sp.csr_matrix((href["y_val"], col, rp), shape=(ws.n, ws.n))
    Hp = sp.csr_matrix((href["hp_val"], col, rp), shape=(ws.n, ws.n))
    t0 = time.perf_counter()
    nref = D.density_matrix_nonorth(Hp, Sh, color, sign, b, MU, KT, wl["depth"], rp, col, H=ws.H.to_scipy(),
                                    S=So.to_scipy())
    print(f"10k oracle non-orthogonal density: {time.perf_counter() - t0:.2f} s", flush=True)
    S64 = css.DeviceCSR.from_host(So.row_ptr, So.col, So.val, "cuda", torch.float64)
    pn, en, nn, _, ninfo = css.css_density_matrix_nonorth(
        css.pattern_csr(g_rp, g_col, torch.as_tensor(href["hp_val"]).cuda()),
        css.pattern_csr(g_rp, g_col, torch.as_tensor(href["y_val"]).cuda()), g_color, g_sign, g_b, MU, KT,
        wl["depth"], g_rp, g_col, bench.flags_for("fp32"), H=H32, S=S64)
    # P = S^(-1/2) X' (Eq.(9)): an error in X' reaches P through S^(-1/2), so the
    # tolerance is the X-level one times max(1, ||S^(-1/2)||_inf)
    sinf = max(1.0, float(np.max(np.abs(Sh).sum(axis=1))))
    dpn = float(np.max(np.abs(pn.cpu().numpy() - nref["p_val"])))
    dn = abs(nn - nref["n_elec"]) / abs(nref["n_elec"])
    den = abs(en - nref["e_band"]) / abs(nref["e_band"])
    print(f"10k non-orthogonal mixed: max|dP| {dpn:.3e} (||S^-1/2||_inf {sinf:.2f})  rel dN {dn:.3e}  "
          f"rel dE {den:.3e} ({ninfo['t_phase_ms']['total']:.1f} ms)", flush=True)
    assert ninfo["depth_eff"] == nref["v_eff"] and dpn <= 1e-5 * sinf and dn <= 1e-7 and den <= 1e-7


def test_1m_identities_and_mixed_against_fp64():
    """Tr P = sum_k g f(l_k) w_k and sum H.P = sum_k l_k g f(l_k) w_k hold exactly for the
    Lanczos relation; P is symmetric; the mixed path agrees with the FP64 two-pass path."""
    wl = bench.WORKLOADS["1m"]
    print("1m: generating", flush=True)
    ws = synth.water_system(wl["n_mol"], wl["seed"])
    print("1m: mixed path", flush=True)
    H32 = css.DeviceCSR.from_host(ws.H.row_ptr, ws.H.col, ws.H.val, "cuda", torch.float32)
    *_, p32, e32, t32, i32 = _gpu_step(ws, wl["seed"], H32, bench.flags_for("fp32"))
    p32 = p32.cpu()
    del H32
    torch.cuda.empty_cache()
    print("1m: fp64 two-pass path", flush=True)
    H64 = css.DeviceCSR.from_host(ws.H.row_ptr, ws.H.col, ws.H.val, "cuda", torch.float64)
    *_, p64, e64, t64, i64 = _gpu_step(ws, wl["seed"], H64, bench.flags_for("fp64", True))
    assert i32["depth_eff"] == i64["depth_eff"] == wl["depth"]
    for name, e, t, info, tol in (("fp64", e64, t64, i64, 1e-10), ("mixed", e32, t32, i32, 1e-7)):
        rt = abs(t - info["trace_krylov"]) / abs(t)
        re = abs(e - info["e_band_krylov"]) / abs(e)
        print(f"1m {name}: trace identity {rt:.2e}  energy identity {re:.2e}  asym {info['asym_max']:.2e}",
              flush=True)
        assert rt <= tol and re <= tol
    dp = float(torch.max(torch.abs(p64.cpu() - p32)))
    de = abs(e32 - e64) / abs(e64)
    print(f"1m mixed vs fp64: max|dP| {dp:.3e}  rel dE {de:.3e}", flush=True)
    assert dp <= 2e-5 and de <= 1e-7
