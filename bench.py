#!/usr/bin/env python3
"""Benchmark of the CSS density-matrix path on one MI355X.

One step = the whole hot path on device-resident inputs: conflict pattern and
greedy colouring (css_color), probes (css_build_probes) and the density
matrix (css_density_matrix: block Lanczos, subspace diagonalisation, Fermi
contraction, reconstruction, gather). The metric is orbital*Krylov-steps per
second, N * v_eff / step time.

Workloads (seeded synthetic water, 6 orbitals per molecule, R_c = 6 A,
kT = 0.01 Ha, depth 40):
  10k   10 000 molecules (60 000 orbitals), mixed precision (FP32 blocks with
        full re-orthogonalisation, FP64 small matrices / eigensolve / sums);
        the FP64 path (local re-orthogonalisation) is timed beside it
  1m    1 000 000 molecules (6 000 000 orbitals), mixed precision with a stored
        basis; FP64 beside it with the two-pass (no stored basis) variant
  1k    1 000 molecules, FP64 (full re-orthogonalisation)
  batch48  48 independent boxes of 200..8000 molecules (log-uniform sizes, seed
        20922), mixed precision: all boxes coloured in one css_color_batched call,
        then all densities in one css_density_matrix_batched call; compared with
        one density call per box
Before the timed steps the launch choices are autotuned for the workload
(--no-tune keeps the built-in ones). The default run (10k) also carries, after its
timed region, sub-records for depth 60, for 10^6 molecules (one mixed step, one
FP64 two-pass step, the SpMM roofline at that size) and for the 48-box batch
(--no-sub skips them). Prints one JSON line.

--copy-calibration copies 1 GiB device to device three times and prints its
size: the reference for scaling the HBM byte counters of a profiler run.
"""
from __future__ import annotations

import argparse
import json
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

KT = 0.01
R_CUT = 6.0
MU_WATER = -0.41      # mid-gap of the water model (dense spectrum of the 1000-molecule box: -0.4095)
PEAK_HBM_GBS = 8000.0

WORKLOADS = {
    "10k": dict(n_mol=10000, seed=20921, depth=40, prec="fp32", fp64_twopass=False),
    "1m": dict(n_mol=1000000, seed=20923, depth=40, prec="fp32", fp64_twopass=True),
    # FP64 at 1 000 molecules re-orthogonalises against every block (on alternate steps):
    # at depth 40 the Krylov space spans more than half of the 6 000 orbitals, and a
    # local re-orthogonalisation loses orthogonality there (P then moves by ~3e-5 under a
    # 2e-16 perturbation of H)
    "1k": dict(n_mol=1000, seed=20920, depth=40, prec="fp64", fp64_twopass=False, reorth="full"),
    "batch48": dict(n_mol=0, seed=20922, depth=40, prec="fp32", fp64_twopass=False),
}
BATCH_SIZE_SEED = 20922
# library streams of the batched calls: 8 measured fastest for the 48 boxes (densities 201 ms, against
# 229 ms on 4, 208 ms on 16 and 299 ms on 2): the extra host workers cover each system's host checks
BATCH_STREAMS = 8
BATCH_COUNT = 48


def batch_sizes():
    rng = np.random.default_rng(BATCH_SIZE_SEED)
    return np.round(np.exp(rng.uniform(np.log(200.0), np.log(8000.0), BATCH_COUNT))).astype(int)


def run_batch(args):
    """48 uneven water boxes: colouring per box, then one batched density call.
    Returns the record (a dict)."""
    import torch
    from paper_2605_20918_amd import css, synth
    wl = WORKLOADS["batch48"]
    sizes = batch_sizes()
    dev = torch.device("cuda:0")
    boxes = []
    t_gen = time.perf_counter()
    for k, M in enumerate(sizes):
        w = synth.water_system(int(M), BATCH_SIZE_SEED * 100 + k)
        H = css.DeviceCSR.from_host(w.H.row_ptr, w.H.col, w.H.val, dev, torch.float32)
        boxes.append((w, H, torch.as_tensor(w.orb_xyz, dtype=torch.float64, device=dev),
                      [float(x) for x in w.box]))
    print(f"[bench] generated {len(boxes)} boxes, {int(sizes.sum())} molecules "
          f"({time.perf_counter() - t_gen:.0f} s)", file=sys.stderr, flush=True)
    flags = flags_for(wl["prec"])
    depth = wl["depth"]
    state = {}

    def colour_all():
        systems = []
        cols = css.css_color_batched([(xyz, box) for (w, H, xyz, box) in boxes], R_CUT, concurrency=BATCH_STREAMS)
        for k, ((w, H, xyz, box), (color, b, p_rp, p_col, _)) in enumerate(zip(boxes, cols)):
            sign, _ = css.css_build_probes(color, b, BATCH_SIZE_SEED * 100 + k)
            systems.append(dict(H=H, color=color, sign=sign, n_colors=b, mu=MU_WATER, p_row_ptr=p_rp, p_col=p_col))
        return systems

    def step():
        t0 = time.perf_counter()
        systems = colour_all()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        res = css.css_density_matrix_batched(systems, KT, depth, flags, concurrency=BATCH_STREAMS)
        torch.cuda.synchronize()
        state.update(systems=systems, res=res, t_colour=t1 - t0, t_density=time.perf_counter() - t1)

    for i in range(args.warmup):
        step()
        print(f"[bench] warmup {i + 1}/{args.warmup} done", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    tc = td = 0.0
    for i in range(args.steps):
        step()
        tc += state["t_colour"]
        td += state["t_density"]
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / args.steps
    systems, res = state["systems"], state["res"]
    work = sum(int(d["H"].n) * r[3]["depth_eff"] for d, r in zip(systems, res))
    # the same densities, one call per box
    torch.cuda.synchronize()
    ts = time.perf_counter()
    seq = []
    for d in systems:
        seq.append(css.css_density_matrix(d["H"], d["color"], d["sign"], d["n_colors"], d["mu"], KT, depth,
                                          d["p_row_ptr"], d["p_col"], flags))
    torch.cuda.synchronize()
    ts = time.perf_counter() - ts
    same = all(torch.equal(a[0], b[0]) and a[1] == b[1] for a, b in zip(res, seq))
    out = {
        "metric": "aggregate orbital*Krylov-steps/s (48 boxes: colouring + batched P-build)",
        "value": work / dt, "unit": "orbital*steps/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": dt * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32+f64", "data": "synthetic",
        "config": {"workload": f"{BATCH_COUNT} water boxes of {int(sizes.min())}..{int(sizes.max())} molecules "
                               f"({int(sizes.sum())} in all, {sum(int(d['H'].n) for d in systems)} orbitals), "
                               f"fp32 blocks, depth {depth}",
                   "sizes": [int(x) for x in sizes], "flags": flags, "concurrency": BATCH_STREAMS},
        "colour_ms_per_step": tc / args.steps * 1e3,
        "batched_density_ms": td / args.steps * 1e3,
        "sequential_density_ms": ts * 1e3,
        "batched_vs_sequential_density": ts / (td / args.steps),
        "density_rate_batched": work / (td / args.steps),
        "density_rate_sequential": work / ts,
        "batched_equals_sequential_bitwise": same,
    }
    return out

# HBM bytes per launch of the grouped SpMM from FETCH_SIZE + WRITE_SIZE counter runs
# (scaled by a 1 GiB copy), valid while the kernel source hashes to the recorded value
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "spmm_grp_traffic_{}.json")


# One Cholesky QR per step (no repetition): with re-orthogonalisation the basis keeps
# the same orthogonality as with CholQR2 on these inputs (measured, 10k mixed: 3.5e-6
# either way), and the FP64 comparators use the same choice.
BENCH_CHOLQR2 = False


def flags_for(prec: str, twopass: bool = False, reorth: str = "local"):
    """Mixed path: re-orthogonalisation against every block on alternate steps (against
    the previous two on the others). FP64 path: local (the previous two blocks) unless
    `reorth` is "full" (then the same alternating schedule); local suffices while the
    Krylov space is a small part of the orbital space (10^4 and 10^6 molecules at depth
    40). Cholesky QR once per step in both (BENCH_CHOLQR2)."""
    from paper_2605_20918_amd import css
    alternate = css.REORTH_FULL | css.REORTH_ALTERNATE
    qr = css.CHOLQR2 if BENCH_CHOLQR2 else 0
    if prec == "fp32":
        return css.PREC_FP32 | alternate | qr | css.SYMMETRIZE
    ro = alternate if reorth == "full" else css.REORTH_LOCAL
    return css.PREC_FP64 | ro | qr | css.SYMMETRIZE | (css.BASIS_TWOPASS if twopass else 0)


def kernel_hash() -> str:
    import hashlib
    with open(os.path.join(ROOT, "paper_2605_20918_amd", "csrc", "spmm_grp.hip"), "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def measured_traffic(workload: str):
    """HBM bytes per launch from the committed counter summary, or None."""
    try:
        with open(TRAFFIC_FILE.format(workload)) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("kernel_sha256_16") != kernel_hash() or t.get("workload") != workload:
        return None
    return t.get("bytes_per_launch")


def copy_calibration():
    import torch
    n = 1 << 30
    src = torch.ones(n, dtype=torch.uint8, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes": n, "copies": 3}), flush=True)


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or "unknown"


def cpu_baseline(ws, depth_sample: int, mu: float):
    """The oracle, as it stands, on the same workload at depth depth_sample (the whole
    step at the workload's depth for the 10k and 1k inputs)."""
    from threadpoolctl import threadpool_info
    from oracle import density as D
    from oracle.coloring import greedy_color
    from oracle.pattern import conflict_pattern
    from oracle.probes import probe_signs
    H = ws.H.to_scipy()
    t0 = time.perf_counter()
    rp, col, deg = conflict_pattern(ws.orb_xyz, ws.box, R_CUT)
    color, b = greedy_color(rp, col, deg)
    sign = probe_signs(ws.n, ws.seed)
    r = D.density_matrix(H, color, sign, b, mu, KT, depth_sample, rp, col, reorth="alternate",
                         cholqr2=BENCH_CHOLQR2)
    dt = time.perf_counter() - t0
    threads = max([int(i.get("num_threads", 1)) for i in threadpool_info()] or [1])
    return {"value": ws.n * r["v_eff"] / dt, "unit": "orbital*steps/s", "cores": threads, "kind": "oracle",
            "sample": f"same {ws.n_mol}-molecule input at depth {depth_sample} (v_eff={r['v_eff']}): pattern, "
                      f"colouring, block Lanczos (full re-orthogonalisation on alternate steps, as the GPU "
                      f"step), eigensolve, contraction, gather; {dt:.1f} s; "
                      f"BLAS threads {threads}, SciPy SpMM single-threaded; host {cpu_model()}, nproc {os.cpu_count()}"}


def spmm_roofline(css, H, ws_n: int, nnz: int, b: int, tdt, label: str, grouped: bool):
    """The SpMM of the Lanczos steps (same kernel and launch shape), timed with events
    on the stream it is launched on; algorithmic bytes nnz (val + col) + row pointers
    + one read of V and one write of W (N x b)."""
    import torch
    dev = H.row_ptr.device
    ld = css.block_ld(b)
    V = torch.zeros((ws_n, ld), dtype=tdt, device=dev)
    V[:, :b] = torch.randn((ws_n, b), dtype=tdt, device=dev)
    W = torch.empty_like(V)
    spmm_ws = css.css_spmm_prepare(H) if grouped else None      # the kernel the Lanczos steps ran
    for _ in range(3):
        css.css_spmm(H, V, b, ws=spmm_ws, out=W)
    reps = 50 if ws_n < 10 ** 6 else 20
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        css.css_spmm(H, V, b, ws=spmm_ws, out=W)
    e1.record()
    torch.cuda.synchronize()
    t_spmm = e0.elapsed_time(e1) / reps * 1e-3
    s_val = 4 if tdt == torch.float32 else 8
    bytes_alg = nnz * (s_val + 4) + 4 * (ws_n + 1) + 2 * ws_n * b * s_val
    achieved = bytes_alg / t_spmm / 1e9
    del V, W, spmm_ws
    return {"bound": "hbm", "label": label, "kernel": "k_spmm_grp" if grouped else "k_spmm_csr",
            "achieved": achieved, "peak": PEAK_HBM_GBS, "unit": "GB/s", "frac": achieved / PEAK_HBM_GBS,
            "bytes_per_launch": bytes_alg, "avg_launch_us": t_spmm * 1e6, "grouped": grouped}


def timed_call(torch, fn, reps: int = 1):
    """fn() once untimed, then the mean wall time of `reps` calls (device synchronised)."""
    r = fn()
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(reps):
        r = fn()
    torch.cuda.synchronize()
    return r, (time.perf_counter() - t) / reps


def measure_single(name: str, steps: int, warmup: int, extras: bool, fp64: bool, tune: bool,
                   cpu: bool, depth60: bool = False):
    """One workload: `steps` timed steps of colouring + probes + density matrix on
    device-resident inputs, then the sub-measurements. Returns the record (a dict)."""
    import torch
    from paper_2605_20918_amd import autotune, css, synth
    wl = WORKLOADS[name]
    print(f"[bench] {name}: generating {wl['n_mol']} molecules", file=sys.stderr, flush=True)
    t_gen = time.perf_counter()
    ws = synth.water_system(wl["n_mol"], wl["seed"], progress=lambda m: print(
        f"[bench] generator: {m} ({time.perf_counter() - t_gen:.0f} s)", file=sys.stderr, flush=True))
    dev = torch.device("cuda:0")
    tdt = torch.float32 if wl["prec"] == "fp32" else torch.float64
    H = css.DeviceCSR.from_host(ws.H.row_ptr, ws.H.col, ws.H.val, dev, tdt)
    xyz = torch.as_tensor(ws.orb_xyz, dtype=torch.float64, device=dev)
    box = [float(x) for x in ws.box]
    flags = flags_for(wl["prec"], reorth=wl.get("reorth", "local"))
    depth = wl["depth"]
    mu = MU_WATER
    state = {}

    def colour():
        color, b, p_rp, p_col, rounds = css.css_color(xyz, box, R_CUT)
        sign, _ = css.css_build_probes(color, b, wl["seed"])
        return color, b, p_rp, p_col, rounds, sign

    css.reset_tuning()
    tuning = None
    if tune:
        # launch choices for this workload shape, swept on the library's own kernels
        color, b, _, _, _, sign = colour()
        res = autotune.autotune(H, color, sign, b, depth, flags, write=False,
                                lanczos_depth=depth if ws.n < 10 ** 6 else 4)
        tuning = {"choice": res["choice"], "seconds": res["seconds"],
                  "spmm_ms_best": min(t["ms"] for t in res["spmm_trials"]),
                  "spmm_ms_default": next((t["ms"] for t in res["spmm_trials"]
                                           if t["config"].get("spmm_run") == 512 and t["config"].get("spmm_depth") == 4),
                                          None),
                  "spmm_trials": len(res["spmm_trials"]), "lanczos_trials": len(res["lanczos_trials"])}
        print(f"[bench] tuned in {res['seconds']:.1f} s: {res['choice']}", file=sys.stderr, flush=True)
        del color, sign

    def step(fl=flags, d=depth):
        color, b, p_rp, p_col, rounds, sign = colour()
        p_val, e_band, trace, info = css.css_density_matrix(H, color, sign, b, mu, KT, d, p_rp, p_col, fl)
        state.update(b=b, nnz_p=int(p_col.numel()), rounds=rounds, e_band=e_band, trace=trace, info=info,
                     p_val=p_val)

    for i in range(warmup):
        step()
        print(f"[bench] warmup {i + 1}/{warmup} done", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(steps):
        step()
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    info = state["info"]
    v_eff = info["depth_eff"]
    b = state["b"]
    print(f"[bench] {name}: timed {steps} steps: {dt * 1e3:.2f} ms/step", file=sys.stderr, flush=True)

    # colouring alone (css_color) for the phase table
    _, t_color = timed_call(torch, lambda: css.css_color(xyz, box, R_CUT))
    nnz = ws.H.nnz
    big = ws.n >= 10 ** 6
    roof = spmm_roofline(css, H, ws.n, nnz, b, tdt,
                         "HBM-streaming (working set far above the 256 MB last-level cache)" if big else
                         "effective (MALL-resident): the 10k working set fits the 256 MB last-level cache",
                         info["spmm_kernel"] == "grouped")
    roof["traffic"] = measured_traffic(name) if roof["grouped"] else None
    roof["kernel_sha256_16"] = kernel_hash()

    out = {
        "metric": "orbital*Krylov-steps/s (P-build incl. colouring)",
        "value": ws.n * v_eff / dt,
        "unit": "orbital*steps/s",
        "n_gpus": 1, "steps": steps, "warmup": warmup,
        "ms_per_step": dt * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32+f64" if wl["prec"] == "fp32" else "f64",
        "dtype_detail": ("H and Krylov blocks FP32; SpMM FP32 (FP32 MFMA, FP32 accumulation); Gram and block "
                         "updates on BF16/FP16 MFMA with operands split in 2-3 parts (FP32-accurate terms), "
                         "FP32 partial sums reduced in FP64; Cholesky, T, subspace solve, gather, sums FP64")
        if wl["prec"] == "fp32" else "FP64 throughout (FP64 MFMA for the block products)",
        "data": "synthetic",
        "config": {"workload": f"water {wl['n_mol']} H2O ({ws.n} orbitals), {wl['prec']} blocks, depth {depth}",
                   "n_orbitals": ws.n, "nnz_H": nnz, "nnz_P": state["nnz_p"], "n_colors": b,
                   "depth": depth, "depth_eff": v_eff, "kT": KT, "mu": mu, "r_cut": R_CUT,
                   "flags": flags,
                   "reorth": ("full on alternate steps, local between" if flags & css.REORTH_ALTERNATE else "full")
                   if flags & css.REORTH_FULL else "local"},
        "phases_ms": {**info["t_phase_ms"], "colour_probe_total": t_color * 1e3,
                      "colour_rounds": state["rounds"]},
        "trace": state["trace"], "e_band": state["e_band"], "trace_krylov": info["trace_krylov"],
        "idem_defect_per_electron": info["idem_defect"] / state["trace"],
        "roofline": roof,
    }
    if tuning is not None:
        out["tuning"] = tuning
    # loss of orthogonality of the basis the timed step builds (an extra, untimed call)
    color, bb, p_rp, p_col, _, sign = colour()
    _, _, _, dinfo = css.css_density_matrix(H, color, sign, bb, mu, KT, depth, p_rp, p_col, flags | css.DIAG_ORTHO)
    out["ortho_err"] = dinfo["ortho_err"]
    del dinfo

    if extras:
        dm_args = (H, color, sign, bb, mu, KT, depth, p_rp, p_col, flags)
        _, t_d = timed_call(torch, lambda: css.css_density_matrix(*dm_args))
        r, t_e = timed_call(torch, lambda: css.css_energy_density_matrix(*dm_args))
        _, _, _, _, pe_trace, einfo = r
        out["energy_weighted"] = {"extra_ms": (t_e - t_d) * 1e3, "density_ms": t_d * 1e3, "energy_ms": t_e * 1e3,
                                  "pe_trace": pe_trace, "e_band_krylov": einfo["e_band_krylov"]}
        del r
        # mu for the workload's electron count from the Krylov quadrature
        (mu_k, count_k, minfo), t_mu = timed_call(
            torch, lambda: css.css_find_mu(H, color, sign, bb, float(ws.n_electrons), KT, depth, flags))
        out["mu_search"] = {"ms": t_mu * 1e3, "mu": mu_k, "count": count_k, "n_electrons": ws.n_electrons,
                            "mu_used": mu, "phase_ms": minfo["t_phase_ms"], "count_evaluations": minfo["n_evals"]}
        # S^(-1/2) of the overlap matrix on the same pattern (non-orthogonal basis), v^s = 10
        So = synth.water_overlap(ws)
        Sdev = css.DeviceCSR.from_host(So.row_ptr, So.col, So.val, dev, torch.float32)
        inv_args = (Sdev, color, sign, bb, 10, p_rp, p_col, flags)
        (_, ytr, _, yinfo), t_y = timed_call(torch, lambda: css.css_inv_sqrt_overlap(*inv_args))
        out["inv_sqrt_overlap"] = {"ms": t_y * 1e3, "depth": 10, "depth_eff": yinfo["depth_eff"], "trace": ytr,
                                   "phase_ms": yinfo["t_phase_ms"]}
        (y_s, hp_s, _, _, _), t_h = timed_call(torch, lambda: css.css_transform_hamiltonian(H, *inv_args))
        out["transform_hamiltonian"] = {"ms": t_h * 1e3, "depth": 10}
        # density matrix of the non-orthogonal basis from that S^(-1/2) and H'
        no_args = (css.pattern_csr(p_rp, p_col, hp_s), css.pattern_csr(p_rp, p_col, y_s), color, sign, bb, mu, KT,
                   depth, p_rp, p_col, flags)
        (_, e_no, n_no, _, ninfo), t_n = timed_call(
            torch, lambda: css.css_density_matrix_nonorth(*no_args, H=H, S=Sdev))
        out["density_nonorth"] = {"ms": t_n * 1e3, "depth_eff": ninfo["depth_eff"], "n_elec": n_no, "e_band": e_no,
                                  "phase_ms": ninfo["t_phase_ms"]}
        del y_s, hp_s, no_args, Sdev

    if depth60:
        # the same input at Krylov depth 60 (mixed, timed) against FP64 at depth 60
        state.clear()
        step(flags, 60)
        torch.cuda.synchronize()
        t = time.perf_counter()
        step(flags, 60)
        torch.cuda.synchronize()
        t60 = time.perf_counter() - t
        p60, e60, i60 = state["p_val"].double().cpu(), state["e_band"], state["info"]
        # at depth 60 local re-orthogonalisation in FP64 loses orthogonality (max|Q^T Q - I|
        # about 1e-2 at 10^4 molecules), so the comparator re-orthogonalises against every
        # block (on alternate steps)
        f64 = flags_for("fp64", reorth="full")
        H64 = css.DeviceCSR.from_host(ws.H.row_ptr, ws.H.col, ws.H.val, dev, torch.float64)
        (q64, e64, _, i64), t64 = timed_call(
            torch, lambda: css.css_density_matrix(H64, color, sign, bb, mu, KT, 60, p_rp, p_col, f64 | css.DIAG_ORTHO))
        out["depth60"] = {"ms_per_step": t60 * 1e3, "value": ws.n * i60["depth_eff"] / t60,
                          "depth_eff": i60["depth_eff"], "phases_ms": i60["t_phase_ms"],
                          "fp64_density_ms": t64 * 1e3, "fp64_mode": "FP64, full re-orthogonalisation on alternate steps, stored basis",
                          "fp64_ortho_err": i64["ortho_err"],
                          "mixed_vs_fp64_max_abs_dP": float(torch.max(torch.abs(q64.cpu() - p60))),
                          "mixed_vs_fp64_rel_dE": abs(e60 - e64) / abs(e64),
                          "idem_defect_per_electron": i60["idem_defect"] / state["trace"]}
        del H64, q64, p60
        print(f"[bench] depth 60: {t60 * 1e3:.1f} ms mixed, {t64 * 1e3:.1f} ms FP64", file=sys.stderr, flush=True)

    if wl["prec"] == "fp32" and fp64:
        step()
        p_mixed = state["p_val"].double().cpu()
        e_mixed = state["e_band"]
        del state["p_val"]
        H64 = css.DeviceCSR.from_host(ws.H.row_ptr, ws.H.col, ws.H.val, dev, torch.float64)
        f64 = flags_for("fp64", wl["fp64_twopass"])
        res = {}

        def step64():
            c, b64, rp64, col64, _, sg = colour()
            res["p"], res["e"], _, res["info"] = css.css_density_matrix(H64, c, sg, b64, mu, KT, depth, rp64, col64,
                                                                         f64)
        _, t64 = timed_call(torch, step64)
        dp = float(torch.max(torch.abs(res["p"].cpu() - p_mixed)))
        out["fp64_ms_per_step"] = t64 * 1e3
        out["fp64_flags"] = f64
        out["fp64_mode"] = ("FP64, local re-orthogonalisation (previous two blocks), "
                            + ("two-pass (no stored basis)" if wl["fp64_twopass"] else "stored basis"))
        out["fp64_phases_ms"] = res["info"]["t_phase_ms"]
        out["mixed_vs_fp64_speedup"] = t64 / dt
        out["mixed_vs_fp64_max_abs_dP"] = dp
        out["mixed_vs_fp64_rel_dE"] = abs(e_mixed - res["e"]) / abs(res["e"])
        del H64, res

    if cpu:
        print("[bench] timing the oracle on the CPU sample", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(ws, depth, mu)       # the whole step (about 15 s on 16 cores)
    css.reset_tuning()
    del H, xyz, state
    torch.cuda.empty_cache()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="10k", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the 10k-only extra entry points (energy-weighted, mu, S^-1/2, H', "
                         "non-orthogonal) after the timed region")
    ap.add_argument("--no-sub", action="store_true",
                    help="10k: skip the sub-records (depth 60, 10^6 molecules, 48-box batch)")
    ap.add_argument("--no-tune", action="store_true", help="keep the built-in launch choices")
    ap.add_argument("--copy-calibration", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {args.gpus} is not supported "
              "(the multi-GPU sharding is described in DESIGN.md, not built)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2605_20918_amd import css
    if not torch.cuda.is_available():
        print("no ROCm device visible", file=sys.stderr)
        sys.exit(1)
    css.load()
    if args.copy_calibration:
        copy_calibration()
        return
    if args.workload == "batch48":
        print(json.dumps(run_batch(args)), flush=True)
        return
    name = args.workload
    sub = name == "10k" and not args.no_sub
    out = measure_single(name, args.steps, args.warmup, extras=name == "10k" and not args.no_extras,
                         fp64=not args.no_fp64, tune=not args.no_tune,
                         cpu=not args.no_cpu_baseline and name != "1m", depth60=sub)
    if sub:
        # the 10^6-molecule P-build (mixed, then FP64 two-pass) and its SpMM roofline
        one_m = measure_single("1m", 1, 1, extras=False, fp64=True, tune=not args.no_tune, cpu=False)
        out["roofline_1m"] = one_m.pop("roofline")
        keep = ("value", "ms_per_step", "config", "phases_ms", "trace", "e_band", "idem_defect_per_electron",
                "ortho_err", "tuning", "fp64_ms_per_step", "fp64_mode", "fp64_phases_ms", "mixed_vs_fp64_speedup",
                "mixed_vs_fp64_max_abs_dP", "mixed_vs_fp64_rel_dE")
        out["1m"] = {k: one_m[k] for k in keep if k in one_m}
        # 48 uneven boxes in one batched call against one call per box
        bargs = argparse.Namespace(steps=2, warmup=1)
        b48 = run_batch(bargs)
        out["batch48"] = {k: b48[k] for k in ("value", "ms_per_step", "colour_ms_per_step", "batched_density_ms",
                                             "sequential_density_ms", "batched_vs_sequential_density",
                                             "batched_equals_sequential_bitwise") if k in b48}
        out["batch48"]["workload"] = b48["config"]["workload"]
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
