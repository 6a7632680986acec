"""Autotuner for the launch choices of the density-matrix path (css_tuning).

It times the library's own kernels on the caller's workload and keeps the fastest
launch shape, for the two places where the shape is a free choice:

* the sparse x block product W = H V (the product the method reduces to): kernel
  (16-row grouped MFMA kernel or row-parallel CSR), row groups per XCD run, and
  k-steps in flight per wavefront; timed with css_spmm_time on the block shape the
  Lanczos steps use;
* the FP32 split block products of the Lanczos steps: row chunks of the split Gram
  (work-groups per compute unit) and rows per work-group of the split update;
  timed as whole css_block_lanczos passes (the objective itself).

No choice changes the arithmetic of the method, only launch shapes and hence the
order of FP32 partial sums. Results go to a JSON cache keyed by (arch, N, nnz per
row, b, precision); `apply_cached` sets a cached choice before a density build.
The timing and the kernels are the library's; this module only sweeps and records.
"""
from __future__ import annotations

import json
import os
import time

from . import css

CACHE_ENV = "CSS_TUNE_CACHE"
DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "css_tune.json")

SPMM_RUNS = (64, 128, 256, 512, 1024, 4096)
SPMM_DEPTHS = (4, 8)
GRAM_CHUNKS = (1, 2, 4)
UPDATE_ROWS = (64, 128)


def cache_path(path: str | None = None) -> str:
    return path or os.environ.get(CACHE_ENV) or DEFAULT_CACHE


def arch_name() -> str:
    import torch
    props = torch.cuda.get_device_properties(torch.cuda.current_device())
    return str(getattr(props, "gcnArchName", props.name)).split(":")[0]


def key(n: int, nnz: int, n_colors: int, precision: str) -> str:
    return f"{arch_name()}|N={n}|nnz/row={nnz / max(1, n):.1f}|b={n_colors}|{precision}"


def load_cache(path: str | None = None) -> dict:
    try:
        with open(cache_path(path)) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def save_cache(entries: dict, path: str | None = None) -> None:
    p = cache_path(path)
    os.makedirs(os.path.dirname(p) or ".", exist_ok=True)
    tmp = p + ".tmp"
    with open(tmp, "w") as f:
        json.dump(entries, f, indent=1, sort_keys=True)
    os.replace(tmp, p)


def apply_cached(n: int, nnz: int, n_colors: int, precision: str, path: str | None = None) -> dict | None:
    """Set the cached launch choice for this workload shape; None (defaults kept) if absent."""
    entry = load_cache(path).get(key(n, nnz, n_colors, precision))
    if entry is None:
        return None
    css.set_tuning(**entry["choice"])
    return entry["choice"]


def tune_spmm(H: css.DeviceCSR, n_colors: int, reps: int = 30) -> tuple[dict, list]:
    """Fastest SpMM launch for H times an N x ld block (random values, the Lanczos
    block shape). Returns (choice, [(config, ms), ...])."""
    import torch
    ld = css.block_ld(n_colors)
    g = torch.Generator(device=H.row_ptr.device).manual_seed(0)
    V = torch.zeros((H.n, ld), dtype=H.val.dtype, device=H.row_ptr.device)
    V[:, :n_colors] = torch.randn((H.n, n_colors), dtype=H.val.dtype, device=V.device, generator=g)
    W = torch.empty_like(V)
    try:
        ws = css.css_spmm_prepare(H)
    except css.CssError:
        ws = None
    trials = [({"spmm_kernel": "csr"}, css.css_spmm_time(H, V, n_colors, None, W, reps=reps, spmm_kernel="csr"))]
    if ws is not None:
        for run in SPMM_RUNS:
            for depth in SPMM_DEPTHS:
                cfg = {"spmm_kernel": "grouped", "spmm_run": run, "spmm_depth": depth}
                trials.append((cfg, css.css_spmm_time(H, V, n_colors, ws, W, reps=reps, **cfg)))
    best = min(trials, key=lambda t: t[1])[0]
    del V, W, ws
    return dict(best), trials


def tune_lanczos(H: css.DeviceCSR, color, sign, n_colors: int, depth: int, flags: int, spmm: dict,
                 reps: int = 2) -> tuple[dict, list]:
    """Fastest split Gram / update launch (FP32 only) for whole Lanczos passes with the
    SpMM choice `spmm`. Returns (choice, [(config, ms), ...])."""
    import torch
    trials = []
    if not flags & css.PREC_FP32:
        return {}, trials
    for gc in GRAM_CHUNKS:
        for ur in UPDATE_ROWS:
            cfg = {**spmm, "gram_chunks": gc, "update_rows": ur}
            css.set_tuning(**cfg)
            css.css_block_lanczos(H, color, sign, n_colors, depth, flags)      # untimed
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(reps):
                css.css_block_lanczos(H, color, sign, n_colors, depth, flags)
            torch.cuda.synchronize()
            trials.append((cfg, (time.perf_counter() - t0) / reps * 1e3))
    best = min(trials, key=lambda t: t[1])[0]
    return {k: v for k, v in best.items() if k in ("gram_chunks", "update_rows")}, trials


def autotune(H: css.DeviceCSR, color, sign, n_colors: int, depth: int, flags: int, path: str | None = None,
             lanczos_depth: int | None = None, write: bool = True) -> dict:
    """Sweep, record in the cache and apply the fastest launch choice for this workload.

    lanczos_depth: depth of the timed Lanczos passes (default: depth); a smaller one
    keeps the sweep short on large systems. Returns {"key", "choice", "spmm_trials",
    "lanczos_trials", "seconds"}."""
    t0 = time.perf_counter()
    precision = "fp32" if flags & css.PREC_FP32 else "fp64"
    css.reset_tuning()
    spmm, spmm_trials = tune_spmm(H, n_colors)
    rest, lz_trials = tune_lanczos(H, color, sign, n_colors, lanczos_depth or depth, flags, spmm)
    choice = {**spmm, **rest}
    css.set_tuning(**choice)
    k = key(H.n, H.nnz, n_colors, precision)
    out = {"key": k, "choice": choice,
           "spmm_trials": [{"config": c, "ms": ms} for c, ms in spmm_trials],
           "lanczos_trials": [{"config": c, "ms": ms} for c, ms in lz_trials],
           "seconds": time.perf_counter() - t0}
    if write:
        entries = load_cache(path)
        entries[k] = {"choice": choice, "spmm_ms": min(ms for _, ms in spmm_trials),
                      "lanczos_ms": min((ms for _, ms in lz_trials), default=None)}
        save_cache(entries, path)
    return out
