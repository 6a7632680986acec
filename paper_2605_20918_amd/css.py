"""Python binding of libcss (include/css.h): argument marshalling only.

Every function here takes torch tensors on a ROCm device, passes their
pointers and the current HIP stream to the C ABI, and returns tensors or
scalars. No step of the method runs in Python. When libcss.so has not been
built, loading fails loudly: there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os
import re
from dataclasses import dataclass

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libcss.so")
HEADER = os.path.join(os.path.dirname(PKG), "include", "css.h")

# status codes
CSS_OK = 0
STATUS = {0: "CSS_OK", 1: "CSS_E_ARG", 2: "CSS_E_CSR", 3: "CSS_E_WORKSPACE", 4: "CSS_E_DEVICE",
          5: "CSS_E_BREAKDOWN_AT_1", 6: "CSS_E_NONFINITE", 7: "CSS_E_EIG", 8: "CSS_E_UNSUPPORTED",
          9: "CSS_E_CAPACITY"}
CSS_F64, CSS_F32 = 0, 1

# flags
PREC_FP64 = 0x0
PREC_FP32 = 0x1
BASIS_STORED = 0x0
BASIS_TWOPASS = 0x4
REORTH_NONE = 0x0
REORTH_LOCAL = 0x8
REORTH_FULL = 0x10
CHOLQR2 = 0x20
SYMMETRIZE = 0x40
SIGNS_ONES = 0x80
SUBSPACE_EIG = 0x100
SPMM_CSR = 0x200
DIAG_ORTHO = 0x400
REORTH_ALTERNATE = 0x800

(ENTRY_COLOR, ENTRY_LANCZOS, ENTRY_DENSITY, ENTRY_SPMM, ENTRY_ENERGY_DENSITY, ENTRY_FIND_MU, ENTRY_INV_SQRT,
 ENTRY_TRANSFORM_H, ENTRY_DENSITY_NONORTH) = 0, 1, 2, 3, 4, 5, 6, 7, 8


class CssError(RuntimeError):
    def __init__(self, fn: str, code: int, msg: str):
        super().__init__(f"{fn} failed: {STATUS.get(code, code)} ({msg})")
        self.code = code


class CsrStruct(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("nnz", ctypes.c_int64), ("row_ptr", ctypes.c_void_p),
                ("col", ctypes.c_void_p), ("val", ctypes.c_void_p), ("val_dtype", ctypes.c_int32)]


class InfoStruct(ctypes.Structure):
    _fields_ = [("depth_eff", ctypes.c_int32), ("n_colors", ctypes.c_int32), ("breakdown", ctypes.c_int32),
                ("n_poles", ctypes.c_int32), ("spmm_kernel", ctypes.c_int32), ("n_evals", ctypes.c_int32),
                ("min_diag_r", ctypes.c_double), ("asym_max", ctypes.c_double),
                ("trace_krylov", ctypes.c_double), ("e_band_krylov", ctypes.c_double),
                ("t_phase_ms", ctypes.c_double * 6), ("ortho_err", ctypes.c_double),
                ("idem_defect", ctypes.c_double)]

    def as_dict(self) -> dict:
        return {"depth_eff": self.depth_eff, "n_colors": self.n_colors, "breakdown": self.breakdown,
                "n_poles": self.n_poles, "spmm_kernel": "grouped" if self.spmm_kernel else "csr",
                "min_diag_r": self.min_diag_r, "asym_max": self.asym_max, "trace_krylov": self.trace_krylov,
                "e_band_krylov": self.e_band_krylov, "ortho_err": self.ortho_err,
                "idem_defect": self.idem_defect,
                "t_phase_ms": {k: self.t_phase_ms[i] for i, k in
                               enumerate(["lanczos", "subspace", "f_pad", "reconstruction", "gather", "total"])}}


class SystemStruct(ctypes.Structure):
    _fields_ = [("H", CsrStruct), ("color", ctypes.c_void_p), ("sign", ctypes.c_void_p),
                ("n_colors", ctypes.c_int32), ("mu", ctypes.c_double), ("p_row_ptr", ctypes.c_void_p),
                ("p_col", ctypes.c_void_p), ("p_nnz", ctypes.c_int64), ("p_val", ctypes.c_void_p),
                ("e_band", ctypes.c_double), ("trace", ctypes.c_double), ("info", InfoStruct),
                ("status", ctypes.c_int32)]


class ColorJobStruct(ctypes.Structure):
    _fields_ = [("xyz", ctypes.c_void_p), ("n", ctypes.c_int32), ("box", ctypes.c_double * 3),
                ("r_cut", ctypes.c_double), ("color", ctypes.c_void_p), ("n_colors", ctypes.c_int32),
                ("p_row_ptr", ctypes.c_void_p), ("p_col", ctypes.c_void_p), ("p_nnz", ctypes.c_int64),
                ("rounds", ctypes.c_int32), ("status", ctypes.c_int32)]


class TuningStruct(ctypes.Structure):
    _fields_ = [("spmm_kernel", ctypes.c_int32), ("spmm_run", ctypes.c_int32), ("spmm_depth", ctypes.c_int32),
                ("gram_chunks", ctypes.c_int32), ("update_rows", ctypes.c_int32), ("cholqr2_series", ctypes.c_int32),
                ("reserved", ctypes.c_int32 * 2)]


SPMM_KERNELS = {"auto": 0, "grouped": 1, "csr": 2}

_lib = None


def declared_symbols() -> list[str]:
    """Entry points declared in include/css.h."""
    with open(HEADER) as f:
        text = f.read()
    return sorted(set(re.findall(r"^\s*(?:css_status|int32_t|const char\*)\s+(css_\w+)\s*\(", text, re.M)))


def load(path: str = LIB_PATH) -> ctypes.CDLL:
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with `python -m paper_2605_20918_amd.build`")
    lib = ctypes.CDLL(path)
    vp, i32, i64, u32, u64, dbl, sz = (ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32,
                                      ctypes.c_uint64, ctypes.c_double, ctypes.c_size_t)
    pcsr, pinfo = ctypes.POINTER(CsrStruct), ctypes.POINTER(InfoStruct)
    lib.css_color.argtypes = [vp, i32, ctypes.POINTER(dbl * 3), dbl, vp, ctypes.POINTER(i32), vp, vp,
                              ctypes.POINTER(i64), ctypes.POINTER(i32), vp, sz, vp]
    lib.css_build_probes.argtypes = [vp, i32, i32, u64, u32, vp, vp, vp]
    pjob = ctypes.POINTER(ColorJobStruct)
    lib.css_color_batched.argtypes = [pjob, i32, i32, vp, sz, vp]
    lib.css_color_batched_workspace_size.argtypes = [pjob, i32, i32, ctypes.POINTER(sz)]
    psys = ctypes.POINTER(SystemStruct)
    lib.css_density_matrix_batched.argtypes = [psys, i32, dbl, i32, dbl, u32, i32, vp, sz, vp]
    lib.css_batched_workspace_size.argtypes = [psys, i32, i32, u32, i32, ctypes.POINTER(sz)]
    lib.css_spmm_prepare.argtypes = [pcsr, vp, sz, vp]
    lib.css_spmm.argtypes = [pcsr, vp, vp, i32, i32, vp, sz, vp]
    ptune = ctypes.POINTER(TuningStruct)
    lib.css_set_tuning.argtypes = [ptune]
    lib.css_get_tuning.argtypes = [ptune]
    lib.css_spmm_time.argtypes = [pcsr, vp, vp, i32, i32, vp, sz, ptune, i32, ctypes.POINTER(ctypes.c_float), vp]
    lib.css_block_lanczos.argtypes = [pcsr, vp, vp, i32, i32, u32, vp, vp, pinfo, vp, sz, vp]
    lib.css_density_matrix.argtypes = [pcsr, vp, vp, i32, dbl, dbl, i32, dbl, vp, vp, i64, u32, vp,
                                       ctypes.POINTER(dbl), ctypes.POINTER(dbl), pinfo, vp, sz, vp]
    lib.css_density_matrix_noalloc.argtypes = [pcsr, vp, vp, i32, dbl, dbl, i32, dbl, vp, vp, i64, u32, vp,
                                               ctypes.POINTER(dbl), ctypes.POINTER(dbl), pinfo, vp]
    lib.css_energy_density_matrix.argtypes = [pcsr, vp, vp, i32, dbl, dbl, i32, dbl, vp, vp, i64, u32, vp, vp,
                                              ctypes.POINTER(dbl), ctypes.POINTER(dbl), ctypes.POINTER(dbl), pinfo,
                                              vp, sz, vp]
    lib.css_find_mu.argtypes = [pcsr, vp, vp, i32, dbl, dbl, i32, dbl, u32, ctypes.POINTER(dbl),
                                ctypes.POINTER(dbl), pinfo, vp, sz, vp]
    lib.css_inv_sqrt_overlap.argtypes = [pcsr, vp, vp, i32, i32, vp, vp, i64, u32, vp, ctypes.POINTER(dbl),
                                         ctypes.POINTER(dbl), pinfo, vp, sz, vp]
    lib.css_transform_hamiltonian.argtypes = [pcsr, pcsr, vp, vp, i32, i32, vp, vp, i64, u32, vp, vp,
                                              ctypes.POINTER(dbl), ctypes.POINTER(dbl), pinfo, vp, sz, vp]
    lib.css_density_matrix_nonorth.argtypes = [pcsr, pcsr, pcsr, pcsr, vp, vp, i32, dbl, dbl, i32, dbl, vp, vp, i64,
                                               u32, vp, ctypes.POINTER(dbl), ctypes.POINTER(dbl),
                                               ctypes.POINTER(dbl), pinfo, vp, sz, vp]
    lib.css_workspace_size.argtypes = [i32, i32, i64, i32, i32, u32, ctypes.POINTER(sz)]
    lib.css_fermi_poles.argtypes = [i32, vp, vp, ctypes.POINTER(i32)]
    lib.css_fermi_poles.restype = i32
    lib.css_block_ld.argtypes = [i32]
    lib.css_block_ld.restype = i32
    lib.css_status_string.argtypes = [i32]
    lib.css_status_string.restype = ctypes.c_char_p
    for name in ("css_color", "css_build_probes", "css_spmm_prepare", "css_spmm", "css_block_lanczos",
                 "css_density_matrix", "css_density_matrix_batched", "css_batched_workspace_size",
                 "css_color_batched", "css_color_batched_workspace_size",
                 "css_energy_density_matrix", "css_find_mu", "css_inv_sqrt_overlap", "css_transform_hamiltonian",
                 "css_density_matrix_nonorth", "css_workspace_size", "css_set_tuning", "css_get_tuning",
                 "css_spmm_time", "css_density_matrix_noalloc"):
        getattr(lib, name).restype = i32
    _lib = lib
    return lib


def _check(fn: str, code: int):
    if code != CSS_OK:
        raise CssError(fn, code, load().css_status_string(code).decode())


def _torch():
    import torch
    return torch


def _stream(device):
    torch = _torch()
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _ptr(t) -> ctypes.c_void_p:
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


_ws_cache: dict = {}


def workspace(nbytes: int, device):
    """A cached device byte buffer of at least nbytes (grown on demand)."""
    torch = _torch()
    key = str(device)
    buf = _ws_cache.get(key)
    if buf is None or buf.numel() < nbytes:
        _ws_cache.pop(key, None)
        buf = torch.empty(max(nbytes, 256), dtype=torch.uint8, device=device)
        _ws_cache[key] = buf
    return buf


@dataclass
class DeviceCSR:
    """CSR matrix held in device tensors (int32 row_ptr/col, float64 or float32 values)."""
    n: int
    row_ptr: object
    col: object
    val: object

    @property
    def nnz(self) -> int:
        return int(self.col.numel())

    @staticmethod
    def from_host(row_ptr, col, val, device="cuda", dtype=None):
        torch = _torch()
        rp = torch.as_tensor(row_ptr, dtype=torch.int32).to(device)
        c = torch.as_tensor(col, dtype=torch.int32).to(device)
        v = torch.as_tensor(val).to(device)
        if dtype is not None:
            v = v.to(dtype)
        return DeviceCSR(int(rp.numel()) - 1, rp.contiguous(), c.contiguous(), v.contiguous())

    def struct(self) -> CsrStruct:
        torch = _torch()
        dt = CSS_F64 if self.val.dtype == torch.float64 else CSS_F32
        return CsrStruct(self.n, self.nnz, self.row_ptr.data_ptr(), self.col.data_ptr(), self.val.data_ptr(), dt)


def fermi_poles(depth: int):
    """(kappa, weight) of the truncated continued-fraction Fermi expansion (host only)."""
    import numpy as np
    lib = load()
    n = ctypes.c_int32(0)
    _check("css_fermi_poles", lib.css_fermi_poles(depth, None, None, ctypes.byref(n)))
    kap = np.zeros(n.value)
    wgt = np.zeros(n.value)
    _check("css_fermi_poles", lib.css_fermi_poles(depth, kap.ctypes.data_as(ctypes.c_void_p),
                                                  wgt.ctypes.data_as(ctypes.c_void_p), ctypes.byref(n)))
    return kap, wgt


def block_ld(n_colors: int) -> int:
    return int(load().css_block_ld(n_colors))


def workspace_size(entry: int, n: int, nnz: int, n_colors: int, depth: int, flags: int) -> int:
    out = ctypes.c_size_t(0)
    _check("css_workspace_size", load().css_workspace_size(entry, n, nnz, n_colors, depth, flags, ctypes.byref(out)))
    return int(out.value)


_color_capacity: dict = {}


def css_color(xyz, box, r_cut: float):
    """Conflict pattern and greedy colouring. Returns (color, n_colors, p_row_ptr, p_col, rounds).

    The pattern's column array is allocated from the last size seen for this orbital
    count (+5%), so a repeated call does the work once; a first call (or one that
    outgrows the capacity) asks for the exact size first."""
    torch = _torch()
    lib = load()
    xyz = xyz.to(torch.float64).contiguous()
    n = int(xyz.shape[0])
    dev = xyz.device
    ws = workspace(workspace_size(ENTRY_COLOR, n, 0, 1, 1, 0), dev)
    boxa = (ctypes.c_double * 3)(*[float(x) for x in box])
    p_row_ptr = torch.empty(n + 1, dtype=torch.int64, device=dev)
    nnz = ctypes.c_int64(0)
    ncol = ctypes.c_int32(0)
    rounds = ctypes.c_int32(0)
    s = _stream(dev)
    color = torch.empty(n, dtype=torch.int32, device=dev)
    cap = _color_capacity.get((n, str(dev)))
    if cap is not None:
        p_col = torch.empty(cap, dtype=torch.int32, device=dev)
        nnz.value = cap
        code = lib.css_color(_ptr(xyz), n, ctypes.byref(boxa), float(r_cut), _ptr(color), ctypes.byref(ncol),
                             _ptr(p_row_ptr), _ptr(p_col), ctypes.byref(nnz), ctypes.byref(rounds), _ptr(ws),
                             ws.numel(), s)
        if code == CSS_OK:
            return color, int(ncol.value), p_row_ptr, p_col[:int(nnz.value)], int(rounds.value)
        if code != 9:                                   # anything but "capacity too small"
            _check("css_color", code)
    nnz.value = 0
    _check("css_color", lib.css_color(_ptr(xyz), n, ctypes.byref(boxa), float(r_cut), None, ctypes.byref(ncol),
                                      _ptr(p_row_ptr), None, ctypes.byref(nnz), ctypes.byref(rounds),
                                      _ptr(ws), ws.numel(), s))
    need = int(nnz.value)
    p_col = torch.empty(need, dtype=torch.int32, device=dev)
    _check("css_color", lib.css_color(_ptr(xyz), n, ctypes.byref(boxa), float(r_cut), _ptr(color),
                                      ctypes.byref(ncol), _ptr(p_row_ptr), _ptr(p_col), ctypes.byref(nnz),
                                      ctypes.byref(rounds), _ptr(ws), ws.numel(), s))
    _color_capacity[(n, str(dev))] = need + need // 20 + 64
    return color, int(ncol.value), p_row_ptr, p_col, int(rounds.value)


def css_build_probes(color, n_colors: int, seed: int, flags: int = 0):
    """Returns (sign int8[n], color_count int32[b])."""
    torch = _torch()
    n = int(color.numel())
    sign = torch.empty(n, dtype=torch.int8, device=color.device)
    counts = torch.empty(n_colors, dtype=torch.int32, device=color.device)
    _check("css_build_probes", load().css_build_probes(_ptr(color), n, n_colors, ctypes.c_uint64(seed & (2**64 - 1)),
                                                       flags, _ptr(sign), _ptr(counts), _stream(color.device)))
    return sign, counts


def css_spmm_prepare(H: DeviceCSR):
    """Row-group column unions of H for the grouped SpMM; returns the workspace tensor."""
    torch = _torch()
    nbytes = workspace_size(ENTRY_SPMM, H.n, H.nnz, 1, 1, 0)
    ws = torch.empty(nbytes, dtype=torch.uint8, device=H.row_ptr.device)
    csr = H.struct()
    _check("css_spmm_prepare", load().css_spmm_prepare(ctypes.byref(csr), _ptr(ws), nbytes,
                                                       _stream(H.row_ptr.device)))
    return ws


def css_spmm(H: DeviceCSR, V, b: int, ws=None, out=None):
    """W = H V for V of shape (n, ld) with b meaningful columns. ws from css_spmm_prepare
    selects the grouped kernel; None the CSR kernel."""
    torch = _torch()
    W = torch.empty_like(V) if out is None else out
    csr = H.struct()
    _check("css_spmm", load().css_spmm(ctypes.byref(csr), _ptr(V), _ptr(W), b, int(V.shape[1]),
                                       None if ws is None else _ptr(ws), 0 if ws is None else ws.numel(),
                                       _stream(V.device)))
    return W


TUNING_FIELDS = ("spmm_kernel", "spmm_run", "spmm_depth", "gram_chunks", "update_rows", "cholqr2_series")


def _tuning_struct(cfg: dict) -> TuningStruct:
    t = TuningStruct()
    for k, v in cfg.items():
        if k not in TUNING_FIELDS:
            raise KeyError(k)
        setattr(t, k, SPMM_KERNELS[v] if k == "spmm_kernel" and isinstance(v, str) else int(v))
    return t


def set_tuning(**cfg):
    """Process-wide launch choices (css_set_tuning); fields not given take the defaults."""
    t = _tuning_struct(cfg)
    _check("css_set_tuning", load().css_set_tuning(ctypes.byref(t)))


def reset_tuning():
    _check("css_set_tuning", load().css_set_tuning(None))


def get_tuning() -> dict:
    t = TuningStruct()
    _check("css_get_tuning", load().css_get_tuning(ctypes.byref(t)))
    names = {v: k for k, v in SPMM_KERNELS.items()}
    out = {k: getattr(t, k) for k in TUNING_FIELDS}
    out["spmm_kernel"] = names[out["spmm_kernel"]]
    return out


def css_spmm_time(H: DeviceCSR, V, b: int, ws, W, reps: int = 20, **cfg) -> float:
    """Average device milliseconds of `reps` launches of W = H V with the launch choices cfg."""
    t = _tuning_struct(cfg)
    ms = ctypes.c_float(0.0)
    csr = H.struct()
    _check("css_spmm_time", load().css_spmm_time(ctypes.byref(csr), _ptr(V), _ptr(W), b, int(V.shape[1]),
                                                 None if ws is None else _ptr(ws), 0 if ws is None else ws.numel(),
                                                 ctypes.byref(t), reps, ctypes.byref(ms), _stream(V.device)))
    return float(ms.value)


def css_block_lanczos(H: DeviceCSR, color, sign, n_colors: int, depth: int, flags: int):
    """Returns (A [v_eff, b, b], B [v_eff-1, b, b], info dict) as float64 device tensors."""
    torch = _torch()
    dev = color.device
    b = n_colors
    A = torch.zeros(depth * b * b, dtype=torch.float64, device=dev)
    B = torch.zeros(max(1, depth - 1) * b * b, dtype=torch.float64, device=dev)
    ws = workspace(workspace_size(ENTRY_LANCZOS, H.n, H.nnz, b, depth, flags), dev)
    info = InfoStruct()
    csr = H.struct()
    _check("css_block_lanczos", load().css_block_lanczos(ctypes.byref(csr), _ptr(color), _ptr(sign), b, depth, flags,
                                                         _ptr(A), _ptr(B), ctypes.byref(info), _ptr(ws), ws.numel(),
                                                         _stream(dev)))
    v = info.depth_eff
    return A[: v * b * b].view(v, b, b), B[: max(0, v - 1) * b * b].view(max(0, v - 1), b, b), info.as_dict()


def css_density_matrix(H: DeviceCSR, color, sign, n_colors: int, mu: float, kT: float, depth: int, p_row_ptr,
                       p_col, flags: int, spin_deg: float = 2.0, p_val=None):
    """Returns (p_val float64 [nnz_P], e_band, trace, info dict)."""
    torch = _torch()
    dev = color.device
    nnz = int(p_col.numel())
    if p_val is None:
        p_val = torch.empty(nnz, dtype=torch.float64, device=dev)
    ws = workspace(workspace_size(ENTRY_DENSITY, H.n, H.nnz, n_colors, depth, flags), dev)
    e_band = ctypes.c_double(0.0)
    trace = ctypes.c_double(0.0)
    info = InfoStruct()
    csr = H.struct()
    _check("css_density_matrix",
           load().css_density_matrix(ctypes.byref(csr), _ptr(color), _ptr(sign), n_colors, float(mu), float(kT),
                                     depth, float(spin_deg), _ptr(p_row_ptr), _ptr(p_col), nnz, flags, _ptr(p_val),
                                     ctypes.byref(e_band), ctypes.byref(trace), ctypes.byref(info), _ptr(ws),
                                     ws.numel(), _stream(dev)))
    return p_val, float(e_band.value), float(trace.value), info.as_dict()


def css_energy_density_matrix(H: DeviceCSR, color, sign, n_colors: int, mu: float, kT: float, depth: int,
                              p_row_ptr, p_col, flags: int, spin_deg: float = 2.0):
    """P and the energy-weighted P_E on the pattern. Returns (p_val, pe_val float64
    [nnz_P], e_band, trace, pe_trace, info dict)."""
    torch = _torch()
    dev = color.device
    nnz = int(p_col.numel())
    p_val = torch.empty(nnz, dtype=torch.float64, device=dev)
    pe_val = torch.empty(nnz, dtype=torch.float64, device=dev)
    ws = workspace(workspace_size(ENTRY_ENERGY_DENSITY, H.n, H.nnz, n_colors, depth, flags), dev)
    e_band = ctypes.c_double(0.0)
    trace = ctypes.c_double(0.0)
    pe_trace = ctypes.c_double(0.0)
    info = InfoStruct()
    csr = H.struct()
    _check("css_energy_density_matrix",
           load().css_energy_density_matrix(ctypes.byref(csr), _ptr(color), _ptr(sign), n_colors, float(mu),
                                            float(kT), depth, float(spin_deg), _ptr(p_row_ptr), _ptr(p_col), nnz,
                                            flags, _ptr(p_val), _ptr(pe_val), ctypes.byref(e_band),
                                            ctypes.byref(trace), ctypes.byref(pe_trace), ctypes.byref(info),
                                            _ptr(ws), ws.numel(), _stream(dev)))
    return p_val, pe_val, float(e_band.value), float(trace.value), float(pe_trace.value), info.as_dict()


def css_find_mu(H: DeviceCSR, color, sign, n_colors: int, n_electrons: float, kT: float, depth: int, flags: int,
                spin_deg: float = 2.0):
    """The mu at which the Krylov quadrature count equals n_electrons. Returns
    (mu, count at mu, info dict)."""
    dev = color.device
    ws = workspace(workspace_size(ENTRY_FIND_MU, H.n, H.nnz, n_colors, depth, flags), dev)
    mu = ctypes.c_double(0.0)
    count = ctypes.c_double(0.0)
    info = InfoStruct()
    csr = H.struct()
    _check("css_find_mu",
           load().css_find_mu(ctypes.byref(csr), _ptr(color), _ptr(sign), n_colors, float(n_electrons), float(kT),
                              depth, float(spin_deg), flags, ctypes.byref(mu), ctypes.byref(count),
                              ctypes.byref(info), _ptr(ws), ws.numel(), _stream(dev)))
    d = info.as_dict()
    d["t_phase_ms"] = {"lanczos": info.t_phase_ms[0], "subspace": info.t_phase_ms[1], "search": info.t_phase_ms[2],
                       "total": info.t_phase_ms[5]}
    d["n_evals"] = info.n_evals
    return float(mu.value), float(count.value), d


def css_inv_sqrt_overlap(S: DeviceCSR, color, sign, n_colors: int, depth: int, p_row_ptr, p_col, flags: int):
    """S^(-1/2) on the pattern. Returns (y_val float64 [nnz_P], trace, s_dot, info dict)."""
    torch = _torch()
    dev = color.device
    nnz = int(p_col.numel())
    y_val = torch.empty(nnz, dtype=torch.float64, device=dev)
    ws = workspace(workspace_size(ENTRY_INV_SQRT, S.n, S.nnz, n_colors, depth, flags), dev)
    trace = ctypes.c_double(0.0)
    s_dot = ctypes.c_double(0.0)
    info = InfoStruct()
    csr = S.struct()
    _check("css_inv_sqrt_overlap",
           load().css_inv_sqrt_overlap(ctypes.byref(csr), _ptr(color), _ptr(sign), n_colors, depth, _ptr(p_row_ptr),
                                       _ptr(p_col), nnz, flags, _ptr(y_val), ctypes.byref(trace), ctypes.byref(s_dot),
                                       ctypes.byref(info), _ptr(ws), ws.numel(), _stream(dev)))
    return y_val, float(trace.value), float(s_dot.value), info.as_dict()


def css_transform_hamiltonian(H: DeviceCSR, S: DeviceCSR, color, sign, n_colors: int, depth: int, p_row_ptr, p_col,
                              flags: int):
    """S^(-1/2) and H' = S^(-1/2) H S^(-1/2) on the pattern. Returns (y_val, hp_val
    float64 [nnz_P], y_trace, hp_trace, info dict)."""
    torch = _torch()
    dev = color.device
    nnz = int(p_col.numel())
    y_val = torch.empty(nnz, dtype=torch.float64, device=dev)
    hp_val = torch.empty(nnz, dtype=torch.float64, device=dev)
    ws = workspace(workspace_size(ENTRY_TRANSFORM_H, S.n, S.nnz, n_colors, depth, flags), dev)
    y_trace = ctypes.c_double(0.0)
    hp_trace = ctypes.c_double(0.0)
    info = InfoStruct()
    h_csr, s_csr = H.struct(), S.struct()
    _check("css_transform_hamiltonian",
           load().css_transform_hamiltonian(ctypes.byref(h_csr), ctypes.byref(s_csr), _ptr(color), _ptr(sign),
                                            n_colors, depth, _ptr(p_row_ptr), _ptr(p_col), nnz, flags, _ptr(y_val),
                                            _ptr(hp_val), ctypes.byref(y_trace), ctypes.byref(hp_trace),
                                            ctypes.byref(info), _ptr(ws), ws.numel(), _stream(dev)))
    return y_val, hp_val, float(y_trace.value), float(hp_trace.value), info.as_dict()


def pattern_csr(p_row_ptr, p_col, values) -> DeviceCSR:
    """A device CSR on a cutoff pattern (int64 row pointers narrowed to int32) with the
    given values, e.g. S^(-1/2) or H' from css_transform_hamiltonian."""
    torch = _torch()
    if int(p_col.numel()) >= 2 ** 31:
        raise ValueError("pattern too large for int32 row pointers")
    return DeviceCSR(int(p_row_ptr.numel()) - 1, p_row_ptr.to(torch.int32).contiguous(), p_col.contiguous(),
                     values.contiguous())


def css_density_matrix_nonorth(Hp: DeviceCSR, S_isqrt: DeviceCSR, color, sign, n_colors: int, mu: float, kT: float,
                               depth: int, p_row_ptr, p_col, flags: int, H: DeviceCSR = None, S: DeviceCSR = None,
                               spin_deg: float = 2.0):
    """Density matrix of a non-orthogonal basis on the pattern. Returns (p_val,
    e_band or None, n_elec or None, trace, info dict)."""
    torch = _torch()
    dev = color.device
    nnz = int(p_col.numel())
    p_val = torch.empty(nnz, dtype=torch.float64, device=dev)
    ws = workspace(workspace_size(ENTRY_DENSITY_NONORTH, Hp.n, Hp.nnz, n_colors, depth, flags), dev)
    e_band = ctypes.c_double(0.0)
    n_elec = ctypes.c_double(0.0)
    trace = ctypes.c_double(0.0)
    info = InfoStruct()
    structs = [Hp.struct(), S_isqrt.struct(), H.struct() if H is not None else None,
               S.struct() if S is not None else None]
    refs = [ctypes.byref(x) if x is not None else None for x in structs]
    _check("css_density_matrix_nonorth",
           load().css_density_matrix_nonorth(refs[0], refs[1], refs[2], refs[3], _ptr(color), _ptr(sign), n_colors,
                                             float(mu), float(kT), depth, float(spin_deg), _ptr(p_row_ptr),
                                             _ptr(p_col), nnz, flags, _ptr(p_val),
                                             ctypes.byref(e_band) if H is not None else None,
                                             ctypes.byref(n_elec) if S is not None else None, ctypes.byref(trace),
                                             ctypes.byref(info), _ptr(ws), ws.numel(), _stream(dev)))
    return (p_val, float(e_band.value) if H is not None else None, float(n_elec.value) if S is not None else None,
            float(trace.value), info.as_dict())


def css_density_matrix_batched(systems, kT: float, depth: int, flags: int, concurrency: int = 4,
                               spin_deg: float = 2.0, check: bool = True):
    """Independent systems in one call. `systems`: list of dicts with keys H (DeviceCSR),
    color, sign, n_colors, mu, p_row_ptr, p_col. Returns a list of (p_val, e_band, trace,
    info, status) in input order; with check, raises if any system failed."""
    torch = _torch()
    lib = load()
    n = len(systems)
    arr = (SystemStruct * n)()
    outs = []
    dev = systems[0]["color"].device
    for k, d in enumerate(systems):
        nnz_p = int(d["p_col"].numel())
        p_val = torch.empty(nnz_p, dtype=torch.float64, device=dev)
        outs.append(p_val)
        arr[k].H = d["H"].struct()
        arr[k].color = _ptr(d["color"])
        arr[k].sign = _ptr(d["sign"])
        arr[k].n_colors = int(d["n_colors"])
        arr[k].mu = float(d["mu"])
        arr[k].p_row_ptr = _ptr(d["p_row_ptr"])
        arr[k].p_col = _ptr(d["p_col"])
        arr[k].p_nnz = nnz_p
        arr[k].p_val = _ptr(p_val)
    need = ctypes.c_size_t(0)
    _check("css_batched_workspace_size",
           lib.css_batched_workspace_size(arr, n, depth, flags, concurrency, ctypes.byref(need)))
    ws = workspace(int(need.value), dev)
    code = lib.css_density_matrix_batched(arr, n, float(kT), depth, float(spin_deg), flags, concurrency, _ptr(ws),
                                          ws.numel(), _stream(dev))
    res = [(outs[k], arr[k].e_band, arr[k].trace, arr[k].info.as_dict(), arr[k].status) for k in range(n)]
    if check:
        _check("css_density_matrix_batched", code)
    return res


def css_color_batched(geoms, r_cut: float, concurrency: int = 4):
    """Colours several geometries in one call. `geoms`: list of (xyz tensor, box).
    Returns a list of (color, n_colors, p_row_ptr, p_col, rounds) as css_color does.
    Pattern capacities come from the per-size cache (first sight: the 6 A ball
    estimate); a job that outgrows its capacity is redone alone with the exact size."""
    torch = _torch()
    lib = load()
    n = len(geoms)
    arr = (ColorJobStruct * n)()
    keep = []
    dev = geoms[0][0].device
    for k, (xyz, box) in enumerate(geoms):
        xyz = xyz.to(torch.float64).contiguous()
        m = int(xyz.shape[0])
        cap = _color_capacity.get((m, str(dev)), 200 * m + 64)
        color = torch.empty(m, dtype=torch.int32, device=dev)
        p_row_ptr = torch.empty(m + 1, dtype=torch.int64, device=dev)
        p_col = torch.empty(cap, dtype=torch.int32, device=dev)
        keep.append([xyz, box, color, p_row_ptr, p_col])
        arr[k].xyz = _ptr(xyz)
        arr[k].n = m
        for i in range(3):
            arr[k].box[i] = float(box[i])
        arr[k].r_cut = float(r_cut)
        arr[k].color = _ptr(color)
        arr[k].p_row_ptr = _ptr(p_row_ptr)
        arr[k].p_col = _ptr(p_col)
        arr[k].p_nnz = cap
    need = ctypes.c_size_t(0)
    _check("css_color_batched_workspace_size",
           lib.css_color_batched_workspace_size(arr, n, concurrency, ctypes.byref(need)))
    ws = workspace(int(need.value), dev)
    code = lib.css_color_batched(arr, n, concurrency, _ptr(ws), ws.numel(), _stream(dev))
    out = []
    for k in range(n):
        xyz, box, color, p_row_ptr, p_col = keep[k]
        m = int(arr[k].n)
        if arr[k].status == 9:                           # capacity: redo alone at the exact size
            _color_capacity.pop((m, str(dev)), None)
            out.append(css_color(xyz, box, r_cut))
            continue
        _check("css_color_batched", arr[k].status)
        nnz = int(arr[k].p_nnz)
        _color_capacity[(m, str(dev))] = nnz + nnz // 20 + 64
        out.append((color, int(arr[k].n_colors), p_row_ptr, p_col[:nnz], int(arr[k].rounds)))
    if code not in (0, 9):
        _check("css_color_batched", code)
    return out
