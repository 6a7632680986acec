"""css_density_matrix_noalloc through the C ABI against css_density_matrix: the same
results bitwise, on two calls in a row (the second system smaller than the first),
in FP64 and in the mixed precision."""
import ctypes

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from paper_2605_20918_amd import css  # noqa: E402

from gpu_common import KT, dev_i8, dev_i32, dev_i64, to_dev, water_case  # noqa: E402

FLAGS = {"fp64": css.PREC_FP64 | css.REORTH_FULL | css.CHOLQR2 | css.SYMMETRIZE,
         "fp32": css.PREC_FP32 | css.REORTH_FULL | css.CHOLQR2 | css.SYMMETRIZE}


def setup_module(module):
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    css.load()


def _noalloc(H, color, sign, b, mu, depth, rp, col, flags):
    lib = css.load()
    nnz = int(col.numel())
    p_val = torch.empty(nnz, dtype=torch.float64, device="cuda")
    e_band, trace = ctypes.c_double(0.0), ctypes.c_double(0.0)
    info = css.InfoStruct()
    csr = H.struct()
    torch.cuda.synchronize()
    code = lib.css_density_matrix_noalloc(ctypes.byref(csr), css._ptr(color), css._ptr(sign), b, float(mu), KT,
                                          depth, 2.0, css._ptr(rp), css._ptr(col), nnz, flags, css._ptr(p_val),
                                          ctypes.byref(e_band), ctypes.byref(trace), ctypes.byref(info),
                                          css._stream(color.device))
    return code, p_val, e_band.value, trace.value, info


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_noalloc_equals_workspace_call_twice_shrinking(prec):
    flags = FLAGS[prec]
    dtype = torch.float64 if prec == "fp64" else torch.float32
    for M, seed in ((216, 3), (64, 20919)):           # the second call has a smaller input
        print(f"noalloc {prec} M={M}", flush=True)
        ws, H, rp, col, color, b, sign, mu = water_case(M, seed)
        Hd, cd, sd, rpd, cold = to_dev(ws, dtype), dev_i32(color), dev_i8(sign), dev_i64(rp), dev_i32(col)
        code, p_na, e_na, t_na, info = _noalloc(Hd, cd, sd, b, mu, 40, rpd, cold, flags)
        assert code == 0, css.load().css_status_string(code)
        p_ws, e_ws, t_ws, i_ws = css.css_density_matrix(Hd, cd, sd, b, mu, KT, 40, rpd, cold, flags)
        assert torch.equal(p_na, p_ws), float(torch.max(torch.abs(p_na - p_ws)))
        assert e_na == e_ws and t_na == t_ws
        assert info.depth_eff == i_ws["depth_eff"] and info.n_colors == b
        assert all(x == 0.0 for x in info.t_phase_ms)


def test_noalloc_rejects_the_dense_eigensolver():
    ws, H, rp, col, color, b, sign, mu = water_case(64, 20919)
    code, *_ = _noalloc(to_dev(ws), dev_i32(color), dev_i8(sign), b, mu, 40, dev_i64(rp), dev_i32(col),
                        FLAGS["fp64"] | css.SUBSPACE_EIG)
    assert code == 8
