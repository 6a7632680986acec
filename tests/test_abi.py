"""The C-ABI library loads and exports every entry point include/css.h declares (CPU only)."""
import ctypes
import os

import pytest

from paper_2605_20918_amd import css

pytestmark = pytest.mark.skipif(not os.path.exists(css.LIB_PATH), reason="libcss.so not built")


def test_every_declared_symbol_is_exported():
    names = css.declared_symbols()
    assert {"css_color", "css_build_probes", "css_block_lanczos", "css_density_matrix", "css_spmm",
            "css_spmm_prepare", "css_workspace_size", "css_status_string", "css_block_ld",
            "css_density_matrix_batched", "css_batched_workspace_size", "css_color_batched",
            "css_color_batched_workspace_size", "css_energy_density_matrix", "css_find_mu",
            "css_inv_sqrt_overlap", "css_transform_hamiltonian", "css_density_matrix_nonorth"} <= set(names)
    lib = ctypes.CDLL(css.LIB_PATH)
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing


def test_host_only_entry_points():
    lib = css.load()
    assert lib.css_status_string(0) == b"ok"
    assert lib.css_status_string(3) == b"workspace too small"
    assert lib.css_status_string(1234) == b"unknown status"
    assert [lib.css_block_ld(b) for b in (1, 16, 17, 88, 256, 257, 300, 513)] == [16, 16, 32, 96, 256, 288, 320, 576]


def test_argument_errors_before_any_device_work():
    lib = css.load()
    assert lib.css_build_probes(None, 0, 1, 0, 0, None, None, None) == 1
    assert lib.css_spmm(None, None, None, 1, 16, None, 0, None) == 1
    assert lib.css_spmm_prepare(None, None, 0, None) == 1
    assert lib.css_density_matrix_batched(None, 0, 0.01, 4, 2.0, 0, 4, None, 0, None) == 1
    out_b = ctypes.c_size_t(0)
    assert lib.css_batched_workspace_size(None, 0, 4, 0, 4, ctypes.byref(out_b)) == 1
    out = ctypes.c_size_t(0)
    assert lib.css_workspace_size(0, 0, 0, 1, 1, 0, ctypes.byref(out)) == 1
    # the energy-weighted call needs the density workspace and one more N x ld block;
    # without its output array it is an argument error
    d = ctypes.c_size_t(0)
    e = ctypes.c_size_t(0)
    assert lib.css_workspace_size(css.ENTRY_DENSITY, 1000, 50000, 40, 10, css.PREC_FP32, ctypes.byref(d)) == 0
    assert lib.css_workspace_size(css.ENTRY_ENERGY_DENSITY, 1000, 50000, 40, 10, css.PREC_FP32, ctypes.byref(e)) == 0
    assert e.value >= d.value + 4 * 1000 * css.block_ld(40)
    assert lib.css_energy_density_matrix(None, None, None, 40, 0.0, 0.01, 10, 2.0, None, None, 0, 0, None, None,
                                         None, None, None, None, None, 0, None) == 1
    # shape-only CSR with placeholder pointers: the size checks come before any device work
    csr = css.CsrStruct(1000, 5000, 8, 8, 8, css.CSS_F64)
    assert lib.css_workspace_size(css.ENTRY_SPMM, 1000, 5000, 1, 1, 0, ctypes.byref(out)) == 0
    need = out.value
    assert need >= 2 * 4 * 5000 + 4 * 63
    assert lib.css_spmm_prepare(ctypes.byref(csr), ctypes.c_void_p(256), need - 1, None) == 3
    assert lib.css_spmm(ctypes.byref(csr), ctypes.c_void_p(256), ctypes.c_void_p(256), 8, 16,
                        ctypes.c_void_p(256), need - 1, None) == 3
    # mu search: null arguments, and an electron count outside (0, g n), are argument
    # errors before any device work
    mu = ctypes.c_double(0.0)
    assert lib.css_find_mu(None, None, None, 40, 8.0, 0.01, 10, 2.0, 0, None, None, None, None, 0, None) == 1
    assert lib.css_inv_sqrt_overlap(None, None, None, 40, 10, None, None, 0, 0, None, None, None, None, None, 0,
                                    None) == 1
    assert lib.css_transform_hamiltonian(None, None, None, None, 40, 10, None, None, 0, 0, None, None, None, None,
                                         None, None, 0, None) == 1
    assert lib.css_density_matrix_nonorth(None, None, None, None, None, None, 40, 0.0, 0.01, 10, 2.0, None, None, 0,
                                          0, None, None, None, None, None, None, 0, None) == 1
    p = ctypes.c_void_p(256)
    for ne, kT in ((0.0, 0.01), (-1.0, 0.01), (2000.0, 0.01), (float("nan"), 0.01), (100.0, 0.0)):
        assert lib.css_find_mu(ctypes.byref(csr), p, p, 40, ne, kT, 10, 2.0, 0, ctypes.byref(mu), None, None, p,
                               1 << 20, None) == 1


def test_oracle_not_imported_by_product_path():
    import sys
    for name in list(sys.modules):
        if name.startswith("paper_2605_20918_amd"):
            mod = sys.modules[name]
            src = getattr(mod, "__file__", "") or ""
            if src.endswith(".py"):
                with open(src) as f:
                    text = f.read()
                assert "import oracle" not in text and "from oracle" not in text, src


def test_struct_layout_matches_header(tmp_path):
    """ctypes mirrors of css_csr, css_info and css_system have the C header's field offsets."""
    import shutil
    import subprocess
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("no C compiler")
    structs = {"css_csr": css.CsrStruct, "css_info": css.InfoStruct, "css_system": css.SystemStruct,
               "css_color_job": css.ColorJobStruct, "css_tuning": css.TuningStruct}
    lines = ['#include <stddef.h>', '#include <stdio.h>', '#include "css.h"', "int main(void) {"]
    for cname, py in structs.items():
        lines.append(f'printf("{cname} size %zu\\n", sizeof({cname}));')
        for fname, _ in py._fields_:
            lines.append(f'printf("{cname} {fname} %zu\\n", offsetof({cname}, {fname}));')
    lines.append("return 0; }")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    inc = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include")
    exe = tmp_path / "layout"
    subprocess.run([gcc, "-I", inc, str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {tuple(l.split()[:2]): int(l.split()[2]) for l in out if l.strip()}
    for cname, py in structs.items():
        assert got[(cname, "size")] == ctypes.sizeof(py), cname
        for fname, _ in py._fields_:
            assert got[(cname, fname)] == getattr(py, fname).offset, (cname, fname)


def test_tuning_roundtrip_and_range_checks():
    """css_set_tuning / css_get_tuning are host-only: values round-trip, out-of-range
    fields are CSS_E_ARG and leave the current tuning unchanged, NULL resets."""
    lib = css.load()
    css.reset_tuning()
    assert css.get_tuning() == {"spmm_kernel": "auto", "spmm_run": 0, "spmm_depth": 0, "gram_chunks": 0,
                                "update_rows": 0, "cholqr2_series": 0}
    css.set_tuning(spmm_kernel="grouped", spmm_run=256, spmm_depth=8, gram_chunks=2, update_rows=64,
                   cholqr2_series=2)
    assert css.get_tuning() == {"spmm_kernel": "grouped", "spmm_run": 256, "spmm_depth": 8, "gram_chunks": 2,
                                "update_rows": 64, "cholqr2_series": 2}
    for bad in ({"spmm_kernel": 3}, {"spmm_run": -1}, {"spmm_depth": 5}, {"gram_chunks": 3}, {"update_rows": 96},
                {"cholqr2_series": 3}):
        t = css._tuning_struct(bad)
        assert lib.css_set_tuning(ctypes.byref(t)) == 1
    assert css.get_tuning()["spmm_run"] == 256
    css.reset_tuning()
    assert css.get_tuning()["spmm_kernel"] == "auto"
    assert lib.css_get_tuning(None) == 1
    assert lib.css_spmm_time(None, None, None, 1, 16, None, 0, None, 1, None, None) == 1


def test_autotune_cache_keys_and_roundtrip(tmp_path, monkeypatch):
    """The autotuner's JSON cache: one entry per (arch, N, nnz/row, b, precision)."""
    from paper_2605_20918_amd import autotune
    monkeypatch.setattr(autotune, "arch_name", lambda: "gfx950")
    p = str(tmp_path / "tune.json")
    assert autotune.load_cache(p) == {}
    k = autotune.key(60000, 6616104, 88, "fp32")
    assert k == "gfx950|N=60000|nnz/row=110.3|b=88|fp32"
    autotune.save_cache({k: {"choice": {"spmm_kernel": "grouped", "spmm_run": 512, "spmm_depth": 4}}}, p)
    assert autotune.load_cache(p)[k]["choice"]["spmm_run"] == 512
    assert autotune.apply_cached(60000, 6616104, 89, "fp32", p) is None
    css.reset_tuning()
    assert autotune.apply_cached(60000, 6616104, 88, "fp32", p) == {"spmm_kernel": "grouped", "spmm_run": 512,
                                                                      "spmm_depth": 4}
    assert css.get_tuning()["spmm_run"] == 512
    css.reset_tuning()


def test_noalloc_rejects_oversized_systems_before_device_work():
    """css_density_matrix_noalloc checks its fixed 256 MiB scratch against the system's
    buffers on the host: 10^6 and 1000 water molecules at depth 40 do not fit
    (CSS_E_WORKSPACE); CSS_SUBSPACE_EIG is CSS_E_UNSUPPORTED. Placeholder device
    pointers are never touched."""
    lib = css.load()
    e, t = ctypes.c_double(0.0), ctypes.c_double(0.0)
    tail = (ctypes.c_void_p(256), ctypes.byref(e), ctypes.byref(t), None, None)
    for n, nnz, b in ((1_000_000, 110_000_000, 88), (6000, 675_000, 86)):      # 10^6 and 1000 molecules
        csr = css.CsrStruct(n, nnz, 8, 8, 8, css.CSS_F64)
        args = (ctypes.byref(csr), ctypes.c_void_p(256), ctypes.c_void_p(256), b, -0.4, 0.01, 40, 2.0,
                ctypes.c_void_p(256), ctypes.c_void_p(256), 170 * n)
        assert lib.css_density_matrix_noalloc(*args, 0, *tail) == 3
        assert lib.css_density_matrix_noalloc(*args, css.PREC_FP32 | css.REORTH_FULL, *tail) == 3
        assert lib.css_density_matrix_noalloc(*args, css.SUBSPACE_EIG, *tail) == 8
