"""C-ABI checks that need no GPU: the library loads, exports every entry
point that include/rbp.h declares, and rejects bad arguments before any
device work."""
import ctypes
import os
import re

import pytest

from paper_2411_13507_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    text = open(os.path.join(ROOT, "include", "rbp.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(rbp_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(_lib.LIB_PATH):
        pytest.skip("librbp.so not built")
    return _lib.load()


def test_header_symbols_exported(lib):
    names = declared_symbols()
    assert set(names) == set(_lib.EXPORTED), names
    for n in names:
        assert hasattr(lib, n), n


def test_default_opts(lib):
    o = _lib.default_opts()
    assert o.admm_iters == 10 and abs(o.rho - 0.1) < 1e-7 and abs(o.alpha - 1.6) < 1e-6
    assert o.max_polish_steps == 0 and o.store_for_backward == 1 and o.plain == 0
    assert o.feas_tol == 1e-11 and o.kkt_tol == 1e-6
    assert o.launch_shape == 0 and o.schedule == 0


def test_status_strings(lib):
    for code in (0, 1, 2, 3, 4, 5, -1, -2, -3, -4, -5, -6):
        s = lib.rbp_status_string(code).decode()
        assert s and s != "unknown code"
    assert lib.rbp_status_string(1234).decode() == "unknown code"


def test_null_arguments_rejected(lib):
    out = ctypes.c_void_p()
    assert lib.rbp_build_batch(None, None, ctypes.byref(out)) == _lib.RBP_E_INVALID
    d = _lib.ProblemDesc()
    d.n_instances = 1
    d.vmax = 3.0
    d.amax = 5.0
    d.n_poly = 1
    # null device pointers with N > 0
    assert lib.rbp_build_batch(ctypes.byref(d), None, ctypes.byref(out)) == _lib.RBP_E_INVALID
    d.vmax = 0.0
    assert lib.rbp_build_batch(ctypes.byref(d), None, ctypes.byref(out)) == _lib.RBP_E_INVALID
    d.vmax, d.n_instances = 3.0, -1
    assert lib.rbp_build_batch(ctypes.byref(d), None, ctypes.byref(out)) == _lib.RBP_E_INVALID
    o = _lib.default_opts()
    z = [None] * 7
    assert lib.rbp_solve_batch(None, None, None, None, ctypes.byref(o), *z) == _lib.RBP_E_INVALID
    assert lib.rbp_backward(None, *([None] * 7)) == _lib.RBP_E_INVALID
    sz = _lib.BatchSizes()
    assert lib.rbp_batch_get_sizes(None, ctypes.byref(sz)) == _lib.RBP_E_INVALID
    lib.rbp_destroy_batch(None)


def test_graph_noalloc_rejects_before_device_work(lib):
    """The allocation-free graph run checks its arguments and the size of
    its fixed workspace before any HIP call (so this runs without a GPU)."""
    import numpy as np
    host = np.zeros(16)
    hp = host.ctypes.data
    d = _lib.GraphDesc(1 << 20, 3, 64, 0, hp, hp, hp)
    assert lib.rbp_graph_run_noalloc(ctypes.byref(d), hp, hp, hp, None) == _lib.RBP_E_SCRATCH
    # the largest node count that fits with 64 rows: 2 n m + 2 ceil(n/64) m <= 2^20
    n_fit = max(n for n in range(8000, 8200) if 2 * n * 64 + 2 * ((n + 63) // 64) * 64 <= _lib.GRAPH_NOALLOC_DOUBLES)
    d.n_nodes = n_fit + 1
    assert lib.rbp_graph_run_noalloc(ctypes.byref(d), hp, hp, hp, None) == _lib.RBP_E_SCRATCH
    d.n_nodes = n_fit
    # fits; null node and output pointers are rejected next, still on the host
    assert lib.rbp_graph_run_noalloc(ctypes.byref(d), None, None, None, None) == _lib.RBP_E_INVALID
    d.reserved = 1
    assert lib.rbp_graph_run_noalloc(ctypes.byref(d), hp, hp, hp, None) == _lib.RBP_E_INVALID
    d.reserved, d.n_rows = 0, 0
    assert lib.rbp_graph_run_noalloc(ctypes.byref(d), hp, hp, hp, None) == _lib.RBP_E_SHAPE
    assert lib.rbp_graph_run_noalloc(None, hp, hp, hp, None) == _lib.RBP_E_INVALID


def test_no_cpu_fallback():
    import torch
    if torch.cuda.is_available():
        pytest.skip("GPU present")
    from paper_2411_13507_amd.api import SegmentBatchGPU
    from workloads import gen
    with pytest.raises(_lib.RbpError):
        SegmentBatchGPU(gen.gen_cfg0(2))


def test_missing_library_is_an_error(tmp_path):
    saved = _lib._LIB
    try:
        _lib._LIB = None
        with pytest.raises(_lib.RbpError):
            _lib.load(str(tmp_path / "missing.so"))
    finally:
        _lib._LIB = saved


def test_descriptor_layouts_match_header(tmp_path):
    """The ctypes descriptors have the field offsets and sizes the C compiler
    gives the structs of include/rbp.h."""
    import shutil
    import subprocess
    if not shutil.which("gcc") or not os.path.exists("/opt/rocm/include/hip/hip_runtime_api.h"):
        pytest.skip("no host C compiler or HIP headers")
    structs = {"rbp_problem_desc": _lib.ProblemDesc, "rbp_chain_desc": _lib.ChainDesc,
               "rbp_cut_desc": _lib.CutDesc, "rbp_graph_desc": _lib.GraphDesc, "rbp_mpc_desc": _lib.MpcDesc,
               "rbp_solve_opts": _lib.SolveOpts, "rbp_batch_sizes": _lib.BatchSizes}
    lines = ['#include <stddef.h>', '#include <stdio.h>', '#include "rbp.h"', "int main(void) {"]
    for cname, cls in structs.items():
        lines.append(f'  printf("{cname} size %zu\\n", sizeof({cname}));')
        for f in cls._fields_:
            lines.append(f'  printf("{cname} {f[0]} %zu\\n", offsetof({cname}, {f[0]}));')
    lines.append("  return 0;\n}")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-D__HIP_PLATFORM_AMD__", "-I", os.path.join(ROOT, "include"), "-I", "/opt/rocm/include",
                    str(src), "-o", str(exe)], check=True, capture_output=True)
    got = {}
    for ln in subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.splitlines():
        c, f, v = ln.split()
        got[(c, f)] = int(v)
    for cname, cls in structs.items():
        assert got[(cname, "size")] == ctypes.sizeof(cls), cname
        for f in cls._fields_:
            assert got[(cname, f[0])] == getattr(cls, f[0]).offset, (cname, f[0])
