"""CPU checks of the C-ABI library: it loads, exports every symbol include/msp.h
declares, and rejects bad arguments before touching the device."""
import ctypes
import os
import re

import pytest

import paper_2405_05865_amd as msp
from paper_2405_05865_amd import _binding as B

HDR = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include", "msp.h")


def _declared():
    txt = open(HDR).read()
    return sorted(set(re.findall(r"^\s*(?:msp_status|void|const char\*)\s+(msp_\w+)\s*\(", txt, re.M)))


def test_library_loads_and_exports_every_declared_symbol():
    L = msp.library()
    names = _declared()
    assert len(names) >= 14
    for name in names:
        assert hasattr(L, name), name
    assert set(names) == set(B.EXPORTS)


def test_version_and_defaults():
    L = msp.library()
    assert L.msp_version().decode().startswith("libmsp")
    o = B.SolveOpts()
    L.msp_solve_opts_default(ctypes.byref(o))
    assert o.tol == 1e-8 and o.max_outer > 0 and o.inner_tol > 0
    assert o.level2_form == 1 and o.sym_sweep == 1
    assert o.autotune == 0


def test_batched_adjoint_rejects_empty_batch():
    L = msp.library()
    arr = (B.SystemGrad * 1)()
    need = B.size_out()
    assert B.STATUS[L.msp_solve_batched_backward_workspace(0, arr, 1, None, ctypes.byref(need))] == "MSP_ERR_INVALID_ARG"
    dl = (ctypes.c_double * 1)()
    code = L.msp_solve_batched_backward(None, 1, arr, 0, 0, 1, None, None, 0, dl, None)
    assert B.STATUS[code] == "MSP_ERR_INVALID_ARG"  # null handle, rejected before any device work


@pytest.mark.parametrize("m,n,s,gamma", [(0, 10, 4, 2), (10, 10, 0, 1), (10, 10, 4, 5), (10, 10, 11, 2),
                                         (10, 100, 64, 33)])
def test_sketch_workspace_rejects_bad_sizes(m, n, s, gamma):
    L = msp.library()
    out = ctypes.c_size_t(0)
    assert L.msp_sketch_workspace(m, n, s, gamma, ctypes.byref(out)) == 1
    assert L.msp_last_error()


def test_sketch_validation_happens_before_device_work():
    L = msp.library()
    # null pointers and an F64 Y from F32 A are rejected without any HIP call
    assert L.msp_sketch(None, None, 0, 10, 10, 10, 4, 2, 1, None, None, None, 0, 4, None, 0) == 1
    dummy = ctypes.c_void_p(256)
    assert L.msp_sketch(None, dummy, B.MSP_F32, 10, 10, 10, 4, 2, 1, dummy, dummy, dummy, B.MSP_F64, 4, dummy,
                        1 << 20) == 1
    assert b"F64 Y" in L.msp_last_error()


def test_nystrom_validation():
    L = msp.library()
    out = ctypes.c_size_t(0)
    assert L.msp_nystrom_workspace(0, 100, 100, 16, 64, 8, ctypes.byref(out)) == 0 and out.value > 0
    assert L.msp_nystrom_workspace(5, 100, 100, 16, 64, 8, ctypes.byref(out)) == 1
    h = ctypes.c_void_p()
    dummy = ctypes.c_void_p(256)
    # lam + lam0 must be > 0
    assert L.msp_nystrom(None, 0, 100, 100, 16, 8, dummy, dummy, dummy, 0, 16, None, 0, 0, 0.0, 0.0, 64, 8, 3,
                         dummy, 1 << 30, ctypes.byref(h)) == 1
    # NaN lambda
    assert L.msp_nystrom(None, 0, 100, 100, 16, 8, dummy, dummy, dummy, 0, 16, None, 0, 0, float("nan"), 0.0, 64, 8,
                         3, dummy, 1 << 30, ctypes.byref(h)) == 5
    # PSD needs a square system
    assert L.msp_nystrom(None, 0, 90, 100, 16, 8, dummy, dummy, dummy, 0, 16, None, 0, 0, 1.0, 0.0, 64, 8, 3, dummy,
                         1 << 30, ctypes.byref(h)) == 1
    # the lam0 estimator (lambda0 < 0) needs A, and only PSD handles have it
    assert L.msp_nystrom(None, 0, 100, 100, 16, 8, dummy, dummy, dummy, 0, 16, None, 0, 0, 1.0, -1.0, 64, 8, 3,
                         dummy, 1 << 30, ctypes.byref(h)) == 1
    assert b"needs A" in L.msp_last_error()
    assert L.msp_nystrom(None, 1, 100, 100, 16, 8, dummy, dummy, dummy, 0, 16, dummy, 0, 100, 1.0, -1.0, 64, 8, 3,
                         dummy, 1 << 30, ctypes.byref(h)) == 7


def test_solve_rejects_null_handle():
    L = msp.library()
    info = B.SolveInfo()
    assert L.msp_solve(None, None, None, 0, None, 0, 10, 0.0, None, 10, 1, None, 10, None, None, 0,
                       ctypes.byref(info)) == 1


def test_least_squares_validation_before_device_work():
    L = msp.library()
    need = ctypes.c_size_t(0)
    assert L.msp_left_sketch_workspace(100, 0, 8, ctypes.byref(need)) == 1
    assert L.msp_left_sketch_workspace(100, 40, 33, ctypes.byref(need)) == 1
    assert L.msp_left_sketch_workspace(100, 40, 8, ctypes.byref(need)) == 0 and need.value > 0
    assert L.msp_lstsq_workspace(None, 100, 1, None, ctypes.byref(need)) == 1
    o = B.SolveOpts()
    L.msp_solve_opts_default(ctypes.byref(o))
    info = B.SolveInfo()
    assert L.msp_lstsq(None, None, None, 0, None, 0, 10, 10, None, 10, 1, None, 10, ctypes.byref(o), None, 0,
                       ctypes.byref(info)) == 1


@pytest.mark.parametrize("cc,std", [("gcc", "-std=c99"), ("g++", "-std=c++17")])
def test_header_compiles_as_c_and_cpp(tmp_path, cc, std):
    # the boundary is plain C: no HIP or torch types, usable from C and C++ callers
    import shutil
    import subprocess
    if shutil.which(cc) is None:
        pytest.skip(f"{cc} not available")
    src = tmp_path / ("t.c" if cc == "gcc" else "t.cpp")
    src.write_text('#include "msp.h"\nint main(void) { msp_solve_opts o; msp_solve_opts_default(&o); '
                   'return (int)sizeof(msp_solve_info) > 0 ? 0 : 1; }\n')
    inc = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include")
    r = subprocess.run([cc, std, "-Wall", "-Wextra", "-Werror", "-fsyntax-only", "-I", inc, str(src)],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr


def test_bench_refuses_several_gpus():
    # one GPU per process and box: --gpus above 1 exits with a message before any device work
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr


def test_noalloc_scratch_size_and_oversized_request():
    # the binding's copy of MSP_NOALLOC_SCRATCH_BYTES matches the header, and a sketch whose
    # scratch exceeds it is rejected on the host before any device work
    m = re.search(r"#define MSP_NOALLOC_SCRATCH_BYTES \((\d+)u << (\d+)\)", open(HDR).read())
    assert m and int(m.group(1)) << int(m.group(2)) == B.NOALLOC_SCRATCH_BYTES
    L = msp.library()
    n = 1 << 22
    code = L.msp_sketch_noalloc(None, None, B.MSP_F32, n, n, n, 2048, 8, 1, None, None, None, B.MSP_F32, 2048)
    assert B.STATUS[code] == "MSP_ERR_WORKSPACE"
    assert b"static scratch" in L.msp_last_error()
