"""ctypes marshalling for libmsp (include/msp.h). No arithmetic happens here: every
step of the method runs in the library's HIP kernels; torch only supplies device
memory and the current HIP stream."""
from __future__ import annotations

import ctypes
import os

import torch  # noqa: F401  (loads the HIP runtime libmsp links against)

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmsp.so")

MSP_F64, MSP_F32, MSP_BF16 = 0, 1, 2
MSP_SYM_PSD, MSP_GENERAL = 0, 1
MSP_TRACE_SCHATTEN_P, MSP_TRACE_EFFDIM = 0, 1
NOALLOC_SCRATCH_BYTES = 16 << 20  # MSP_NOALLOC_SCRATCH_BYTES of include/msp.h

STATUS = {
    0: "MSP_OK",
    1: "MSP_ERR_INVALID_ARG",
    2: "MSP_ERR_NOT_POSDEF",
    3: "MSP_ERR_BREAKDOWN",
    4: "MSP_ERR_NO_CONVERGENCE",
    5: "MSP_ERR_NONFINITE",
    6: "MSP_ERR_WORKSPACE",
    7: "MSP_ERR_UNSUPPORTED",
    8: "MSP_ERR_HIP",
}

EXPORTS = (
    "msp_sketch_workspace", "msp_sketch", "msp_sketch_autotune", "msp_nystrom_workspace", "msp_nystrom", "msp_precond_destroy",
    "msp_precond_params",
    "msp_precond_set_lambda", "msp_precond_factors", "msp_solve_opts_default", "msp_solve_workspace", "msp_solve",
    "msp_solve_batched_workspace", "msp_solve_batched", "msp_solve_batched_backward_workspace",
    "msp_solve_batched_backward", "msp_solve_backward",
    "msp_schatten_workspace", "msp_schatten", "msp_orlicz", "msp_kyfan_workspace", "msp_kyfan",
    "msp_gaussian_probes", "msp_left_sketch_workspace", "msp_left_sketch",
    "msp_lstsq_workspace", "msp_lstsq", "msp_sketch_noalloc", "msp_last_error", "msp_version",
)


STATUS_CODE = {v: k for k, v in STATUS.items()}


class MspError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{STATUS.get(code, code)}: {msg}")
        self.code = code
        self.status = STATUS.get(code, str(code))


class SolveOpts(ctypes.Structure):
    _fields_ = [
        ("tol", ctypes.c_double),
        ("max_outer", ctypes.c_int32),
        ("inner_tol", ctypes.c_double),
        ("max_inner", ctypes.c_int32),
        ("level3_tol", ctypes.c_double),
        ("max_level3", ctypes.c_int32),
        ("normal", ctypes.c_int32),
        ("refine", ctypes.c_int32),
        ("refine_inner_tol", ctypes.c_double),
        ("max_refine", ctypes.c_int32),
        ("profile", ctypes.c_int32),
        ("level2_form", ctypes.c_int32),
        ("sym_sweep", ctypes.c_int32),
        ("use_graph", ctypes.c_int32),
        ("batch_teams", ctypes.c_int32),
        ("autotune", ctypes.c_int32),
        ("level3_kernels", ctypes.c_int32),
    ]


class System(ctypes.Structure):
    """msp_system: one system of a batched solve."""
    _fields_ = [
        ("P", ctypes.c_void_p),
        ("A_hi", ctypes.c_void_p),
        ("A_lo", ctypes.c_void_p),
        ("lda", ctypes.c_int64),
        ("B", ctypes.c_void_p),
        ("ldb", ctypes.c_int64),
        ("X", ctypes.c_void_p),
        ("ldx", ctypes.c_int64),
    ]


class SystemGrad(ctypes.Structure):
    """msp_system_grad: one system of a batched adjoint."""
    _fields_ = [
        ("P", ctypes.c_void_p),
        ("A_hi", ctypes.c_void_p),
        ("A_lo", ctypes.c_void_p),
        ("lda", ctypes.c_int64),
        ("X", ctypes.c_void_p),
        ("ldx", ctypes.c_int64),
        ("G", ctypes.c_void_p),
        ("ldg", ctypes.c_int64),
        ("dB", ctypes.c_void_p),
        ("lddb", ctypes.c_int64),
        ("dA", ctypes.c_void_p),
        ("ldda", ctypes.c_int64),
    ]


class SolveInfo(ctypes.Structure):
    _fields_ = [
        ("status", ctypes.c_int),
        ("outer_iters", ctypes.c_int32),
        ("inner_iters", ctypes.c_int64),
        ("level3_iters", ctypes.c_int64),
        ("refine_steps", ctypes.c_int32),
        ("krylov_refine", ctypes.c_int32),
        ("restarts", ctypes.c_int32),
        ("rel_residual_max", ctypes.c_double),
        ("sweep_bytes", ctypes.c_double),
        ("sweeps", ctypes.c_int64),
        ("sweep_ms", ctypes.c_double),
        ("timed_sweeps", ctypes.c_int64),
        ("sweep_segments", ctypes.c_int32),
        ("seconds", ctypes.c_double),
        ("trace_nodes", ctypes.c_int32),
    ]

    def as_dict(self):
        d = {f: getattr(self, f) for f, _ in self._fields_}
        d["status"] = STATUS.get(self.status, self.status)
        return d


_lib = None

P = ctypes.c_void_p
I64 = ctypes.c_int64
I32 = ctypes.c_int32
U64 = ctypes.c_uint64
D = ctypes.c_double
SZ = ctypes.POINTER(ctypes.c_size_t)


def lib_path() -> str:
    return LIB_PATH


def load(path: str | None = None):
    """Load libmsp.so and declare its signatures; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    path = path or LIB_PATH
    if not os.path.exists(path):
        raise RuntimeError(f"libmsp.so not found at {path}; build it with paper_2405_05865_amd.build.build()")
    L = ctypes.CDLL(path)
    L.msp_sketch_workspace.argtypes = [I64, I64, I64, I32, SZ]
    L.msp_sketch.argtypes = [P, P, ctypes.c_int, I64, I64, I64, I64, I32, U64, P, P, P, ctypes.c_int, I64, P,
                             ctypes.c_size_t]
    L.msp_sketch_autotune.argtypes = [P, P, ctypes.c_int, I64, I64, I64, I64, I32, U64, P, P, P, ctypes.c_int, I64, P,
                                      ctypes.c_size_t, ctypes.POINTER(I32)]
    L.msp_sketch_noalloc.argtypes = [P, P, ctypes.c_int, I64, I64, I64, I64, I32, U64, P, P, P, ctypes.c_int, I64]
    L.msp_nystrom_workspace.argtypes = [ctypes.c_int, I64, I64, I64, I64, I32, SZ]
    L.msp_nystrom.argtypes = [P, ctypes.c_int, I64, I64, I64, I32, P, P, P, ctypes.c_int, I64, P, ctypes.c_int, I64,
                              D, D, I64, I32, U64, P, ctypes.c_size_t, ctypes.POINTER(P)]
    L.msp_precond_params.argtypes = [P, ctypes.POINTER(D), ctypes.POINTER(D)]
    L.msp_precond_destroy.argtypes = [P]
    L.msp_precond_set_lambda.argtypes = [P, P, D]
    L.msp_precond_factors.argtypes = [P, P, P, P, P]
    L.msp_solve_opts_default.argtypes = [ctypes.POINTER(SolveOpts)]
    L.msp_solve_opts_default.restype = None
    L.msp_solve_workspace.argtypes = [P, I64, ctypes.POINTER(SolveOpts), SZ]
    L.msp_solve.argtypes = [P, P, P, ctypes.c_int, P, ctypes.c_int, I64, D, P, I64, I64, P, I64,
                            ctypes.POINTER(SolveOpts), P, ctypes.c_size_t, ctypes.POINTER(SolveInfo)]
    L.msp_solve_batched_workspace.argtypes = [I32, ctypes.POINTER(System), I64, ctypes.POINTER(SolveOpts), SZ]
    L.msp_solve_batched.argtypes = [P, I32, ctypes.POINTER(System), ctypes.c_int, ctypes.c_int, I64,
                                    ctypes.POINTER(SolveOpts), P, ctypes.c_size_t, ctypes.POINTER(SolveInfo)]
    L.msp_solve_batched_backward_workspace.argtypes = [I32, ctypes.POINTER(SystemGrad), I64,
                                                       ctypes.POINTER(SolveOpts), SZ]
    L.msp_solve_batched_backward.argtypes = [P, I32, ctypes.POINTER(SystemGrad), ctypes.c_int, ctypes.c_int, I64,
                                             ctypes.POINTER(SolveOpts), P, ctypes.c_size_t, ctypes.POINTER(D),
                                             ctypes.POINTER(SolveInfo)]
    L.msp_solve_backward.argtypes = [P, P, P, ctypes.c_int, P, ctypes.c_int, I64, D, P, I64, P, I64, I64, P, I64,
                                     ctypes.POINTER(D), P, I64, ctypes.POINTER(SolveOpts), P, ctypes.c_size_t,
                                     ctypes.POINTER(SolveInfo)]
    L.msp_schatten_workspace.argtypes = [P, I64, ctypes.POINTER(SolveOpts), SZ]
    L.msp_schatten.argtypes = [P, ctypes.c_int, P, P, ctypes.c_int, P, ctypes.c_int, I64, D, P, I64, I64, U64, D, D,
                               D, ctypes.POINTER(SolveOpts), P, ctypes.c_size_t, ctypes.POINTER(D), ctypes.POINTER(D),
                               ctypes.POINTER(SolveInfo)]
    L.msp_orlicz.argtypes = [P, P, P, ctypes.c_int, P, ctypes.c_int, I64, P, P, I64, P, I64, I64, U64, D, D, D,
                             ctypes.POINTER(SolveOpts), P, ctypes.c_size_t, ctypes.POINTER(D), ctypes.POINTER(D), P,
                             ctypes.POINTER(SolveInfo)]
    L.msp_kyfan_workspace.argtypes = [I64, I64, I64, SZ]
    L.msp_kyfan.argtypes = [P, P, ctypes.c_int, I64, I64, I64, I64, I64, I32, U64, P, ctypes.c_size_t,
                            ctypes.POINTER(D), P]
    L.msp_gaussian_probes.argtypes = [P, I64, I64, U64, P, I64]
    L.msp_left_sketch_workspace.argtypes = [I64, I64, I32, SZ]
    L.msp_left_sketch.argtypes = [P, P, ctypes.c_int, I64, I64, I64, I64, I32, U64, P, P, P, I64, P, ctypes.c_size_t]
    L.msp_lstsq_workspace.argtypes = [P, I64, I64, ctypes.POINTER(SolveOpts), SZ]
    L.msp_lstsq.argtypes = [P, P, P, I64, P, ctypes.c_int, I64, I64, P, I64, I64, P, I64, ctypes.POINTER(SolveOpts),
                            P, ctypes.c_size_t, ctypes.POINTER(SolveInfo)]
    L.msp_last_error.restype = ctypes.c_char_p
    L.msp_last_error.argtypes = []
    L.msp_version.restype = ctypes.c_char_p
    L.msp_version.argtypes = []
    for name in EXPORTS:
        if name not in ("msp_solve_opts_default", "msp_last_error", "msp_version"):
            getattr(L, name).restype = ctypes.c_int
    _lib = L
    return L


def check(code: int):
    if code != 0:
        raise MspError(code, _lib.msp_last_error().decode())


def size_out():
    return ctypes.c_size_t(0)
