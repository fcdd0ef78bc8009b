"""MI355X (gfx950) implementation of the hot path of Multi-level Sketched
Preconditioning (Derezinski, Musco, Yang): the sparse sketch Y = A S^T, the Nystrom
preconditioner with its inner levels, and the multi-level preconditioned iteration.

This module is argument marshalling over the C-ABI library libmsp.so
(include/msp.h); every step of the method runs in hand-written HIP kernels. Torch
supplies device memory and the current stream. If the library is missing, every call
raises: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import math
from dataclasses import dataclass
from types import SimpleNamespace

import torch

from . import _binding as B
from ._binding import MspError, SolveInfo, SolveOpts  # noqa: F401

__all__ = ["sketch", "sketch_noalloc", "Precond", "nystrom", "solve", "solve_batched", "solve_batched_backward", "solve_backward", "schatten", "orlicz", "kyfan", "effective_dimension", "gaussian_probes",
           "MSPSolve", "msp_solve", "library", "MspError", "SolveOpts"]

_DT = {torch.float64: B.MSP_F64, torch.float32: B.MSP_F32, torch.bfloat16: B.MSP_BF16}


def library():
    """The loaded ctypes library (raises if libmsp.so has not been built)."""
    return B.load()


def _code(t: torch.Tensor) -> int:
    if t.dtype not in _DT:
        raise TypeError(f"unsupported dtype {t.dtype}")
    return _DT[t.dtype]


def _stream(dev: torch.device) -> int:
    return torch.cuda.current_stream(dev).cuda_stream


def _rowmajor(A: torch.Tensor, name: str):
    if A.dim() != 2 or A.stride(1) != 1:
        raise ValueError(f"{name} must be a 2-D row-major tensor (unit column stride)")
    if not A.is_cuda:
        raise ValueError(f"{name} must be a CUDA (HIP) tensor")


def _check_layout(P, A: torch.Tensor, name: str, rows: int | None = None):
    """A is the handle's matrix: (n, n) for a "psd" handle, (m, n) for a "general" one (or
    `rows` x n), a supported dtype, row-major with ld >= n. The C-ABI cannot see A's extent,
    so this is checked before any launch."""
    if not isinstance(A, torch.Tensor) or A.dim() != 2:
        raise ValueError(f"{name} must be a 2-D tensor")
    if rows is None:
        rows = P.m if P.structure == "general" else P.n
    if tuple(A.shape) != (rows, P.n):
        raise ValueError(f"{name} must have shape ({rows}, {P.n}) for this handle, got {tuple(A.shape)}")
    if A.dtype not in _DT:
        raise TypeError(f"{name}: unsupported dtype {A.dtype}")
    if A.stride(1) != 1 or A.stride(0) < P.n:
        raise ValueError(f"{name} must be row-major with leading dimension >= {P.n}")


def _check_device(A: torch.Tensor, name: str, dev=None):
    if not A.is_cuda:
        raise ValueError(f"{name} must be a CUDA (HIP) tensor")
    if dev is not None and A.device != dev:
        raise ValueError(f"{name} is on {A.device}, the vectors on {dev}")


def _pair(P, A_hi, A_lo, dev, rows=None):
    """Checks A_hi and A_lo (A_lo None: A_hi) against the handle and returns A_lo."""
    A_lo = A_hi if A_lo is None else A_lo
    _check_layout(P, A_hi, "A_hi", rows)
    _check_layout(P, A_lo, "A_lo", rows)
    if A_hi.dtype == torch.bfloat16:
        raise TypeError("A_hi must be float64 or float32")
    if A_hi.stride(0) != A_lo.stride(0):
        raise ValueError("A_hi and A_lo must share the leading dimension")
    _check_device(A_hi, "A_hi", dev)
    _check_device(A_lo, "A_lo", dev)
    return A_lo


def _workspace(nbytes: int, dev) -> torch.Tensor:
    ws = torch.empty(int(nbytes) + 256, dtype=torch.uint8, device=dev)
    off = (-ws.data_ptr()) % 256
    return ws[off:off + int(nbytes)] if nbytes else ws[off:off + 1]


def _vectors(X: torch.Tensor, length: int, name: str):
    """(length,) or (k, length) float64 CUDA tensor with unit inner stride -> (k, ld)."""
    if X.dtype != torch.float64 or not X.is_cuda:
        raise ValueError(f"{name} must be a float64 CUDA tensor")
    if X.dim() == 1:
        if X.shape[0] != length or X.stride(0) != 1:
            raise ValueError(f"{name} must have length {length} and unit stride")
        return 1, length
    if X.dim() != 2 or X.shape[1] != length or X.stride(1) != 1:
        raise ValueError(f"{name} must be (k, {length}) with unit inner stride")
    return X.shape[0], X.stride(0)


def _opts(**kw) -> SolveOpts:
    L = library()
    o = SolveOpts()
    L.msp_solve_opts_default(ctypes.byref(o))
    for k, v in kw.items():
        if v is None:
            continue
        if not hasattr(o, k):
            raise TypeError(f"unknown option {k}")
        setattr(o, k, int(v) if isinstance(getattr(o, k), int) else float(v))
    return o


# -----------------------------------------------------------------------------------
# msp_sketch
# -----------------------------------------------------------------------------------
def sketch(A: torch.Tensor, s: int, gamma: int, seed: int, y_dtype: torch.dtype | None = None,
           autotune: bool = False):
    """S (Definition 2.1) and Y = A S^T. Returns (S_rows int32 [n, gamma],
    S_signs int8 [n, gamma], Y [m, s]). autotune=True calls msp_sketch_autotune: the rows of
    A per block of the sketch kernel are timed on this matrix and the fastest is kept for
    this shape (returned as a fourth value)."""
    L = library()
    _rowmajor(A, "A")
    m, n = A.shape
    if y_dtype is None:
        y_dtype = torch.float64 if A.dtype == torch.float64 else torch.float32
    rows = torch.empty((n, gamma), dtype=torch.int32, device=A.device)
    signs = torch.empty((n, gamma), dtype=torch.int8, device=A.device)
    Y = torch.empty((m, s), dtype=y_dtype, device=A.device)
    need = B.size_out()
    B.check(L.msp_sketch_workspace(m, n, s, gamma, ctypes.byref(need)))
    ws = _workspace(need.value, A.device)
    if autotune:
        chosen = ctypes.c_int32(0)
        B.check(L.msp_sketch_autotune(_stream(A.device), A.data_ptr(), _code(A), m, n, A.stride(0), s, gamma,
                                      ctypes.c_uint64(seed & (2 ** 64 - 1)), rows.data_ptr(), signs.data_ptr(),
                                      Y.data_ptr(), _code(Y), Y.stride(0), ws.data_ptr(), ws.numel(),
                                      ctypes.byref(chosen)))
        return rows, signs, Y, chosen.value
    B.check(L.msp_sketch(_stream(A.device), A.data_ptr(), _code(A), m, n, A.stride(0), s, gamma,
                         ctypes.c_uint64(seed & (2 ** 64 - 1)), rows.data_ptr(), signs.data_ptr(), Y.data_ptr(),
                         _code(Y), Y.stride(0), ws.data_ptr(), ws.numel()))
    return rows, signs, Y


def sketch_noalloc(A: torch.Tensor, s: int, gamma: int, seed: int, out=None, y_dtype: torch.dtype | None = None):
    """msp_sketch_noalloc: the same S and Y = A S^T as sketch(), with the library's static
    device scratch instead of a workspace. ``out`` = (S_rows, S_signs, Y) preallocated by
    the caller (then nothing is allocated here either); returns that triple."""
    L = library()
    _rowmajor(A, "A")
    m, n = A.shape
    if out is None:
        if y_dtype is None:
            y_dtype = torch.float64 if A.dtype == torch.float64 else torch.float32
        out = (torch.empty((n, gamma), dtype=torch.int32, device=A.device),
               torch.empty((n, gamma), dtype=torch.int8, device=A.device),
               torch.empty((m, s), dtype=y_dtype, device=A.device))
    rows, signs, Y = out
    if rows.dtype != torch.int32 or signs.dtype != torch.int8 or tuple(rows.shape) != (n, gamma) \
            or tuple(signs.shape) != (n, gamma) or not rows.is_contiguous() or not signs.is_contiguous():
        raise ValueError("S_rows / S_signs must be contiguous int32 / int8 tensors of shape (n, gamma)")
    _rowmajor(Y, "Y")
    if Y.shape[0] != m or Y.shape[1] != s:
        raise ValueError(f"Y must be ({m}, {s})")
    for t in (rows, signs, Y):
        if t.device != A.device:
            raise ValueError("outputs must live on A's device")
    B.check(L.msp_sketch_noalloc(_stream(A.device), A.data_ptr(), _code(A), m, n, A.stride(0), s, gamma,
                                 ctypes.c_uint64(seed & (2 ** 64 - 1)), rows.data_ptr(), signs.data_ptr(),
                                 Y.data_ptr(), _code(Y), Y.stride(0)))
    return rows, signs, Y


# -----------------------------------------------------------------------------------
# msp_nystrom
# -----------------------------------------------------------------------------------
class Precond:
    """Handle of the Nystrom preconditioner and its inner levels (msp_nystrom)."""

    def __init__(self, structure: str, S_rows, S_signs, Y, lam: float, lam0: float | None, phi: int,
                 phi_gamma: int, phi_seed: int, A: torch.Tensor | None = None):
        """lam0 None (or < 0): estimated on the GPU from the sketch and A's diagonal
        (needs A, the matrix Y was sketched from; PSD handles only); self.lam0 holds the
        value used."""
        L = library()
        self.structure = structure
        code = B.MSP_SYM_PSD if structure == "psd" else B.MSP_GENERAL
        _rowmajor(Y, "Y")
        m, s = Y.shape
        n, gamma = S_rows.shape
        self.m, self.n, self.s, self.gamma = m, n, s, gamma
        self.phi, self.phi_gamma = phi, phi_gamma
        lam0 = -1.0 if lam0 is None else float(lam0)
        if lam0 < 0:
            if A is None:
                raise ValueError("estimating lam0 needs A")
            _check_layout(SimpleNamespace(structure="psd", m=n, n=n), A, "A")
            _check_device(A, "A", Y.device)
        self.lam = float(lam)
        need = B.size_out()
        B.check(L.msp_nystrom_workspace(code, m, n, s, phi, phi_gamma, ctypes.byref(need)))
        self._ws = _workspace(need.value, Y.device)
        self._keep = (S_rows, S_signs, Y)
        self.device = Y.device
        h = ctypes.c_void_p()
        B.check(L.msp_nystrom(_stream(Y.device), code, m, n, s, gamma, S_rows.data_ptr(), S_signs.data_ptr(),
                              Y.data_ptr(), _code(Y), Y.stride(0), A.data_ptr() if A is not None else None,
                              _code(A) if A is not None else 0, A.stride(0) if A is not None else 0, float(lam),
                              lam0, phi, phi_gamma, ctypes.c_uint64(phi_seed & (2 ** 64 - 1)), self._ws.data_ptr(),
                              self._ws.numel(), ctypes.byref(h)))
        self.handle = h
        lv, l0 = ctypes.c_double(), ctypes.c_double()
        B.check(L.msp_precond_params(h, ctypes.byref(lv), ctypes.byref(l0)))
        self.lam0 = l0.value

    @property
    def Y(self):
        return self._keep[2]

    def factors(self):
        """(W or None, M2^{-1} or M3a^{-1}, M3b^{-1} or None) as s x s float64 tensors."""
        s = self.s
        mk = lambda: torch.empty((s, s), dtype=torch.float64, device=self.device)
        W = mk() if self.structure == "psd" else None
        Mi = mk()
        M2 = mk() if self.structure != "psd" else None
        ptr = lambda t: t.data_ptr() if t is not None else None
        B.check(library().msp_precond_factors(_stream(self.device), self.handle, ptr(W), ptr(Mi), ptr(M2)))
        torch.cuda.current_stream(self.device).synchronize()
        return W, Mi, M2

    def set_lambda(self, lam: float):
        B.check(library().msp_precond_set_lambda(_stream(self.device), self.handle, float(lam)))
        self.lam = float(lam)

    def close(self):
        if getattr(self, "handle", None) is not None and self.handle.value:
            library().msp_precond_destroy(self.handle)
            self.handle = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def nystrom(structure, S_rows, S_signs, Y, lam, lam0, phi, phi_gamma, phi_seed, A=None) -> Precond:
    return Precond(structure, S_rows, S_signs, Y, lam, lam0, phi, phi_gamma, phi_seed, A=A)


# -----------------------------------------------------------------------------------
# msp_solve / msp_solve_backward
# -----------------------------------------------------------------------------------
def solve(P: Precond, A_hi: torch.Tensor, Bv: torch.Tensor, A_lo: torch.Tensor | None = None,
          lam: float | None = None, **opts):
    """X solving the system of P's structure for the right-hand sides Bv ((n,) or (k, n)),
    with regulariser lam (default: the handle's; another value reuses the handle's
    preconditioner). Returns (X, info dict)."""
    L = library()
    A_lo = _pair(P, A_hi, A_lo, Bv.device)
    lam = P.lam if lam is None else float(lam)
    o = _opts(**opts)
    blen = P.m if (P.structure == "general" and not o.normal) else P.n
    k, ldb = _vectors(Bv, blen, "B")
    X = torch.empty((k, P.n) if Bv.dim() == 2 else (P.n,), dtype=torch.float64, device=Bv.device)
    need = B.size_out()
    B.check(L.msp_solve_workspace(P.handle, k, ctypes.byref(o), ctypes.byref(need)))
    ws = _workspace(need.value, Bv.device)
    info = SolveInfo()
    code = L.msp_solve(_stream(Bv.device), P.handle, A_hi.data_ptr(), _code(A_hi), A_lo.data_ptr(), _code(A_lo),
                       A_hi.stride(0), lam, Bv.data_ptr(), ldb, k, X.data_ptr(), P.n, ctypes.byref(o),
                       ws.data_ptr(), ws.numel(), ctypes.byref(info))
    if code not in (0, 3, 4):
        B.check(code)
    d = info.as_dict()
    d["code"] = B.STATUS.get(code, code)
    return X, d


def solve_batched(systems, **opts):
    """Many independent PSD systems in one launch (msp_solve_batched).

    systems: sequence of (P, A_hi, A_lo or None, Bv) with P a "psd" Precond of that
    system, A_hi / A_lo its (n, n) row-major matrices (one leading dimension), Bv of
    shape (k, n) with the same k for every system. Returns (list of X (k, n), list of
    info dicts)."""
    L = library()
    o = _opts(**opts)
    nsys = len(systems)
    if nsys == 0:
        raise ValueError("no systems")
    arr = (B.System * nsys)()
    xs, keep = [], []
    k = None
    hi_t = lo_t = None
    dev = None
    for i, (P, A_hi, A_lo, Bv) in enumerate(systems):
        if P.structure != "psd":
            raise ValueError("batched solves take 'psd' handles")
        if Bv.dim() != 2:
            raise ValueError("Bv must be (k, n)")
        A_lo = _pair(P, A_hi, A_lo, Bv.device)
        kk, ldb = _vectors(Bv, P.n, "B")
        if k is None:
            k, hi_t, lo_t, dev = kk, _code(A_hi), _code(A_lo), Bv.device
        elif kk != k or _code(A_hi) != hi_t or _code(A_lo) != lo_t:
            raise ValueError("every system needs the same k and matrix dtypes")
        X = torch.empty((k, P.n), dtype=torch.float64, device=Bv.device)
        xs.append(X)
        keep.append((A_hi, A_lo, Bv))
        arr[i] = B.System(P.handle.value, A_hi.data_ptr(), A_lo.data_ptr(), A_hi.stride(0), Bv.data_ptr(), ldb,
                          X.data_ptr(), P.n)
    need = B.size_out()
    B.check(L.msp_solve_batched_workspace(nsys, arr, k, ctypes.byref(o), ctypes.byref(need)))
    ws = _workspace(need.value, dev)
    infos = (SolveInfo * nsys)()
    code = L.msp_solve_batched(_stream(dev), nsys, arr, hi_t, lo_t, k, ctypes.byref(o), ws.data_ptr(), ws.numel(),
                               infos)
    if code not in (0, 3, 4, 5):
        B.check(code)
    return xs, [infos[i].as_dict() for i in range(nsys)]


def solve_batched_backward(systems, Xs, Gs, want_dA: bool = False, **opts):
    """Adjoints of many batched PSD solves in one launch (msp_solve_batched_backward).

    systems: the (P, A_hi, A_lo or None, ...) tuples of the forward solve (only the first
    three entries are used); Xs the forward solutions and Gs = dL/dX, each (k, n).
    Returns (list of dB (k, n), list of dlambda, list of dA (n, n) or None, list of info
    dicts)."""
    L = library()
    o = _opts(**opts)
    nsys = len(systems)
    if nsys == 0 or len(Xs) != nsys or len(Gs) != nsys:
        raise ValueError("need one X and one G per system")
    arr = (B.SystemGrad * nsys)()
    dbs, das, keep = [], [], []
    k = hi_t = lo_t = dev = None
    for i, sysd in enumerate(systems):
        P, A_hi, A_lo = sysd[0], sysd[1], sysd[2]
        if P.structure != "psd":
            raise ValueError("batched adjoints take 'psd' handles")
        A_lo = _pair(P, A_hi, A_lo, Gs[i].device)
        kx, ldx = _vectors(Xs[i], P.n, "X")
        kg, ldg = _vectors(Gs[i], P.n, "G")
        if kx != kg:
            raise ValueError("X and G differ in the number of vectors")
        if k is None:
            k, hi_t, lo_t, dev = kx, _code(A_hi), _code(A_lo), Gs[i].device
        elif kx != k or _code(A_hi) != hi_t or _code(A_lo) != lo_t:
            raise ValueError("every system needs the same k and matrix dtypes")
        dB = torch.empty((k, P.n), dtype=torch.float64, device=dev)
        dA = torch.empty((P.n, P.n), dtype=torch.float64, device=dev) if want_dA else None
        dbs.append(dB)
        das.append(dA)
        keep.append((A_hi, A_lo))
        arr[i] = B.SystemGrad(P.handle.value, A_hi.data_ptr(), A_lo.data_ptr(), A_hi.stride(0), Xs[i].data_ptr(), ldx,
                              Gs[i].data_ptr(), ldg, dB.data_ptr(), P.n,
                              dA.data_ptr() if dA is not None else None, P.n)
    need = B.size_out()
    B.check(L.msp_solve_batched_backward_workspace(nsys, arr, k, ctypes.byref(o), ctypes.byref(need)))
    ws = _workspace(need.value, dev)
    infos = (SolveInfo * nsys)()
    dl = (ctypes.c_double * nsys)()
    code = L.msp_solve_batched_backward(_stream(dev), nsys, arr, hi_t, lo_t, k, ctypes.byref(o), ws.data_ptr(),
                                        ws.numel(), dl, infos)
    if code not in (0, 3, 4, 5):
        B.check(code)
    return dbs, [dl[i] for i in range(nsys)], das, [infos[i].as_dict() for i in range(nsys)]


def solve_backward(P: Precond, A_hi, X, G, A_lo=None, want_dA: bool = False, lam: float | None = None, **opts):
    """Adjoint of X = (A + lam I)^{-1} B for PSD A (lam default: the handle's). Returns
    (dB, dlam, dA or None, info)."""
    L = library()
    A_lo = _pair(P, A_hi, A_lo, G.device)
    lam = P.lam if lam is None else float(lam)
    o = _opts(**opts)
    k, ldx = _vectors(X, P.n, "X")
    k2, ldg = _vectors(G, P.n, "G")
    if k != k2:
        raise ValueError("X and G differ in the number of vectors")
    dB = torch.empty_like(G, memory_format=torch.contiguous_format)
    dA = torch.empty((P.n, P.n), dtype=torch.float64, device=G.device) if want_dA else None
    dl = ctypes.c_double(0.0)
    need = B.size_out()
    B.check(L.msp_solve_workspace(P.handle, k, ctypes.byref(o), ctypes.byref(need)))
    ws = _workspace(need.value, G.device)
    info = SolveInfo()
    code = L.msp_solve_backward(_stream(G.device), P.handle, A_hi.data_ptr(), _code(A_hi), A_lo.data_ptr(),
                                _code(A_lo), A_hi.stride(0), lam, X.data_ptr(), ldx, G.data_ptr(), ldg, k,
                                dB.data_ptr(),
                                P.n, ctypes.byref(dl), dA.data_ptr() if dA is not None else None, P.n,
                                ctypes.byref(o), ws.data_ptr(), ws.numel(), ctypes.byref(info))
    if code not in (0, 3, 4):
        B.check(code)
    return dB, dl.value, dA, info.as_dict()


def gaussian_probes(n: int, N: int, seed: int, device="cuda:0") -> torch.Tensor:
    """msp_gaussian_probes: (N, n) float64 Gaussian probes drawn on the device from seed."""
    L = library()
    G = torch.empty((N, n), dtype=torch.float64, device=device)
    B.check(L.msp_gaussian_probes(_stream(G.device), n, N, ctypes.c_uint64(seed & (2 ** 64 - 1)), G.data_ptr(), n))
    return G


def schatten(P: Precond, A_hi, probes, p: float = 1.0, A_lo=None, h: float = 1.5, u_lo: float = float("nan"),
             u_hi: float = float("nan"), kind: str = "schatten", probe_seed: int = 0, nprobes: int | None = None,
             **opts):
    """Hutchinson + quadrature estimate of ||A||_p^p (kind "schatten", P general) or of
    d_lam (kind "effdim", P psd; p is lam). probes: (N, n) float64 on the GPU, or None with
    nprobes = N: the library draws them from probe_seed. Returns (estimate, std_err, info)."""
    L = library()
    if probes is None:
        if not nprobes or nprobes < 1:
            raise ValueError("probes None needs nprobes >= 1")
        dev = A_hi.device
        A_lo = _pair(P, A_hi, A_lo, dev)
        N, ldg = int(nprobes), P.n
        gptr = None
    else:
        A_lo = _pair(P, A_hi, A_lo, probes.device)
        N, ldg = _vectors(probes, P.n, "probes")
        dev = probes.device
        gptr = probes.data_ptr()
    o = _opts(**opts)
    need = B.size_out()
    B.check(L.msp_schatten_workspace(P.handle, N, ctypes.byref(o), ctypes.byref(need)))
    ws = _workspace(need.value, dev)
    est, se = ctypes.c_double(), ctypes.c_double()
    info = SolveInfo()
    kc = B.MSP_TRACE_SCHATTEN_P if kind == "schatten" else B.MSP_TRACE_EFFDIM
    code = L.msp_schatten(_stream(dev), kc, P.handle, A_hi.data_ptr(), _code(A_hi), A_lo.data_ptr(),
                          _code(A_lo), A_hi.stride(0), float(p), gptr, ldg, N,
                          ctypes.c_uint64(probe_seed & (2 ** 64 - 1)), float(h), float(u_lo), float(u_hi),
                          ctypes.byref(o), ws.data_ptr(), ws.numel(), ctypes.byref(est), ctypes.byref(se),
                          ctypes.byref(info))
    if code not in (0, 4):  # 4: a ridge solve hit its cap; the estimate is still written
        B.check(code)
    d = info.as_dict()
    d["code"] = B.STATUS.get(code, code)
    return est.value, se.value, d


def orlicz(P: Precond, A_hi, probes, coefs, powers, A_lo=None, h: float = 1.5, u_hi: float = float("nan"),
           eps_q: float = float("nan"), probe_seed: int = 0, nprobes: int | None = None, **opts):
    """Orlicz norm |A|_g for g(s) = sum_q coefs[q] s^powers[q] (msp_orlicz). probes as for
    schatten. Returns (estimate, std_err, sums, info)."""
    L = library()
    coefs = [float(c) for c in coefs]
    powers = [float(p) for p in powers]
    if len(coefs) != len(powers) or not coefs:
        raise ValueError("coefs and powers need the same nonzero length")
    if probes is None:
        if not nprobes or nprobes < 1:
            raise ValueError("probes None needs nprobes >= 1")
        dev = A_hi.device
        A_lo = _pair(P, A_hi, A_lo, dev)
        N, ldg = int(nprobes), P.n
        gptr = None
    else:
        A_lo = _pair(P, A_hi, A_lo, probes.device)
        N, ldg = _vectors(probes, P.n, "probes")
        dev = probes.device
        gptr = probes.data_ptr()
    o = _opts(**opts)
    need = B.size_out()
    B.check(L.msp_schatten_workspace(P.handle, N, ctypes.byref(o), ctypes.byref(need)))
    ws = _workspace(need.value, dev)
    q = len(coefs)
    c_arr = (ctypes.c_double * q)(*coefs)
    p_arr = (ctypes.c_double * q)(*powers)
    s_arr = (ctypes.c_double * q)()
    est, se = ctypes.c_double(), ctypes.c_double()
    info = SolveInfo()
    code = L.msp_orlicz(_stream(dev), P.handle, A_hi.data_ptr(), _code(A_hi), A_lo.data_ptr(), _code(A_lo),
                        A_hi.stride(0), ctypes.cast(c_arr, ctypes.c_void_p), ctypes.cast(p_arr, ctypes.c_void_p), q,
                        gptr, ldg, N, ctypes.c_uint64(probe_seed & (2 ** 64 - 1)), float(h), float(u_hi),
                        float(eps_q), ctypes.byref(o), ws.data_ptr(), ws.numel(), ctypes.byref(est),
                        ctypes.byref(se), ctypes.cast(s_arr, ctypes.c_void_p), ctypes.byref(info))
    if code not in (0, 4):
        B.check(code)
    d = info.as_dict()
    d["code"] = B.STATUS.get(code, code)
    return est.value, se.value, list(s_arr), d


def kyfan(A: torch.Tensor, k: int, b: int | None = None, q: int = 10, seed: int = 0):
    """Ky Fan k-norm sum_{i<=k} sigma_i(A) (msp_kyfan): b >= k vectors (default min(2k, 64)),
    q steps of subspace iteration. Returns (estimate, the b Ritz values as a list)."""
    L = library()
    _rowmajor(A, "A")
    if A.dtype not in (torch.float64, torch.float32):
        raise ValueError("A must be float64 or float32")
    if not A.is_cuda:
        raise ValueError("A must be on the GPU")
    m, n = A.shape
    b = int(b) if b is not None else min(2 * int(k), 64, m, n)
    need = B.size_out()
    B.check(L.msp_kyfan_workspace(m, n, b, ctypes.byref(need)))
    ws = _workspace(need.value, A.device)
    est = ctypes.c_double()
    sig = (ctypes.c_double * b)()
    B.check(L.msp_kyfan(_stream(A.device), A.data_ptr(), _code(A), m, n, A.stride(0), int(k), b, int(q),
                        ctypes.c_uint64(seed & (2 ** 64 - 1)), ws.data_ptr(), ws.numel(), ctypes.byref(est),
                        ctypes.cast(sig, ctypes.c_void_p)))
    return est.value, list(sig)


def effective_dimension(P: Precond, A_hi, probes, lam: float, **opts):
    return schatten(P, A_hi, probes, p=lam, kind="effdim", **opts)


# -----------------------------------------------------------------------------------
# least squares: msp_left_sketch / msp_lstsq
# -----------------------------------------------------------------------------------
def left_sketch(A: torch.Tensor, q: int, gamma: int, seed: int):
    """Psi (q rows over the n rows of A) and A~ = Psi A. Returns (Psi_rows int32 [n, gamma],
    Psi_signs int8 [n, gamma], A~ float64 [q, d])."""
    L = library()
    _rowmajor(A, "A")
    n, d = A.shape
    rows = torch.empty((n, gamma), dtype=torch.int32, device=A.device)
    signs = torch.empty((n, gamma), dtype=torch.int8, device=A.device)
    At = torch.empty((q, d), dtype=torch.float64, device=A.device)
    need = B.size_out()
    B.check(L.msp_left_sketch_workspace(n, q, gamma, ctypes.byref(need)))
    ws = _workspace(need.value, A.device)
    B.check(L.msp_left_sketch(_stream(A.device), A.data_ptr(), _code(A), n, d, A.stride(0), q, gamma,
                              ctypes.c_uint64(seed & (2 ** 64 - 1)), rows.data_ptr(), signs.data_ptr(),
                              At.data_ptr(), At.stride(0), ws.data_ptr(), ws.numel()))
    return rows, signs, At


def lstsq(P: Precond, At: torch.Tensor, A: torch.Tensor, Bv: torch.Tensor, **opts):
    """argmin |A x - b| for each right-hand side ((n,) or (k, n)) with the MSP_GENERAL
    handle P of A~ = Psi A (lambda = 0). Returns (X, info dict)."""
    L = library()
    _rowmajor(A, "A")
    _rowmajor(At, "A~")
    if At.dtype != torch.float64:
        raise ValueError("A~ must be float64")
    if P.structure != "general" or tuple(At.shape) != (P.m, P.n):
        raise ValueError("P must be the MSP_GENERAL handle built from this A~ (shape (q, d))")
    if A.shape[1] != P.n or A.shape[0] < P.n:
        raise ValueError("A must be tall (n x d, n >= d) with the d columns of A~")
    n = A.shape[0]
    o = _opts(**opts)
    k, ldb = _vectors(Bv, n, "B")
    X = torch.empty((k, P.n) if Bv.dim() == 2 else (P.n,), dtype=torch.float64, device=Bv.device)
    need = B.size_out()
    B.check(L.msp_lstsq_workspace(P.handle, n, k, ctypes.byref(o), ctypes.byref(need)))
    ws = _workspace(need.value, Bv.device)
    info = SolveInfo()
    code = L.msp_lstsq(_stream(Bv.device), P.handle, At.data_ptr(), At.stride(0), A.data_ptr(), _code(A), n,
                       A.stride(0), Bv.data_ptr(), ldb, k, X.data_ptr(), P.n, ctypes.byref(o), ws.data_ptr(),
                       ws.numel(), ctypes.byref(info))
    if code not in (0, 4):
        B.check(code)
    d = info.as_dict()
    d["code"] = B.STATUS.get(code, code)
    return X, d


# -----------------------------------------------------------------------------------
# convenience: the whole path in one call, and the autograd wrapper
# -----------------------------------------------------------------------------------
@dataclass
class SketchParams:
    s: int
    gamma: int = 8
    phi: int | None = None
    phi_gamma: int = 8
    seed: int = 0
    phi_seed: int = 1


def msp_solve(A: torch.Tensor, Bv: torch.Tensor, lam: float, lam0: float, sp: SketchParams, A_lo=None,
              structure: str = "psd", **opts):
    """sketch -> nystrom -> solve. Returns (X, info, precond)."""
    A_sk = A if A_lo is None else A_lo
    rows, signs, Y = sketch(A_sk, sp.s, sp.gamma, sp.seed)
    P = Precond(structure, rows, signs, Y, lam, lam0, sp.phi or 4 * sp.s, sp.phi_gamma, sp.phi_seed)
    X, info = solve(P, A, Bv, A_lo=A_lo, **opts)
    return X, info, P


class MSPSolve(torch.autograd.Function):
    """X = (A + lam I)^{-1} B for symmetric PSD A through MSP, with the adjoint solve
    (msp_solve_backward) reusing the same preconditioner. The solve and its adjoint use the
    value of `lam` (a float or a 0-d tensor), whatever the handle was built for; a value
    far from the handle's lambda only costs iterations. A solve or adjoint that does not
    reach its tolerance raises MspError."""

    @staticmethod
    def forward(ctx, A, Bv, lam, P, opts):
        lv = float(lam.detach().item() if isinstance(lam, torch.Tensor) else lam)
        X, info = solve(P, A, Bv, lam=lv, **opts)
        if info["status"] != "MSP_OK":
            raise MspError(B.STATUS_CODE[info["status"]], f"forward solve: {info['status']}")
        ctx.save_for_backward(A, X)
        ctx.P = P
        ctx.lam = lv
        ctx.opts = opts
        ctx.info = info
        return X

    @staticmethod
    def backward(ctx, G):
        A, X = ctx.saved_tensors
        want_dA = ctx.needs_input_grad[0]
        dB, dlam, dA, info = solve_backward(ctx.P, A, X, G.contiguous(), want_dA=want_dA, lam=ctx.lam, **ctx.opts)
        if info["status"] != "MSP_OK":
            raise MspError(B.STATUS_CODE[info["status"]], f"adjoint solve: {info['status']}")
        dl = torch.tensor(dlam, dtype=torch.float64, device=G.device) if ctx.needs_input_grad[2] else None
        return dA, dB, dl, None, None
