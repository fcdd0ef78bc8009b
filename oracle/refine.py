"""Mixed precision around MSP (oracle side).

The paper works in exact arithmetic. The precision scheme here is a design reading:
A is stored and swept in a low precision (FP32, or BF16) and FP64 accuracy is won back
by iterative refinement with residuals on the high-precision matrix:

    x_0 = 0;  r_k = b - (A_hi + lam I) x_k  (FP64);  x_{k+1} = x_k + MSP_lo(r_k)

until |r_k| <= tol |b|. If two consecutive steps each fail to halve |r|, the loop
switches to Krylov-based refinement: flexible PCG in FP64 on (A_hi + lam I) with the
low-precision MSP solve as its (nonlinear) preconditioner.

Rounding: FP32 is round-to-nearest-even from FP64; BF16 is round-to-nearest-even of
the FP32 value to its upper 16 bits.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from .krylov import fcg


def round_f32(a: np.ndarray) -> np.ndarray:
    return np.asarray(a, dtype=np.float64).astype(np.float32)


def round_bf16(a: np.ndarray) -> np.ndarray:
    """BF16 values (returned as float32) of RNE(FP32(a))."""
    f = np.ascontiguousarray(np.asarray(a, dtype=np.float64).astype(np.float32))
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + np.uint64(0x7FFF) + ((u >> np.uint64(16)) & np.uint64(1))) & np.uint64(0xFFFF0000)
    return u.astype(np.uint32).view(np.float32).reshape(f.shape)


@dataclass
class RefineInfo:
    steps: int = 0
    krylov: bool = False
    status: str = ""
    history: list = field(default_factory=list)


def refine(op_hi, b, solve_lo, tol: float, max_steps: int = 50):
    """FP64 iterative refinement; ``op_hi(x)`` applies the FP64 operator and
    ``solve_lo(r)`` returns an approximate correction from the low-precision solve."""
    b = np.asarray(b, dtype=np.float64)
    bn = float(np.linalg.norm(b))
    info = RefineInfo()
    x = np.zeros_like(b)
    if bn == 0.0:
        info.status = "zero_rhs"
        return x, info
    r = b.copy()
    info.history.append(1.0)
    slow = 0
    while info.steps < max_steps:
        x = x + solve_lo(r)
        r = b - op_hi(x)
        info.steps += 1
        rel = float(np.linalg.norm(r)) / bn
        if rel <= tol:
            info.status = "converged"
            info.history.append(rel)
            return x, info
        slow = slow + 1 if rel > 0.5 * info.history[-1] else 0
        info.history.append(rel)
        if slow >= 2:
            break
    # Krylov refinement on the remaining residual
    info.krylov = True
    res = fcg(op_hi, r, solve_lo, tol * bn / float(np.linalg.norm(r)), 500,
              true_residual=None)
    x = x + res.x
    r = b - op_hi(x)
    info.history.append(float(np.linalg.norm(r)) / bn)
    info.status = "converged" if info.history[-1] <= tol else res.status
    return x, info
