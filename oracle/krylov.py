"""Krylov iterations of the oracle: flexible PCG (every level) and Algorithm 6.

Algorithm 6 (preconditioned Lanczos with an inexact SolveM) is the iteration the paper
analyses (Theorem 6.1). Section 6 notes that PCG returns the same iterate as Lanczos
when all arithmetic is exact. Because SolveM at levels 1 and 2 is itself an iterative
solve with a data-dependent stopping rule, the preconditioner is a (slightly) nonlinear
operator, so both the oracle and the GPU path run the *flexible* form of PCG: the
Polak-Ribiere choice beta = <z_new, r_new - r_old> / <z_old, r_old> (the inexact /
flexible CG of Golub-Ye 1999 and Notay 2000). With an exact, fixed preconditioner it
equals ordinary PCG and hence Algorithm 6; ``tests/test_oracle_krylov.py`` pins that.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


@dataclass
class KrylovResult:
    x: np.ndarray
    iterations: int
    status: str                       # "converged" | "max_iter" | "breakdown" | "zero_rhs"
    residual_history: list = field(default_factory=list)
    restarts: int = 0


def fcg(op, b, prec, tol: float, max_iter: int, true_residual=None) -> KrylovResult:
    """Flexible PCG on op(x) = b, x0 = 0.

    Stops when the recurrence residual satisfies |r| <= tol |b|. If ``true_residual``
    is given (a function x -> b - op(x) evaluated afresh), the stop is confirmed on it;
    when it fails the iteration restarts from the recomputed residual.
    """
    b = np.asarray(b, dtype=np.float64)
    x = np.zeros_like(b)
    bnorm = float(np.linalg.norm(b))
    if bnorm == 0.0:
        return KrylovResult(x, 0, "zero_rhs", [0.0])
    target = tol * bnorm
    r = b.copy()
    z = prec(r)
    p = z.copy()
    rz = float(r @ z)
    hist = [1.0]
    restarts = 0
    it = 0
    while it < max_iter:
        q = op(p)
        pq = float(p @ q)
        if not (pq > 0.0):
            return KrylovResult(x, it, "breakdown", hist, restarts)
        alpha = rz / pq
        x = x + alpha * p
        r_old = r
        r = r - alpha * q
        it += 1
        rn = float(np.linalg.norm(r))
        hist.append(rn / bnorm)
        if rn <= target:
            if true_residual is None:
                return KrylovResult(x, it, "converged", hist, restarts)
            r = true_residual(x)
            rn = float(np.linalg.norm(r))
            hist[-1] = rn / bnorm
            if rn <= target:
                return KrylovResult(x, it, "converged", hist, restarts)
            restarts += 1
            z = prec(r)
            p = z.copy()
            rz = float(r @ z)
            continue
        z = prec(r)
        if not (rz != 0.0 and np.isfinite(rz)):
            # beta's denominator <r_old, z_old> vanished (an inexact preconditioner that
            # is not positive definite): no conjugate direction can be formed
            return KrylovResult(x, it, "breakdown", hist, restarts)
        beta = float(z @ (r - r_old)) / rz
        rz = float(r @ z)
        p = z + beta * p
    return KrylovResult(x, it, "max_iter", hist, restarts)


def lanczos_alg6(op, b, solve_m, t: int) -> np.ndarray:
    """Algorithm 6 (preconditioned Lanczos with SolveM), t iterations, x0 = 0.

    Two vector families are carried: q (under-bar, in the space of A's range) and
    q-bar = M^{-1} q. The initialisation uses w0-bar = SolveM(b), z' = <b, w0-bar>^{1/2},
    q-bar_1 = w0-bar / z' and q_1 = b / z' (the printed initialisation divides the
    undefined w' by z; the reading here is the only one that makes q-bar = M^{-1} q).
    Returns x_t = z' Q-bar T^{-1} e_1.
    """
    b = np.asarray(b, dtype=np.float64)
    w0bar = solve_m(b)
    zp = float(np.sqrt(b @ w0bar))
    q_prev = np.zeros_like(b)
    qbar = w0bar / zp
    q = b / zp
    beta = 0.0
    alphas, betas, qbars = [], [], []
    for _ in range(t):
        u = op(qbar) - beta * q_prev
        alpha = float(u @ qbar)
        w = u - alpha * q
        wbar = solve_m(w)
        alphas.append(alpha)
        qbars.append(qbar)
        beta_next = float(np.sqrt(max(w @ wbar, 0.0)))
        if beta_next == 0.0:
            break
        betas.append(beta_next)
        q_prev, q, qbar, beta = q, w / beta_next, wbar / beta_next, beta_next
    k = len(alphas)
    T = np.diag(alphas)
    if k > 1:
        off = np.asarray(betas[:k - 1])
        T += np.diag(off, 1) + np.diag(off, -1)
    e1 = np.zeros(k)
    e1[0] = 1.0
    return zp * (np.column_stack(qbars) @ np.linalg.solve(T, e1))
