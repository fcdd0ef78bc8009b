"""Plain definitions of every final result the hot path produces (oracle side).

These are the results MSP reaches approximately: x* = (A + lam I)^{-1} b for PSD A
(Theorem 3.2), the minimum-norm solution of A x = b (proof of Theorem 1.1), the ridge
solution (A^T A + lam I)^{-1} c (Theorem 3.1), Schatten-p norms and the effective
dimension (Section 2), and the gradients of x = (A + lam I)^{-1} b.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla


def solve_psd(a, b, lam):
    """(A + lam I)^{-1} b by dense Cholesky (one copy of A, shifted on its diagonal)."""
    m = np.array(a, dtype=np.float64, copy=True)
    m[np.diag_indices_from(m)] += lam
    f = sla.cho_factor(m, lower=True, overwrite_a=True)
    return sla.cho_solve(f, b)


def solve_general(a, b):
    """A^{-1} b by dense LU (A square, nonsingular)."""
    return np.linalg.solve(a, b)


def solve_ridge(a, c, lam):
    """(A^T A + lam I)^{-1} c through the SVD of A (no squaring of the condition)."""
    u, sv, vt = np.linalg.svd(a, full_matrices=False)
    return vt.T @ ((vt @ c) / (sv * sv + lam)[:, None] if np.ndim(c) == 2 else (vt @ c) / (sv * sv + lam))


def rel_residual_psd(a, x, b, lam):
    return float(np.linalg.norm(b - a @ x - lam * x) / np.linalg.norm(b))


def schatten_p(sv, p):
    """||A||_p^p = sum_i sigma_i^p."""
    return float(np.sum(np.asarray(sv, dtype=np.float64) ** p))


def effective_dimension(eigs, lam):
    """d_lam = tr(A (A + lam I)^{-1}) = sum_i lambda_i / (lambda_i + lam) (Section 2)."""
    e = np.asarray(eigs, dtype=np.float64)
    return float(np.sum(e / (e + lam)))


def gradients(a, lam, x, g):
    """For X = (A + lam I)^{-1} B and G = dL/dX: dB = (A + lam I)^{-T} G,
    dA = -dB X^T, dlam = -<dB, X>."""
    n = a.shape[0]
    db = np.linalg.solve((a + lam * np.eye(n)).T, g)
    da = -db @ x.T if x.ndim == 2 else -np.outer(db, x)
    dlam = -float(np.sum(db * x))
    return db, da, dlam
