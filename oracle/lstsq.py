"""Least squares min |A x - b| for a tall A by sketch-and-precondition with MSP as the inner
solver (the least-squares corollary of Section 3) -- oracle side, test infrastructure only.

Steps in the corollary's order:
  1. Psi, a Definition 2.1 sketch with q rows over the n rows of A (psi_gamma nonzeros
     +-1/sqrt(psi_gamma) per column), and A~ = Psi A (q x d): a subspace embedding of A.
  2. An outer iterative least-squares solver on A^T A x = A^T b preconditioned by
     (A~^T A~)^{-1}; each application is a ridge-free normal-equation solve with A~, done by
     the three-level MSP of Algorithms 3-5 to a constant relative accuracy.
Readings where the corollary leaves the solver open: the outer solver is the flexible
PCG used at every other level; it stops on |A^T (b - A x)| <= tol |A^T b|, confirmed on the
recomputed residual; the inner accuracy is a parameter (inner_rel).

Parity: `lstsq_dense` is the plain definition (numpy's SVD-based least squares); the
pins in tests/test_oracle_lstsq.py check the iteration against it, its count against the
subspace-embedding bound, and consistent systems.
"""
from __future__ import annotations

import numpy as np

from . import rng, sketch
from .krylov import KrylovResult, fcg
from .msp import GeneralMsp, MspOptions


def lstsq_dense(a, b):
    """argmin_x |A x - b| (minimum-norm) by numpy's SVD-based solver."""
    return np.linalg.lstsq(a, b, rcond=None)[0]


class LstsqMsp:
    def __init__(self, a: np.ndarray, q: int, psi_gamma: int, seed_psi: int, s: int, gamma: int, seed_s: int,
                 phi: int, phi_gamma: int, seed_phi: int, lam0: float, inner_rel: float = 1e-4,
                 opts: MspOptions | None = None):
        self.a = np.asarray(a, dtype=np.float64)
        self.n, self.d = self.a.shape
        self.opts = opts or MspOptions()
        # step 1: A~ = Psi A
        self.psi_rows, self.psi_signs = rng.sketch_indices(seed_psi, self.n, q, psi_gamma)
        self.at = sketch.left_sketch(self.psi_rows, self.psi_signs, q, self.a)
        # the inner three-level MSP on A~ (lam = 0), solved to inner_rel
        inner_opts = MspOptions(tol=inner_rel, inner_tol=self.opts.inner_tol, level3_tol=self.opts.level3_tol,
                                max_outer=self.opts.max_outer, max_inner=self.opts.max_inner,
                                max_level3=self.opts.max_level3, shift_rel=self.opts.shift_rel,
                                m2_form=self.opts.m2_form)
        self.inner = GeneralMsp(self.at, 0.0, lam0, s, gamma, seed_s, phi, phi_gamma, seed_phi, inner_opts)
        self.inner_steps = 0

    def prec(self, g):
        """(A~^T A~)^{-1} g to the inner accuracy."""
        res = self.inner.solve_normal(g)
        self.inner_steps += res.iterations
        return res.x

    def op(self, x):
        return self.a.T @ (self.a @ x)

    def solve(self, b) -> KrylovResult:
        """Step 2: flexible PCG on A^T A x = A^T b with the MSP preconditioner."""
        c = self.a.T @ np.asarray(b, dtype=np.float64)
        return fcg(self.op, c, self.prec, self.opts.tol, self.opts.max_outer,
                   true_residual=lambda x: c - self.op(x))
