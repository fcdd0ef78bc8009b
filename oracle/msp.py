"""Multi-level Sketched Preconditioning, step by step in FP64 (oracle side).

PsdMsp      Algorithm 1 (two-level MSP for (A + lam I) x = b, A PSD) with
            Algorithm 2 (SolveM1, the level-2 solve).
GeneralMsp  Algorithm 3 (three-level MSP for (A^T A + lam I) x = c) with
            Algorithm 4 (SolveM1) and Algorithm 5 (SolveM2, level 3).

Readings taken where the paper is silent or loose:
  * lam~ = lam + lam0 everywhere, including M2 and M3b (Section 4 uses lam once).
  * Phi is a Definition 2.1 sketch with phi rows and phi_gamma nonzeros per column,
    drawn from its own seed (Lemma 2.2 only cites a construction).
  * W is symmetrised, (W + W^T)/2, after W = S C (exact arithmetic makes it symmetric).
  * The explicit inverses the algorithms precompute (M2^{-1}, M3a^{-1}, M3b^{-1}) are
    formed from a Cholesky factor of the matrix plus mu I, mu = shift_rel * tr / s
    (guards rank-deficient W when rank(A) < s; negligible otherwise).
  * Level-2 operator: (C^T C + lam~ W) y = C^T (C y) + lam~ (W y) from the stored C
    and W (the cost paragraph of Section 4 drops the lam~ factor in its shorthand).
  * Iterations at every level are flexible PCG; each stops on its recurrence residual
    |r| <= tau |rhs| (tau: tol at level 1, inner_tol at level 2, level3_tol at level 3)
    or after max_inner / max_level3 steps; level 1 confirms the stop on the residual
    recomputed from A.
  * SolveM2 applies (W^2 + lam~ W)^{-1} r in the product form W^{-1} (W + lam~ I)^{-1} r
    (the first line of the identity in Section 5) by default; the difference form
    (u - v) / lam~ of Algorithm 5 is kept as a switch.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import scipy.linalg as sla

from . import rng, sketch
from .krylov import KrylovResult, fcg


@dataclass
class MspOptions:
    tol: float = 1e-8
    max_outer: int = 5000
    inner_tol: float = 1e-10
    max_inner: int = 200
    level3_tol: float = 1e-10
    max_level3: int = 200
    shift_rel: float = 1e-12
    m2_form: str = "product"      # or "difference" (Algorithm 5 as printed)


def paper_lambda0(eigs_desc: np.ndarray, l: int) -> float:
    """lam0 = (2/l) sum_{i>l} lambda_i (Theorem 4.1; Theorem 3.1 uses sigma_i^2)."""
    e = np.asarray(eigs_desc, dtype=np.float64)
    return float(2.0 / l * e[l:].sum())


def paper_lambda0_from_top(trace: float, top_l: np.ndarray, l: int) -> float:
    """The same lam0 from tr(A) and the l largest eigenvalues: sum_{i>l} = tr - sum_{i<=l}."""
    top = np.sort(np.asarray(top_l, dtype=np.float64))[::-1][:l]
    return float(2.0 / l * (trace - top.sum()))


def lambda0_estimate(a: np.ndarray, c: np.ndarray, w: np.ndarray, l: int) -> float:
    """lam0 when the tail spectrum is unknown (reading of Theorem 4.1's lam0, which needs
    sum_{i>l} lambda_i): (2/l) max(tr(A) - tr(A_nys), 0), where A_nys = C W^+ C^T is the
    Nystrom approximation that Algorithm 1 builds from C = A S^T and W = S C, so
    tr(A_nys) = tr(W^+ C^T C). A - A_nys is PSD and A_nys has rank <= s, hence (Weyl) the
    deficit is at least sum_{i>s} lambda_i, and it is 0 when rank(A) <= s.

    W^+ is taken as (W + mu I)^{-1} with mu = 1e-9 tr(W) / s: C (W + mu I)^{-1} C^T is still
    below A and of rank <= s (so the bound holds), and mu keeps the directions in which a
    rank-deficient W is zero up to rounding from being amplified. A deficit below 1e-6 tr(A)
    is taken as the rounding of an exact recovery and counts as 0."""
    winv = spd_inverse(0.5 * (w + w.T), 1e-9)
    tr_a = float(np.trace(a))
    deficit = tr_a - float(np.sum(winv * (c.T @ c)))
    if deficit <= 1e-6 * tr_a:
        return 0.0
    return float(2.0 / l * deficit)


def spd_inverse(m: np.ndarray, shift_rel: float) -> np.ndarray:
    """(M + mu I)^{-1} from a Cholesky factor, mu = shift_rel * tr(M) / dim."""
    d = m.shape[0]
    mu = shift_rel * float(np.trace(m)) / d
    L = np.linalg.cholesky(m + mu * np.eye(d))
    Linv = sla.solve_triangular(L, np.eye(d), lower=True)
    inv = Linv.T @ Linv
    return 0.5 * (inv + inv.T)


@dataclass
class SolveInfo:
    outer_iterations: int = 0
    inner_iterations: int = 0
    level3_iterations: int = 0
    status: str = ""
    rel_residual: float = float("nan")
    restarts: int = 0


# ==================================================================================
# Two-level MSP for PSD A (Algorithms 1 and 2)
# ==================================================================================
class PsdMsp:
    def __init__(self, a: np.ndarray, lam: float, lam0: float, s: int, gamma: int, seed_s: int,
                 phi: int, phi_gamma: int, seed_phi: int, opts: MspOptions | None = None):
        self.a = a
        self.n = a.shape[0]
        self.lam = float(lam)
        self.lam0 = float(lam0)
        self.opts = opts or MspOptions()
        # Algorithm 1: sparse embedding S (Definition 2.1)
        self.s_rows, self.s_signs = rng.sketch_indices(seed_s, self.n, s, gamma)
        self.s = s
        # then lam~ = lam + lam0, C = A S^T, W = S C
        self.lt = self.lam + self.lam0
        self.c = sketch.right_sketch(a, self.s_rows, self.s_signs, s)
        w = sketch.left_sketch(self.s_rows, self.s_signs, s, self.c)
        self.w = 0.5 * (w + w.T)
        # then C~ = Phi C, M2 = C~^T C~ + lam~ W, and its inverse
        self.phi_rows, self.phi_signs = rng.sketch_indices(seed_phi, self.n, phi, phi_gamma)
        self.ct = sketch.left_sketch(self.phi_rows, self.phi_signs, phi, self.c)
        m2 = self.ct.T @ self.ct + self.lt * self.w
        self.m2 = 0.5 * (m2 + m2.T)
        self.m2inv = spd_inverse(self.m2, self.opts.shift_rel)
        self.info = SolveInfo()

    # level-2 operator and preconditioner
    def op2(self, y):
        return self.c.T @ (self.c @ y) + self.lt * (self.w @ y)

    def prec2(self, v):
        return self.m2inv @ v

    def solve_m1(self, r):
        """Algorithm 2: y^ ~= (C^T C + lam~ W)^{-1} C^T r by level-2 PCG with M2^{-1},
        then w^ = (r - C y^) / lam~."""
        rhs = self.c.T @ r
        res = fcg(self.op2, rhs, self.prec2, self.opts.inner_tol, self.opts.max_inner)
        self.info.inner_iterations += res.iterations
        return (r - self.c @ res.x) / self.lt

    def op1(self, x):
        return self.a @ x + self.lam * x

    def solve(self, b) -> KrylovResult:
        """Algorithm 1, the level-1 iteration on (A + lam I) x = b with SolveM1."""
        b = np.asarray(b, dtype=np.float64)
        self.info = SolveInfo()
        res = fcg(self.op1, b, self.solve_m1, self.opts.tol, self.opts.max_outer,
                  true_residual=lambda x: b - self.op1(x))
        self.info.outer_iterations = res.iterations
        self.info.status = res.status
        self.info.restarts = res.restarts
        bn = np.linalg.norm(b)
        self.info.rel_residual = float(np.linalg.norm(b - self.op1(res.x)) / bn) if bn > 0 else 0.0
        return res

    def m_inverse_dense(self):
        """(C W^+ C^T + lam~ I)^{-1} assembled densely (tests only)."""
        wp = np.linalg.pinv(self.w, rcond=1e-12, hermitian=True)
        m = self.c @ wp @ self.c.T + self.lt * np.eye(self.n)
        return np.linalg.inv(m)


# ==================================================================================
# Three-level MSP for general A (Algorithms 3, 4 and 5)
# ==================================================================================
class GeneralMsp:
    def __init__(self, a: np.ndarray, lam: float, lam0: float, s: int, gamma: int, seed_s: int,
                 phi: int, phi_gamma: int, seed_phi: int, opts: MspOptions | None = None):
        self.a = a
        self.m, self.n = a.shape
        self.lam = float(lam)
        self.lam0 = float(lam0)
        self.opts = opts or MspOptions()
        # Algorithm 3: lam~
        self.lt = self.lam + self.lam0
        # then S (s x n)
        self.s_rows, self.s_signs = rng.sketch_indices(seed_s, self.n, s, gamma)
        self.s = s
        # then A~ = A S^T (m x s), A^ = Phi A~ (phi x s), Phi over the m rows
        self.at = sketch.right_sketch(a, self.s_rows, self.s_signs, s)
        self.phi_rows, self.phi_signs = rng.sketch_indices(seed_phi, self.m, phi, phi_gamma)
        self.ah = sketch.left_sketch(self.phi_rows, self.phi_signs, phi, self.at)
        # then M3a = A^^T A^, M3b = M3a + lam~ I and their inverses
        m3a = self.ah.T @ self.ah
        self.m3a = 0.5 * (m3a + m3a.T)
        self.m3b = self.m3a + self.lt * np.eye(s)
        self.m3a_inv = spd_inverse(self.m3a, self.opts.shift_rel)
        self.m3b_inv = spd_inverse(self.m3b, self.opts.shift_rel)
        self.info = SolveInfo()

    # W y = A~^T A~ y, never formed (Section 5)
    def w_apply(self, y):
        return self.at.T @ (self.at @ y)

    def solve_m2(self, r):
        """Algorithm 5: z ~= (W^2 + lam~ W)^{-1} r through two level-3 PCG solves."""
        o = self.opts
        wb = lambda y: self.w_apply(y) + self.lt * y
        if o.m2_form == "product":
            v = fcg(wb, r, lambda y: self.m3b_inv @ y, o.level3_tol, o.max_level3)
            u = fcg(self.w_apply, v.x, lambda y: self.m3a_inv @ y, o.level3_tol, o.max_level3)
            self.info.level3_iterations += v.iterations + u.iterations
            return u.x
        u = fcg(self.w_apply, r, lambda y: self.m3a_inv @ y, o.level3_tol, o.max_level3)
        v = fcg(wb, r, lambda y: self.m3b_inv @ y, o.level3_tol, o.max_level3)
        self.info.level3_iterations += v.iterations + u.iterations
        return (u.x - v.x) / self.lt

    def op2(self, y):
        """A~^T A A^T A~ y + lam~ A~^T A~ y (the operator of Algorithm 4)."""
        t = self.at @ y
        return self.at.T @ (self.a @ (self.a.T @ t)) + self.lt * (self.at.T @ t)

    def solve_m1(self, r):
        """Algorithm 4: level-2 solve preconditioned by SolveM2, then
        w^ = (r - A^T A~ y^) / lam~."""
        rhs = self.at.T @ (self.a @ r)
        res = fcg(self.op2, rhs, self.solve_m2, self.opts.inner_tol, self.opts.max_inner)
        self.info.inner_iterations += res.iterations
        return (r - self.a.T @ (self.at @ res.x)) / self.lt

    def op1(self, x):
        return self.a.T @ (self.a @ x) + self.lam * x

    def solve_normal(self, c) -> KrylovResult:
        """Algorithm 3, the level-1 iteration on (A^T A + lam I) x = c."""
        c = np.asarray(c, dtype=np.float64)
        self.info = SolveInfo()
        res = fcg(self.op1, c, self.solve_m1, self.opts.tol, self.opts.max_outer,
                  true_residual=lambda x: c - self.op1(x))
        self.info.outer_iterations = res.iterations
        self.info.status = res.status
        self.info.restarts = res.restarts
        cn = np.linalg.norm(c)
        self.info.rel_residual = float(np.linalg.norm(c - self.op1(res.x)) / cn) if cn > 0 else 0.0
        return res

    def solve_system(self, b) -> KrylovResult:
        """A x = b through the normal equations with c = A^T b and lam = 0 (proof of
        Theorem 1.1). The level-1 iteration is the same flexible PCG on A^T A; its stop
        is taken on the residual of the user's system, |b - A x| <= tol |b|, carried by
        the recurrence rho <- rho - alpha (A p) and confirmed on b - A x."""
        if self.lam != 0.0:
            raise ValueError("solve_system needs lam = 0")
        b = np.asarray(b, dtype=np.float64)
        self.info = SolveInfo()
        o = self.opts
        x = np.zeros(self.n)
        bn = float(np.linalg.norm(b))
        if bn == 0.0:
            self.info.status = "zero_rhs"
            self.info.rel_residual = 0.0
            return KrylovResult(x, 0, "zero_rhs")
        rho = b.copy()
        r = self.a.T @ rho
        z = self.solve_m1(r)
        p = z.copy()
        rz = float(r @ z)
        it, status, restarts = 0, "max_iter", 0
        while it < o.max_outer:
            t = self.a @ p
            q = self.a.T @ t
            pq = float(p @ q)
            if not (pq > 0.0):
                status = "breakdown"
                break
            alpha = rz / pq
            x = x + alpha * p
            rho = rho - alpha * t
            r_old = r
            r = r - alpha * q
            it += 1
            if np.linalg.norm(rho) <= o.tol * bn:
                rho = b - self.a @ x
                if np.linalg.norm(rho) <= o.tol * bn:
                    status = "converged"
                    break
                restarts += 1
                r = self.a.T @ rho
                z = self.solve_m1(r)
                p = z.copy()
                rz = float(r @ z)
                continue
            z = self.solve_m1(r)
            beta = float(z @ (r - r_old)) / rz
            rz = float(r @ z)
            p = z + beta * p
        self.info.outer_iterations = it
        self.info.status = status
        self.info.restarts = restarts
        self.info.rel_residual = float(np.linalg.norm(b - self.a @ x) / bn)
        return KrylovResult(x, it, status, restarts=restarts)
