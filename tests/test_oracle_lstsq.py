"""Pins of the least-squares oracle (sketch-and-precondition around MSP, Section 3)."""
import math

import numpy as np
import pytest

import workloads as W
from oracle import lstsq
from oracle import msp as omsp
from oracle.krylov import fcg

N, D, K = 600, 40, 4
Q, S = 4 * D, 16


def _case(cid=601):
    a, sv = W.tall_outlier(N, D, K, cid)
    b = W.gaussian(N, cid)
    lam0 = omsp.paper_lambda0(sv ** 2, S // 2)
    return a, sv, b, lam0


def _solver(a, lam0, tol=1e-12, inner_rel=1e-4):
    return lstsq.LstsqMsp(a, Q, 8, 31, S, 8, 32, 4 * S, 8, 33, lam0, inner_rel=inner_rel,
                          opts=omsp.MspOptions(tol=tol, inner_tol=1e-10, level3_tol=1e-10))


def test_matches_dense_least_squares_within_the_residual_bound():
    a, sv, b, lam0 = _case()
    L = _solver(a, lam0)
    res = L.solve(b)
    assert res.status == "converged", res.status
    xs = lstsq.lstsq_dense(a, b)
    c = a.T @ b
    r = c - a.T @ (a @ res.x)
    assert np.linalg.norm(r) <= 1e-12 * np.linalg.norm(c) * (1 + 1e-9)
    # x - x* = (A^T A)^{-1} r, so |x - x*| <= |r| / sigma_min^2
    assert np.linalg.norm(res.x - xs) <= 1.01 * np.linalg.norm(r) / sv[-1] ** 2 + 1e-13 * np.linalg.norm(xs)
    # the optimality of the residual: b - A x is orthogonal to the range of A
    assert np.linalg.norm(a.T @ (b - a @ res.x)) <= 1e-12 * np.linalg.norm(c) * (1 + 1e-9)


def test_exact_inner_solve_meets_the_subspace_embedding_bound():
    # with (A~^T A~)^{-1} applied exactly the outer iteration is PCG with a fixed SPD
    # preconditioner: |r_t| / |r_0| <= sqrt(cond(A^T A)) 2 rho^t, rho = (sqrt(k)-1)/(sqrt(k)+1),
    # k = cond((A~^T A~)^{-1} A^T A)
    a, sv, b, lam0 = _case(602)
    L = _solver(a, lam0)
    m = L.at.T @ L.at
    minv = np.linalg.inv(m)
    ev = np.linalg.eigvals(minv @ (a.T @ a)).real
    kp = ev.max() / ev.min()
    assert kp < 16.0  # q = 4 d rows, 8 nonzeros per column: a constant-distortion embedding
    tol = 1e-10
    c = a.T @ b
    res = fcg(lambda x: a.T @ (a @ x), c, lambda g: minv @ g, tol, 500)
    assert res.status == "converged"
    rho = (math.sqrt(kp) - 1) / (math.sqrt(kp) + 1)
    cond = (sv[0] / sv[-1]) ** 2
    t_bound = math.ceil(math.log(2 * math.sqrt(cond) / tol) / math.log(1 / rho))
    assert res.iterations <= t_bound


def test_consistent_system_recovers_the_solution():
    a, sv, _, lam0 = _case(603)
    x0 = W.gaussian(D, 603)
    b = a @ x0
    res = _solver(a, lam0).solve(b)
    c = a.T @ b
    r = c - a.T @ (a @ res.x)
    assert np.linalg.norm(res.x - x0) <= 1.01 * np.linalg.norm(r) / sv[-1] ** 2 + 1e-12 * np.linalg.norm(x0)
    assert np.linalg.norm(b - a @ res.x) <= 1e-8 * np.linalg.norm(b)


def test_inexact_inner_solves_still_converge():
    # constant inner accuracy suffices (flexible outer iteration)
    a, sv, b, lam0 = _case(604)
    res = _solver(a, lam0, tol=1e-10, inner_rel=1e-1).solve(b)
    assert res.status == "converged"
    xs = lstsq.lstsq_dense(a, b)
    c = a.T @ b
    r = c - a.T @ (a @ res.x)
    assert np.linalg.norm(res.x - xs) <= 1.01 * np.linalg.norm(r) / sv[-1] ** 2 + 1e-12 * np.linalg.norm(xs)


def test_generator_is_tall_with_the_stated_spectrum():
    a, sv = W.tall_outlier(300, 20, 3, 605)
    assert a.shape == (300, 20)
    assert np.allclose(np.linalg.svd(a, compute_uv=False), sv, rtol=1e-10)
    assert sv[2] >= 1e2 and sv[3] <= 10.0
