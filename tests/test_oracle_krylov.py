"""Pins of the oracle's Krylov iterations (Section 6)."""
import numpy as np
import pytest

from oracle import krylov


def _spd(n, cond, seed):
    r = np.random.default_rng(seed)
    q, _ = np.linalg.qr(r.standard_normal((n, n)))
    ev = np.geomspace(1.0, cond, n)
    return (q * ev) @ q.T, ev


def test_fcg_solves_spd_system():
    a, _ = _spd(60, 1e3, 0)
    b = np.random.default_rng(1).standard_normal(60)
    res = krylov.fcg(lambda x: a @ x, b, lambda r: r, 1e-12, 500)
    assert res.status == "converged"
    assert np.allclose(res.x, np.linalg.solve(a, b), rtol=0, atol=1e-9 * np.linalg.norm(np.linalg.solve(a, b)))


@pytest.mark.parametrize("t", [1, 3, 8, 20])
def test_alg6_equals_pcg_with_exact_preconditioner(t):
    # Section 6: PCG and Lanczos produce the same iterate in exact arithmetic.
    n = 80
    a, _ = _spd(n, 1e4, 2)
    m, _ = _spd(n, 50.0, 3)
    minv = np.linalg.inv(m)
    b = np.random.default_rng(4).standard_normal(n)
    x_l = krylov.lanczos_alg6(lambda x: a @ x, b, lambda r: minv @ r, t)
    res = krylov.fcg(lambda x: a @ x, b, lambda r: minv @ r, 0.0, t)
    assert res.iterations == t
    # the two differ only by rounding (Lanczos loses orthogonality slowly in FP64)
    assert np.linalg.norm(x_l - res.x) <= 1e-7 * np.linalg.norm(res.x)


def test_alg6_converges_to_solution():
    n = 50
    a, _ = _spd(n, 1e2, 5)
    b = np.random.default_rng(6).standard_normal(n)
    x = krylov.lanczos_alg6(lambda v: a @ v, b, lambda r: r, 150)
    assert np.linalg.norm(a @ x - b) <= 1e-8 * np.linalg.norm(b)


def test_cg_error_bound():
    # |e_t|_A <= 2 ((sqrt k - 1)/(sqrt k + 1))^t |e_0|_A for CG with exact arithmetic
    n, cond = 200, 400.0
    a, _ = _spd(n, cond, 7)
    b = np.random.default_rng(8).standard_normal(n)
    xs = np.linalg.solve(a, b)
    e0 = np.sqrt(xs @ a @ xs)
    rate = (np.sqrt(cond) - 1) / (np.sqrt(cond) + 1)
    for t in (5, 20, 40):
        x = krylov.fcg(lambda v: a @ v, b, lambda r: r, 0.0, t).x
        e = x - xs
        assert np.sqrt(e @ a @ e) <= 2 * rate ** t * e0 * (1 + 1e-8)


def test_zero_rhs_and_breakdown():
    a, _ = _spd(10, 10.0, 9)
    res = krylov.fcg(lambda x: a @ x, np.zeros(10), lambda r: r, 1e-8, 10)
    assert res.status == "zero_rhs" and res.iterations == 0
    res = krylov.fcg(lambda x: -x, np.ones(10), lambda r: r, 1e-8, 10)
    assert res.status == "breakdown"


def test_breakdown_when_the_preconditioned_residual_is_orthogonal():
    # a preconditioner whose output is orthogonal to r makes <r, z> = 0: beta cannot be
    # formed, which is reported as a breakdown after the first step (no exception)
    a, _ = _spd(6, 10.0, 11)
    b = np.array([1.0, 2.0, 0.5, -1.0, 0.25, 3.0])

    def prec(r):  # pairs (r0, r1) -> (r1, -r0): <r, z> = r0 r1 - r1 r0 = 0 exactly
        z = np.empty_like(r)
        z[0::2], z[1::2] = r[1::2], -r[0::2]
        return z

    res = krylov.fcg(lambda x: a @ x, b, prec, 1e-12, 10)
    # the first step takes alpha = <r, z> / <p, A p> = 0, the second cannot form beta
    assert res.status == "breakdown" and res.iterations == 1
    assert not np.any(res.x)
