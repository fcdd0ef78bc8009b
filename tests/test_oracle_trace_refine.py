"""Pins of the oracle's spectral-sum estimator, mixed-precision refinement and gradients."""
import math

import numpy as np
import pytest
import torch

import workloads as W
from oracle import dense, msp, refine, trace


# ------------------------------------------------------------------ quadrature (R14)
@pytest.mark.parametrize("p", [1.0, 0.5, 1.5])
def test_quadrature_reproduces_sigma_power(p):
    # sum_j w_j s^2/(s^2 + t_j) ~= s^p over the range the u-interval covers
    sig = np.geomspace(1e-4, 1.0, 50)
    u_lo, u_hi = trace.default_range(1.0, 10 ** 4, p=p, eps_q=1e-6)
    nodes, w = trace.quadrature(p, 0.5, u_lo, u_hi)
    got = trace.quadrature_scalar(sig, p, nodes, w)
    assert np.max(np.abs(got / sig ** p - 1.0)) < 1e-4


def test_schatten1_harmonic_quadrature_only():
    # sigma_i = 1/i: the quadrature on the exact spectrum recovers H_n
    n = 16384
    sig = 1.0 / np.arange(1, n + 1)
    u_lo, u_hi = trace.default_range(1.0, n)
    nodes, w = trace.quadrature(1.0, 1.5, u_lo, u_hi)
    est = trace.quadrature_scalar(sig, 1.0, nodes, w).sum()
    exact = dense.schatten_p(sig, 1.0)
    # H_n = ln n + Euler-gamma + 1/(2n) - 1/(12 n^2) + O(n^-4) = 10.2813067100084...
    h_n = math.log(n) + 0.5772156649015329 + 1 / (2 * n) - 1 / (12 * n * n)
    assert abs(exact - h_n) < 1e-12
    assert abs(est / exact - 1.0) < 1e-4


def test_per_probe_value_equals_gAg_for_psd():
    # For PSD A, (A^T A)^{1/2} = A, so each probe's full-quadrature value -> g^T A g
    n = 200
    a, sig, qv = W.schatten_psd(n, config_id=200)
    g = W.gaussian((n, 6), 200)
    u_lo, u_hi = trace.default_range(1.0, n, eps_q=1e-6)
    nodes, w = trace.quadrature(1.0, 0.5, u_lo, u_hi)
    ridge = lambda t, G: np.linalg.solve(a.T @ a + t * np.eye(n), G)
    est, se, per = trace.schatten_estimate(a, g, 1.0, nodes, w, ridge)
    want = np.einsum("ik,ij,jk->k", g, a, g)
    assert np.max(np.abs(per - want) / np.abs(want).max()) < 1e-5


def test_schatten_estimate_within_statistical_error():
    n, N = 300, 400
    a, sig, _ = W.schatten_psd(n, config_id=201)
    g = W.gaussian((n, N), 201)
    u_lo, u_hi = trace.default_range(1.0, n)
    nodes, w = trace.quadrature(1.0, 1.0, u_lo, u_hi)
    ridge = lambda t, G: np.linalg.solve(a.T @ a + t * np.eye(n), G)
    est, se, _ = trace.schatten_estimate(a, g, 1.0, nodes, w, ridge)
    exact = dense.schatten_p(sig, 1.0)
    sd = math.sqrt(2.0 * np.sum(sig ** 2) / N)   # Hutchinson sd for PSD: sqrt(2 |A|_F^2 / N)
    assert abs(est - exact) < 4 * sd


def test_effective_dimension_estimate():
    n, N, lam = 256, 300, 0.05
    a, eigs, _ = W.psd_outlier(n, 8, config_id=202)
    g = W.gaussian((n, N), 202)
    est, per = trace.effective_dimension_estimate(g, lam, lambda G: dense.solve_psd(a, G, lam))
    d = dense.effective_dimension(eigs, lam)
    sd = math.sqrt(2.0 * np.sum((eigs / (eigs + lam)) ** 2) / N)
    assert abs(est - d) < 4 * sd
    # closed form for one probe: g^T Q diag(e/(e+lam)) Q^T g
    _, _, q = W.psd_outlier(n, 8, config_id=202)
    z = q.T @ g[:, 0]
    assert per[0] == pytest.approx(np.sum(z * z * eigs / (eigs + lam)), rel=1e-10)


# ------------------------------------------------------------------ rounding and IR (R17)
def test_bf16_rounding_matches_torch():
    x = np.random.default_rng(0).standard_normal(10000) * np.geomspace(1e-30, 1e30, 10000)
    ours = refine.round_bf16(x)
    ref = torch.from_numpy(x.astype(np.float32)).to(torch.bfloat16).to(torch.float32).numpy()
    assert np.array_equal(ours, ref)


def test_refinement_reaches_fp64_accuracy_from_f32_inner():
    n, lam = 512, 1e-3
    a, eigs, _ = W.psd_outlier(n, 16, config_id=203)
    b = W.gaussian(n, 203)
    a_lo = refine.round_f32(a).astype(np.float64)
    inner = msp.PsdMsp(a_lo, lam, msp.paper_lambda0(eigs, 16), 32, 8, 1, 128, 8, 2,
                       msp.MspOptions(tol=1e-6, inner_tol=1e-8))
    x, info = refine.refine(lambda v: a @ v + lam * v, b, lambda r: inner.solve(r).x, 1e-12)
    assert info.status == "converged" and not info.krylov
    assert dense.rel_residual_psd(a, x, b, lam) <= 1e-12


def test_refinement_switches_to_krylov_when_stagnating():
    # a correction solve that only ever removes ~10% of the error makes plain IR stall
    n, lam = 64, 1.0
    a, _, _ = W.psd_outlier(n, 4, config_id=204)
    b = W.gaussian(n, 204)
    bad = lambda r: 0.1 * dense.solve_psd(a, r, lam)
    x, info = refine.refine(lambda v: a @ v + lam * v, b, bad, 1e-10)
    assert info.krylov and info.status == "converged"
    assert dense.rel_residual_psd(a, x, b, lam) <= 1e-10


# ------------------------------------------------------------------ gradients
def test_dense_gradients_by_finite_differences():
    n, k, lam = 12, 3, 0.7
    r = np.random.default_rng(3)
    m = r.standard_normal((n, n))
    a = m @ m.T
    bm = r.standard_normal((n, k))
    loss = lambda a_, b_, l_: float(np.sum(np.linalg.solve(a_ + l_ * np.eye(n), b_) ** 2))
    x = np.linalg.solve(a + lam * np.eye(n), bm)
    db, da, dl = dense.gradients(a, lam, x, 2.0 * x)
    h = 1e-6
    fd_l = (loss(a, bm, lam + h) - loss(a, bm, lam - h)) / (2 * h)
    assert dl == pytest.approx(fd_l, rel=1e-6)
    e = np.zeros_like(bm)
    e[4, 1] = h
    assert db[4, 1] == pytest.approx((loss(a, bm + e, lam) - loss(a, bm - e, lam)) / (2 * h), rel=1e-6)
    ea = np.zeros_like(a)
    ea[2, 7] = h
    assert da[2, 7] == pytest.approx((loss(a + ea, bm, lam) - loss(a - ea, bm, lam)) / (2 * h), rel=1e-5)


@pytest.mark.parametrize("dt,u", [(torch.bfloat16, 2.0 ** -8), (torch.float32, 2.0 ** -24)])
def test_rounding_shift_dominates_the_perturbation(dt, u):
    # The inner shift of refinement over low-precision sweeps: elementwise round-to-
    # nearest of a symmetric A gives a symmetric E = A_lo - A_hi with |E_ij| <= u |A_ij|,
    # so ||E||_2 <= ||E||_inf <= u ||A||_inf and A_lo + u ||A||_inf I - A_hi is PSD.
    import workloads as W
    for cid, n in ((61, 120), (62, 300)):
        a = W.rbf_matrix(W.rbf_points(n, 4, cid), lengthscale=1.5)
        lo = torch.from_numpy(a).to(dt).double().numpy()
        e = lo - a
        assert np.array_equal(e, e.T)
        delta = u * np.abs(a).sum(axis=1).max()
        assert np.linalg.norm(e, 2) <= delta
        assert np.linalg.eigvalsh(e + delta * np.eye(n)).min() >= -1e-12 * delta
