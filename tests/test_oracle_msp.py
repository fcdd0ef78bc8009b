"""Pins of the oracle's MSP (Algorithms 1-5) against what the paper and linear algebra fix."""
import numpy as np
import pytest

import workloads as W
from oracle import dense, krylov, msp


@pytest.fixture(scope="module")
def psd_small():
    n, k = 512, 16
    a, eigs, q = W.psd_outlier(n, k, config_id=100)
    b = W.gaussian(n, 100)
    return a, eigs, b


def _psd(a, eigs, lam=1e-3, s=32, lam0=None, l=None, **kw):
    l = s // 2 if l is None else l
    if lam0 is None:
        lam0 = msp.paper_lambda0(eigs, l)
    o = msp.MspOptions(**kw)
    return msp.PsdMsp(a, lam, lam0, s, 8, 17, 4 * s, 8, 25, o)


def test_paper_lambda0_formula():
    e = np.array([10.0, 5.0, 3.0, 2.0, 1.0])
    assert msp.paper_lambda0(e, 2) == pytest.approx(2.0 / 2 * (3 + 2 + 1))


def test_lambda0_from_trace_and_top_eigenvalues():
    e = np.sort(np.random.default_rng(2).uniform(0, 10, 50))[::-1]
    assert msp.paper_lambda0_from_top(e.sum(), e[:7][::-1], 7) == pytest.approx(msp.paper_lambda0(e, 7), rel=1e-12)


def test_nystrom_exact_recovery_low_rank():
    # Section 4.2: A_nys = A S^T (S A S^T)^+ S A equals A when rank(A) <= s.
    n, r, s = 300, 20, 32
    g = np.random.default_rng(3).standard_normal((n, r))
    a = g @ g.T
    P = msp.PsdMsp(a, 1e-2, 0.0, s, 8, 5, 4 * s, 8, 6)
    wp = np.linalg.pinv(P.w, rcond=1e-12, hermitian=True)
    assert np.linalg.norm(a - P.c @ wp @ P.c.T) <= 1e-10 * np.linalg.norm(a)


def test_nystrom_is_below_a_and_within_lambda0(psd_small):
    # A_nys <= A (Loewner order) and |A - A_nys| <= lam0 (Section 4.2). The second
    # holds w.h.p. once s = O(l log(l / delta)); it is checked at s = 4 l.
    a, eigs, _ = psd_small
    P = _psd(a, eigs, s=64, l=16)
    wp = np.linalg.pinv(P.w, rcond=1e-13, hermitian=True)
    d = a - P.c @ wp @ P.c.T
    ev = np.linalg.eigvalsh(0.5 * (d + d.T))
    assert ev.min() >= -1e-9 * eigs[0]
    assert ev.max() <= P.lam0


def test_kappa_m_bound(psd_small):
    # kappa(M^{-1/2}(A + lam I)M^{-1/2}) <= 1 + lam0 / (lambda_n + lam)
    a, eigs, _ = psd_small
    lam = 1e-3
    P = _psd(a, eigs, lam=lam, s=64, l=16)
    minv = P.m_inverse_dense()
    ev = np.linalg.eigvals(minv @ (a + lam * np.eye(a.shape[0]))).real
    kappa = ev.max() / ev.min()
    assert kappa <= 1 + P.lam0 / (eigs[-1] + lam) + 1e-6


def test_m_inverse_identity(psd_small):
    # eq. M_inverse: (C W^{-1} C^T + lam~ I)^{-1} r = (r - C (C^T C + lam~ W)^{-1} C^T r) / lam~
    a, eigs, _ = psd_small
    P = _psd(a, eigs, inner_tol=1e-15, max_inner=500)
    r = np.random.default_rng(9).standard_normal(a.shape[0])
    w_hat = P.solve_m1(r)
    want = P.m_inverse_dense() @ r
    assert np.linalg.norm(w_hat - want) <= 1e-9 * np.linalg.norm(want)


def test_level2_preconditioner_quality(psd_small):
    # Lemma 2.2 with eps = 1/2: kappa(M2^{-1} (C^T C + lam~ W)) <= ((1+eps)/(1-eps))^2 = 9
    a, eigs, _ = psd_small
    P = _psd(a, eigs)
    op = P.c.T @ P.c + P.lt * P.w
    ev = np.linalg.eigvals(P.m2inv @ op).real
    assert ev.max() / ev.min() <= 9.0


def test_psd_solve_matches_dense(psd_small):
    a, eigs, b = psd_small
    P = _psd(a, eigs, tol=1e-10, inner_tol=1e-12)
    res = P.solve(b)
    xs = dense.solve_psd(a, b, 1e-3)
    assert res.status == "converged"
    assert P.info.rel_residual <= 1e-10
    assert np.linalg.norm(res.x - xs) <= 1e-8 * np.linalg.norm(xs)


def test_psd_preconditioning_beats_plain_cg(psd_small):
    a, eigs, b = psd_small
    P = _psd(a, eigs, tol=1e-10, inner_tol=1e-12)
    its = P.solve(b).iterations
    cg = krylov.fcg(lambda x: a @ x + 1e-3 * x, b, lambda r: r, 1e-10, 5000).iterations
    assert its < cg


def test_rank_below_l_converges_in_one_iteration():
    # rank(A) <= l gives lam0 = 0 and exact Nystrom recovery, so M = A + lam I and the
    # preconditioned iteration ends after one step. A is made numerically rank r
    # (plus 1e-8 I) so that W is definite and the level-2 solve is well posed.
    n, r, s = 256, 10, 32
    g = np.random.default_rng(4).standard_normal((n, r))
    a = g @ g.T + 1e-8 * np.eye(n)
    eigs = np.linalg.eigvalsh(a)[::-1]
    lam0 = msp.paper_lambda0(eigs, s // 2)
    assert lam0 < 1e-6
    P = msp.PsdMsp(a, 1e-1, lam0, s, 8, 2, 4 * s, 8, 3,
                   msp.MspOptions(tol=1e-6, inner_tol=1e-13, max_inner=400))
    b = np.random.default_rng(5).standard_normal(n)
    res = P.solve(b)
    assert res.iterations == 1 and res.status == "converged"


def test_huge_regulariser_reduces_to_plain_cg(psd_small):
    # lam~ >> |A| makes M ~= lam~ I; a scalar preconditioner leaves CG unchanged.
    a, eigs, b = psd_small
    P = _psd(a, eigs, lam0=1e9 * eigs[0], tol=1e-8, inner_tol=1e-13)
    its = P.solve(b).iterations
    cg = krylov.fcg(lambda x: a @ x + 1e-3 * x, b, lambda r: r, 1e-8, 5000).iterations
    assert abs(its - cg) <= 1


# ------------------------------ general (three-level) ------------------------------
def _general(a, lam, lam0, s, **kw):
    return msp.GeneralMsp(a, lam, lam0, s, 8, 41, 4 * s, 8, 43, msp.MspOptions(**kw))


def test_level3_identity():
    # (W^2 + lam~ W)^{-1} = W^{-1} (W + lam~ I)^{-1} = (W^{-1} - (W + lam~ I)^{-1}) / lam~
    a, sv, _, _ = W.general_outlier(200, 6, config_id=101, big=(1e1, 1e2))
    lam0 = msp.paper_lambda0(sv ** 2, 8)
    r = np.random.default_rng(1).standard_normal(16)
    outs = []
    for form in ("product", "difference"):
        P = _general(a, 0.0, lam0, 16, level3_tol=1e-15, max_level3=500, m2_form=form)
        outs.append(P.solve_m2(r))
    wm = P.at.T @ P.at
    want = np.linalg.solve(wm @ wm + P.lt * wm, r)
    for z in outs:
        assert np.linalg.norm(z - want) <= 1e-8 * np.linalg.norm(want)


def test_w_squared_factorisation():
    # W^2 + lam~ W = A~^T (A~ A~^T + lam~ I) A~  (Section 5)
    a, sv, _, _ = W.general_outlier(120, 4, config_id=102)
    P = _general(a, 0.0, 3.0, 16)
    wm = P.at.T @ P.at
    rhs = P.at.T @ (P.at @ P.at.T + P.lt * np.eye(120)) @ P.at
    assert np.allclose(wm @ wm + P.lt * wm, rhs, rtol=1e-12, atol=1e-9 * np.abs(rhs).max())


def test_general_solve_matches_lu():
    n, k, s = 400, 12, 32
    a, sv, _, _ = W.general_outlier(n, k, config_id=103, big=(1e2, 1e4))
    lam0 = msp.paper_lambda0(np.sort(sv)[::-1] ** 2, s // 2)
    b = W.gaussian(n, 103)
    P = _general(a, 0.0, lam0, s, tol=1e-10, inner_tol=1e-12, level3_tol=1e-12)
    res = P.solve_system(b)
    xs = dense.solve_general(a, b)
    assert res.status == "converged"
    assert P.info.rel_residual <= 1e-10
    assert np.linalg.norm(res.x - xs) <= 1e-7 * np.linalg.norm(xs)


def test_general_lower_bound_example_one():
    # Section 7: A = I + e_i e_j^T - e_j e_i^T, b = 1 has x = 1 except x_i = 0.
    n, i, j, s = 64, 5, 40, 16
    a = np.eye(n)
    a[i, j] += 1.0
    a[j, i] -= 1.0
    sv = np.array([np.sqrt(2.0)] * 2 + [1.0] * (n - 2))
    lam0 = msp.paper_lambda0(sv ** 2, s // 2)
    P = _general(a, 0.0, lam0, s, tol=1e-12, inner_tol=1e-13, level3_tol=1e-13)
    res = P.solve_system(np.ones(n))
    want = np.ones(n)
    want[i] = 0.0
    assert np.abs(res.x - want).max() <= 1e-10


def test_general_lower_bound_example_two():
    # Section 7: blockdiag(M, sigma_min(M) I) [x; y] = [c; 0] has y = 0, x = M^{-1} c.
    k, n, s = 8, 96, 32
    r = np.random.default_rng(7).standard_normal((k, k))
    m = r + 3 * np.eye(k)
    smin = np.linalg.svd(m, compute_uv=False).min()
    a = np.zeros((n, n))
    a[:k, :k] = m
    a[k:, k:] = smin * np.eye(n - k)
    b = np.zeros(n)
    b[:k] = np.random.default_rng(8).standard_normal(k)
    sv = np.sort(np.linalg.svd(a, compute_uv=False))[::-1]
    lam0 = msp.paper_lambda0(sv ** 2, s // 2)
    P = _general(a, 0.0, lam0, s, tol=1e-12, inner_tol=1e-13, level3_tol=1e-13)
    res = P.solve_system(b)
    assert np.abs(res.x[k:]).max() <= 1e-10 * np.linalg.norm(b)
    assert np.linalg.norm(res.x[:k] - np.linalg.solve(m, b[:k])) <= 1e-9 * np.linalg.norm(b)


def test_general_ridge_normal_equations():
    # (A^T A + lam I) x = c against the SVD route
    n, s = 200, 32
    a, sv, _, _ = W.general_outlier(n, 6, config_id=104, big=(1e1, 1e3))
    lam = 0.5
    lam0 = msp.paper_lambda0(np.sort(sv)[::-1] ** 2, s // 2)
    c = W.gaussian(n, 104)
    P = _general(a, lam, lam0, s, tol=1e-11, inner_tol=1e-12, level3_tol=1e-12)
    res = P.solve_normal(c)
    xs = dense.solve_ridge(a, c, lam)
    assert np.linalg.norm(res.x - xs) <= 1e-8 * np.linalg.norm(xs)


def test_level3_preconditioner_quality():
    # Section 5: A^ = Phi A~ embeds the column space of A~ (phi = 4s rows), so M3a = A^T A^
    # and M3b = M3a + lam~ I are within a constant of W = A~^T A~ and W + lam~ I:
    # kappa(M3a^{-1} W), kappa(M3b^{-1} (W + lam~ I)) <= ((1+eps)/(1-eps))^2 = 9 at eps = 1/2
    a, sv, _, _ = W.general_outlier(400, 12, config_id=104, big=(1e2, 1e4))
    lam0 = msp.paper_lambda0(np.sort(sv)[::-1] ** 2, 16)
    P = _general(a, 0.0, lam0, 32)
    wm = P.at.T @ P.at
    for minv, op in ((P.m3a_inv, wm), (P.m3b_inv, wm + P.lt * np.eye(32))):
        ev = np.linalg.eigvals(minv @ op).real
        assert ev.min() > 0 and ev.max() / ev.min() <= 9.0


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_effective_dimension_bound_at_lambda0(seed):
    # with the paper's lam0 = (2/l) sum_{i>l} lambda_i: d_lam0 = sum_i lambda_i/(lambda_i + lam0)
    # <= l (the top l terms) + sum_{i>l} lambda_i / lam0 = l + l/2
    r = np.random.default_rng(seed)
    for l in (4, 16, 64):
        eigs = np.sort(np.concatenate([10.0 ** r.uniform(1, 6, size=l // 2), r.uniform(0, 1, size=500)]))[::-1]
        lam0 = msp.paper_lambda0(eigs, l)
        d = dense.effective_dimension(eigs, lam0)
        assert d <= 1.5 * l + 1e-9


@pytest.mark.parametrize("seed", [3, 4])
def test_effective_dimension_lemma(seed):
    # Lemma 2.1: (1) j >= (1 + 1/g) d_lam implies lambda_j <= g lam; (2) k >= d_lam implies
    # sum_{i>k} lambda_i <= lam d_lam (eigenvalues non-increasing, indices from 1)
    r = np.random.default_rng(seed)
    eigs = np.sort(np.concatenate([10.0 ** r.uniform(0, 5, size=40), r.uniform(0, 1e-1, size=400)]))[::-1]
    for lam in (1e-3, 1e-1, 10.0):
        d = dense.effective_dimension(eigs, lam)
        for g in (0.25, 1.0, 4.0):
            j = int(np.ceil((1 + 1 / g) * d))
            if j <= eigs.size:
                assert eigs[j - 1] <= g * lam * (1 + 1e-12)
        k = int(np.ceil(d))
        assert eigs[k:].sum() <= lam * d * (1 + 1e-12)


# ---- the lam0 estimator (the trace deficit of the Nystrom approximation) -------------
def _est(a, s, seed=17):
    P = msp.PsdMsp(a, 1e-2, 1.0, s, 8, seed, 4 * s, 8, seed + 8)
    return P, msp.lambda0_estimate(a, P.c, P.w, s // 2)


@pytest.mark.parametrize("cid,k", [(100, 16), (101, 40), (102, 4)])
def test_lambda0_estimate_bounds_the_tail_beyond_s(cid, k):
    # A - C W^+ C^T is PSD and C W^+ C^T has rank <= s, so by Weyl's inequality the deficit
    # is at least the sum of the eigenvalues after the s-th
    n, s = 400, 32
    a, eigs, _ = W.psd_outlier(n, k, config_id=cid)
    _, est = _est(a, s)
    tail_s = float(np.sort(eigs)[::-1][s:].sum())
    assert est >= 2.0 / (s // 2) * tail_s * (1 - 1e-10)
    assert est <= 2.0 / (s // 2) * float(np.trace(a))


@pytest.mark.parametrize("seed", [17, 5, 9])
def test_lambda0_estimate_exact_at_low_rank(seed):
    # rank(A) <= s: the sketch recovers A exactly (Section 4.2), so the deficit is 0; the
    # regularised W^+ leaves a bias of a few 1e-8 tr(A) here, below the 1e-6 tr(A) cut
    n, r, s = 300, 20, 32
    g = np.random.default_rng(3).standard_normal((n, r))
    a = g @ g.T
    _, est = _est(a, s, seed)
    assert est == 0.0


def test_lambda0_estimate_equals_the_dense_trace_deficit():
    # the same deficit through the dense n x n approximation and its trace, with W^+ from
    # the eigendecomposition (the estimator's (W + mu I)^{-1} differs by O(mu))
    n, s = 300, 24
    a, eigs, _ = W.psd_outlier(n, 10, config_id=103)
    P, est = _est(a, s)
    nys = P.c @ np.linalg.pinv(P.w, rcond=1e-12, hermitian=True) @ P.c.T
    want = 2.0 / (s // 2) * (np.trace(a) - np.trace(nys))
    assert est == pytest.approx(want, rel=1e-6)


def test_lambda0_estimate_is_invariant_to_the_sketch_scale():
    # C = A S^T and W = S A S^T: scaling S by t scales C by t and W by t^2, so
    # tr(W^+ C^T C) does not change (the +-1/sqrt(gamma) scale of Definition 2.1 is immaterial)
    n, s = 300, 24
    a, _, _ = W.psd_outlier(n, 10, config_id=104)
    P, est = _est(a, s)
    assert msp.lambda0_estimate(a, 2.0 * P.c, 4.0 * P.w, s // 2) == pytest.approx(est, rel=1e-10)


def test_lambda0_estimate_against_the_paper_value_on_an_rbf_matrix():
    # RBF spectrum (fast decay): the estimator lies between the tail beyond s and the
    # tail beyond l = s/2 times a small factor; recorded here as a trend, not a bound
    pts = W.rbf_points(1024, 8, 7)
    a = W.rbf_matrix(pts)
    s = 64
    eigs = np.linalg.eigvalsh(a)[::-1]
    _, est = _est(a, s)
    paper = msp.paper_lambda0(eigs, s // 2)
    assert 2.0 / (s // 2) * eigs[s:].sum() <= est <= 3.0 * paper


def test_spd_inverse_is_the_shifted_inverse():
    # (M + mu I)^{-1} with mu = shift_rel tr(M) / d: against numpy's inverse of the shifted
    # matrix, symmetric, and with shift_rel = 0 an exact inverse to kappa * eps
    rng = np.random.default_rng(31)
    q, _ = np.linalg.qr(rng.standard_normal((40, 40)))
    for spread in (1e2, 1e8):
        ev = np.geomspace(1.0, spread, 40)
        m = (q * ev) @ q.T
        m = 0.5 * (m + m.T)
        for shift_rel in (0.0, 1e-3):
            mu = shift_rel * float(np.trace(m)) / 40
            got = msp.spd_inverse(m, shift_rel)
            want = np.linalg.inv(m + mu * np.eye(40))
            assert np.array_equal(got, got.T)
            kappa = (spread + mu) / (1.0 + mu)
            assert np.linalg.norm(got - want) <= 100 * kappa * np.finfo(float).eps * np.linalg.norm(want)
            assert np.linalg.norm(got @ (m + mu * np.eye(40)) - np.eye(40)) <= 100 * kappa * np.finfo(float).eps * 40
