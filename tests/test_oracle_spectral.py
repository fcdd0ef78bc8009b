"""Pins of the oracle's descending-node Schatten estimator, the Orlicz norm and the Ky Fan norm
(Section 3.2)."""
import math

import numpy as np
import pytest
from scipy.optimize import brentq

from oracle import trace


def _psd(sig, seed):
    """A = Q diag(sig) Q^T with Q from the QR factors of a seeded Gaussian matrix, and the
    exact ridge solve x = Q diag(1/(sig^2 + t)) Q^T G (A^T A = Q diag(sig^2) Q^T)."""
    n = len(sig)
    q, _ = np.linalg.qr(np.random.default_rng(seed).standard_normal((n, n)))
    a = (q * sig) @ q.T
    ridge = lambda t, G: q @ ((q.T @ G) / (sig[:, None] ** 2 + t))
    return a, ridge


def _exact_probes(n):
    # sqrt(n) e_i: the mean over these n probes of g^T f g is tr f exactly
    return math.sqrt(n) * np.eye(n)


def test_lower_tail_weight_is_the_geometric_series():
    p, h, u = 0.7, 1.3, -4.0
    c = h * math.sin(math.pi * p / 2) / math.pi
    direct = sum(c * math.exp(0.5 * p * (u - i * h)) for i in range(1, 4000))
    assert trace.lower_tail_weight(p, h, u) == pytest.approx(direct, rel=1e-13)


@pytest.mark.parametrize("p", [1.0, 0.5, 1.5])
def test_descending_estimate_is_the_schatten_sum(p):
    # exact solves and the exact trace: only the quadrature and the tail replacement remain
    sig = np.geomspace(1e-3, 1.0, 120)
    a, ridge = _psd(sig, 1)
    u_hi = trace.upper_end(1.0, p, eps_q=1e-6)
    est, _, _, used, bound = trace.schatten_descending(a, _exact_probes(len(sig)), p, 0.5, u_hi, ridge, eps_q=1e-6)
    exact = float(np.sum(sig ** p))
    assert abs(est / exact - 1.0) < 1e-5
    assert bound <= 1e-6 * est


def test_descending_tail_bound_holds():
    # the estimate after the early stop differs from a descent taken far lower by at most
    # the bound the stop reports
    sig = np.concatenate([np.geomspace(1e-2, 1.0, 60), np.full(20, 3e-3)])
    a, ridge = _psd(sig, 2)
    g = np.random.default_rng(3).standard_normal((len(sig), 16))
    u_hi = trace.upper_end(1.0, 1.0)
    est, _, per, used, bound = trace.schatten_descending(a, g, 1.0, 1.0, u_hi, ridge, eps_q=1e-3)
    deep, _, per_deep, used_deep, _ = trace.schatten_descending(a, g, 1.0, 1.0, u_hi, ridge, eps_q=1e-14)
    assert used_deep > used
    assert abs(est - deep) <= bound * (1 + 1e-9)
    # per probe as well (the bound is the mean of per-probe bounds)
    assert np.all(per >= per_deep - 1e-12 * np.abs(per_deep))


def test_descending_stops_near_sigma_min():
    # with sigma in [1, 10] the lower end needs t ~ eps sigma_min^2, far above the
    # (eps / n)^2 sigma_max^2 of the range rule that knows only |A|
    n, p, h = 300, 1.0, 1.5
    sig = np.linspace(1.0, 10.0, n)
    a, ridge = _psd(sig, 4)
    u_hi = trace.upper_end(10.0, p)
    est, _, _, used, _ = trace.schatten_descending(a, _exact_probes(n), p, h, u_hi, ridge)
    u_lo_fixed, _ = trace.default_range(10.0, n, p=p)
    fixed_count = int(math.floor((u_hi - u_lo_fixed) / h)) + 1
    assert used < fixed_count - 5
    assert u_hi - (used - 1) * h > math.log(1e-4 * 1.0) - 2 * h
    assert abs(est / sig.sum() - 1.0) < 2e-4


def test_orlicz_of_one_power_is_the_schatten_norm():
    sig = np.geomspace(1e-2, 2.0, 80)
    a, ridge = _psd(sig, 5)
    for p in (1.0, 1.5):
        u_hi = trace.upper_end(2.0, p, eps_q=1e-6)
        r, _, sums, _ = trace.orlicz_estimate(a, _exact_probes(len(sig)), [1.0], [p], 0.5, u_hi, ridge, eps_q=1e-6)
        assert r == pytest.approx(float(np.sum(sig ** p)) ** (1.0 / p), rel=1e-5)
    # g(s) = c s^p: r = (c S_p)^{1/p}
    assert trace.orlicz_from_sums([3.0], [1.2], [5.0]) == pytest.approx((3.0 * 5.0) ** (1 / 1.2), rel=1e-13)


def test_orlicz_root_matches_a_direct_root_on_the_spectrum():
    # g(s) = 0.5 s + 2 s^1.5 on a known spectrum: the root of sum_i g(sigma_i / r) = 1 by
    # Brent's method on the singular values themselves
    sig = np.concatenate([np.geomspace(0.05, 4.0, 50), [7.0, 9.0]])
    coefs, powers = [0.5, 2.0], [1.0, 1.5]
    g = lambda s: 0.5 * s + 2.0 * s ** 1.5
    want = brentq(lambda r: float(np.sum(g(sig / r))) - 1.0, 1e-3, 1e6, xtol=1e-14, rtol=1e-15)
    sums = [float(np.sum(sig ** p)) for p in powers]
    assert trace.orlicz_from_sums(coefs, powers, sums) == pytest.approx(want, rel=1e-12)
    a, ridge = _psd(sig, 6)
    u_hi = trace.upper_end(9.0, 1.5, eps_q=1e-7)
    r, _, _, _ = trace.orlicz_estimate(a, _exact_probes(len(sig)), coefs, powers, 0.5, u_hi, ridge, eps_q=1e-7)
    assert r == pytest.approx(want, rel=1e-5)


def test_orlicz_is_homogeneous():
    # |t A|_g = t |A|_g: the sums scale by t^{p_q}
    coefs, powers = [1.0, 0.3], [1.0, 1.8]
    sums = np.array([4.0, 2.5])
    r1 = trace.orlicz_from_sums(coefs, powers, sums)
    r3 = trace.orlicz_from_sums(coefs, powers, sums * 3.0 ** np.array(powers))
    assert r3 == pytest.approx(3.0 * r1, rel=1e-12)


def test_orlicz_estimate_within_statistical_error():
    n, N = 200, 300
    sig = 1.0 / np.arange(1, n + 1)
    a, ridge = _psd(sig, 7)
    coefs, powers = [1.0, 1.0], [1.0, 1.5]
    g = np.random.default_rng(8).standard_normal((n, N))
    u_hi = trace.upper_end(1.0, 1.5)
    r, se, _, _ = trace.orlicz_estimate(a, g, coefs, powers, 1.0, u_hi, ridge)
    want = brentq(lambda r: float(np.sum(sig / r + (sig / r) ** 1.5)) - 1.0, 1e-3, 1e6, xtol=1e-14)
    assert abs(r - want) <= 4.0 * se


# ---- Ky Fan norms by subspace iteration ----------------------------------------------
def _general(sig, seed, m=None):
    n = len(sig)
    m = m or n
    rng = np.random.default_rng(seed)
    u, _ = np.linalg.qr(rng.standard_normal((m, n)))
    v, _ = np.linalg.qr(rng.standard_normal((n, n)))
    return (u * sig) @ v.T


def test_kyfan_exact_at_rank_within_the_block():
    # rank(A) <= b: the first step's subspace holds range(A^T), so the Ritz values are the
    # singular values
    n, r, b = 120, 10, 16
    rng = np.random.default_rng(11)
    a = rng.standard_normal((n, r)) @ rng.standard_normal((r, n))
    sig = np.linalg.svd(a, compute_uv=False)
    om = rng.standard_normal((n, b))
    for k in (1, 4, 10):
        est, ritz = trace.kyfan_subspace(a, k, b, 1, om)
        assert est == pytest.approx(float(sig[:k].sum()), rel=1e-11)
    assert np.allclose(ritz[:r], sig[:r], rtol=1e-11)


def test_kyfan_ritz_values_interlace():
    # every Ritz value is at most the singular value of the same rank, for any subspace
    sig = np.geomspace(1.0, 1e-3, 80)
    a = _general(sig, 12, m=100)
    om = np.random.default_rng(13).standard_normal((80, 12))
    for q in (0, 1, 3):
        _, ritz = trace.kyfan_subspace(a, 5, 12, q, om)
        assert np.all(ritz <= sig[:12] * (1 + 1e-12))


def test_kyfan_converges_with_a_gap():
    # sigma_{b+1} / sigma_k = 1/2: the top-k Ritz values converge like (1/2)^{2q}
    sig = np.concatenate([np.linspace(10.0, 6.0, 8), np.linspace(2.0, 0.1, 92)])
    a = _general(sig, 14)
    om = np.random.default_rng(15).standard_normal((100, 10))
    want = float(sig[:6].sum())
    errs = [want - trace.kyfan_subspace(a, 6, 10, q, om)[0] for q in (2, 6, 12)]
    assert errs[0] > 0 and errs[2] >= -1e-12 * want
    assert errs[2] < 1e-10 * want and errs[1] < errs[0]


def test_kyfan_one_vector_is_the_power_method():
    # k = b = 1: the estimate is |A x_q| for the normalised power iterate x_q on A^T A
    sig = np.linspace(3.0, 0.5, 50)
    a = _general(sig, 16)
    x = np.random.default_rng(17).standard_normal(50)
    q = 7
    y = x / np.linalg.norm(x)
    for _ in range(q):
        y = a.T @ (a @ y)
        y /= np.linalg.norm(y)
    est, _ = trace.kyfan_subspace(a, 1, 1, q, x[:, None])
    assert est == pytest.approx(float(np.linalg.norm(a @ y)), rel=1e-13)


def test_orthonormal_columns_drops_a_dependent_direction():
    rng = np.random.default_rng(18)
    z = rng.standard_normal((40, 5))
    z[:, 4] = z[:, 0] + z[:, 1]
    qm = trace.orthonormal_columns(z)
    g = qm.T @ qm
    assert np.count_nonzero(np.abs(np.diag(g)) > 0.5) == 4
    assert np.allclose(g[np.ix_(np.diag(g) > 0.5, np.diag(g) > 0.5)], np.eye(4), atol=1e-12)


@pytest.mark.parametrize("p", [0.5, 1.0, 1.5])
def test_upper_end_leaves_at_most_eps_of_the_top_share(p):
    # sigma^p = (sin(pi p / 2) / pi) * integral over u of e^{(p/2) u} sigma^2 / (sigma^2 + e^u):
    # the part above u_hi, integrated directly, is at most eps_q sigma_max^p for every
    # sigma <= sigma_max, and the whole integral is sigma^p
    from scipy.integrate import quad
    smax, eps = 3.0, 1e-4
    u_hi = trace.upper_end(smax, p, eps_q=eps)
    c = math.sin(math.pi * p / 2) / math.pi
    f = lambda u, sig: c * math.exp(0.5 * p * u) * sig * sig / (sig * sig + math.exp(u))
    for sig in (smax, 0.3 * smax, 1e-2 * smax):
        tail, _ = quad(f, u_hi, u_hi + 400.0, args=(sig,), limit=400)
        assert tail <= eps * smax ** p
        whole = sum(quad(f, a, a + 10.0, args=(sig,), limit=200)[0] for a in np.arange(-200.0, u_hi + 400.0, 10.0))
        assert whole == pytest.approx(sig ** p, rel=1e-7)
    # tight to within the factor sin(pi p / 2) / (pi (1 - p / 2)) at sigma = sigma_max
    tail, _ = quad(f, u_hi, u_hi + 400.0, args=(smax,), limit=400)
    assert tail >= 0.5 * eps * smax ** p * c / (1 - p / 2)
