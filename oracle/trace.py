"""Spectral sums through ridge solves (Section 3.2), oracle side.

The paper uses the Schatten-norm meta-algorithm of Musco et al. as a black box that
needs ridge solves (A^T A + t I)^{-1} g. The reading made concrete here:

  ||A||_p^p = tr((A^T A)^{p/2})
            = (sin(pi p / 2) / pi) int_0^inf t^{p/2 - 1} tr(A^T A (A^T A + t I)^{-1}) dt,

valid for 0 < p < 2 (the scalar identity int_0^inf t^{a-1} / (1 + t) dt = pi / sin(pi a)
with a = p/2). With t = e^u the integrand decays exponentially at both ends, so the
trapezoidal rule with step h on [u_lo, u_hi] converges exponentially (Trefethen and
Weideman 2014). The trace is estimated with Hutchinson's estimator over N Gaussian
probes g_k (Section 1.1): the per-probe value at node t_j is <A g_k, A x_jk> with
x_jk = (A^T A + t_j I)^{-1} g_k.

The effective dimension d_lam = tr(A (A + lam I)^{-1}) (Section 2) is estimated the
same way with PSD solves: g^T A x = g^T g - lam g^T x for x = (A + lam I)^{-1} g.
"""
from __future__ import annotations

import math

import numpy as np


def quadrature(p: float, h: float, u_lo: float, u_hi: float):
    """Nodes t_j = exp(u_j), u_j = u_lo + j h (j = 0..J-1, u_j <= u_hi), and weights
    w_j = h sin(pi p/2)/pi exp((p/2) u_j)."""
    if not (0.0 < p < 2.0):
        raise ValueError("0 < p < 2")
    count = int(math.floor((u_hi - u_lo) / h + 1e-9)) + 1
    u = u_lo + h * np.arange(count)
    w = h * math.sin(math.pi * p / 2.0) / math.pi * np.exp(0.5 * p * u)
    return np.exp(u), w


def quadrature_scalar(sigma, p, nodes, weights):
    """The quadrature applied to one singular value: sum_j w_j s^2 / (s^2 + t_j)."""
    s2 = np.asarray(sigma, dtype=np.float64) ** 2
    return (weights[None, :] * (s2[:, None] / (s2[:, None] + nodes[None, :]))).sum(axis=1)


def default_range(sigma_max: float, n: int, p: float = 1.0, eps_q: float = 1e-4):
    """u-range from an estimate of |A|. The integrand behaves like e^{(p/2) u} below
    the spectrum and like e^{(p/2 - 1) u} above it, so
    u_lo = 2 ln sigma_max + (2/p) ln(eps_q / n) and u_hi = 2 ln sigma_max + (2/(2-p)) ln(1/eps_q)
    (for p = 1: 2 ln(eps_q sigma_max / n) and 2 ln(sigma_max / eps_q))."""
    ls = 2.0 * math.log(sigma_max)
    return ls + (2.0 / p) * math.log(eps_q / n), ls + (2.0 / (2.0 - p)) * math.log(1.0 / eps_q)


def schatten_estimate(a, probes, p, nodes, weights, ridge_solve):
    """Hutchinson + quadrature estimate of ||A||_p^p.

    ridge_solve(t, G) returns X ~= (A^T A + t I)^{-1} G for the probe block G (n x N).
    Returns (estimate, standard error over probes, per-probe values)."""
    g = np.asarray(probes, dtype=np.float64)
    ag = a @ g
    per_probe = np.zeros(g.shape[1])
    for t, w in zip(nodes, weights):
        x = ridge_solve(t, g)
        per_probe += w * np.sum(ag * (a @ x), axis=0)
    est = float(per_probe.mean())
    se = float(per_probe.std(ddof=1) / math.sqrt(g.shape[1])) if g.shape[1] > 1 else float("nan")
    return est, se, per_probe


def effective_dimension_estimate(probes, lam, psd_solve):
    """Hutchinson estimate of d_lam; psd_solve(G) ~= (A + lam I)^{-1} G."""
    g = np.asarray(probes, dtype=np.float64)
    x = psd_solve(g)
    per = np.sum(g * g, axis=0) - lam * np.sum(g * x, axis=0)
    return float(per.mean()), per


# ---------------------------------------------------------------------------------
# Nodes taken from the top down with a bounded lower tail (reading of Section 3.2's
# range: the paper leaves the quadrature range to the black box)
# ---------------------------------------------------------------------------------
# Per probe g and node t the ridge value is T(t) = <A g, A x>, x = (A^T A + t I)^{-1} g, and
# (A^T A + t I) x = g gives T(t) = g^T g - d(t) with the deficit d(t) = t g^T x =
# sum_i c_i^2 t / (sigma_i^2 + t) (c = V^T g), which is nondecreasing in t. Going down the
# grid u_j = u_hi - j h, every node below u_j has d <= d(t_j), so replacing T by its t -> 0
# limit g^T g at all of them (down to -infinity, a geometric series of trapezoid weights)
# changes that probe's value by at most d(t_j) W_below(j), W_below(j) = sum_{i>j} w_i. The
# descent stops when the mean of that bound over the probes is at most eps_q |estimate|.
def lower_tail_weight(p: float, h: float, u_j: float) -> float:
    """sum over the grid nodes u_j - h, u_j - 2h, ... of h sin(pi p/2)/pi e^{(p/2) u}."""
    c = h * math.sin(math.pi * p / 2.0) / math.pi
    return c * math.exp(0.5 * p * (u_j - h)) / (1.0 - math.exp(-0.5 * p * h))


def schatten_descending(a, probes, p, h, u_hi, ridge_solve, eps_q=1e-4, max_nodes=400):
    """||A||_p^p by Hutchinson and the trapezoid rule on nodes u_hi, u_hi - h, ... with the
    lower tail replaced by g^T g once its bound is below eps_q of the estimate.

    ridge_solve(t, G) ~= (A^T A + t I)^{-1} G. Returns (estimate, standard error, per-probe
    values, nodes used, the final tail bound)."""
    if not (0.0 < p < 2.0):
        raise ValueError("0 < p < 2")
    g = np.asarray(probes, dtype=np.float64)
    ag = a @ g
    gg = np.sum(g * g, axis=0)
    c = h * math.sin(math.pi * p / 2.0) / math.pi
    acc = np.zeros(g.shape[1])
    used = 0
    bound = float("inf")
    per = acc
    for j in range(max_nodes):
        u = u_hi - j * h
        t = math.exp(u)
        x = ridge_solve(t, g)
        acc = acc + c * math.exp(0.5 * p * u) * np.sum(ag * (a @ x), axis=0)
        d = t * np.sum(g * x, axis=0)
        wb = lower_tail_weight(p, h, u)
        per = acc + wb * gg
        used = j + 1
        bound = float(np.mean(np.abs(d)) * wb)
        if bound <= eps_q * abs(float(per.mean())):
            break
    est = float(per.mean())
    se = float(per.std(ddof=1) / math.sqrt(g.shape[1])) if g.shape[1] > 1 else float("nan")
    return est, se, per, used, bound


def upper_end(sigma_max: float, p: float, eps_q: float = 1e-4) -> float:
    """u_hi = 2 ln sigma_max + (2/(2-p)) ln(1/eps_q): above it the integrand is below
    e^{(p/2-1)u} sigma_max^2, whose tail is eps_q of the top singular value's share."""
    return 2.0 * math.log(sigma_max) + (2.0 / (2.0 - p)) * math.log(1.0 / eps_q)


# ---------------------------------------------------------------------------------
# Orlicz norms (Section 3.2: the spectral-sum meta-algorithm also gives Orlicz norms)
# ---------------------------------------------------------------------------------
# For an Orlicz function g (convex, increasing, g(0) = 0) the Orlicz norm of A is
# |A|_g = inf {r > 0 : sum_i g(sigma_i / r) <= 1}. The functions handled are positive
# combinations of powers, g(s) = sum_q c_q s^{p_q} with c_q > 0 and 0 < p_q < 2 (convex
# when every p_q >= 1): then sum_i g(sigma_i / r) = sum_q c_q r^{-p_q} ||A||_{p_q}^{p_q}, and
# every Schatten sum comes from the same ridge solves (the nodes of the quadrature do not
# depend on p, only the weights do). The left side is strictly decreasing in r, so the
# root is unique; it is found by bisection on ln r.
def orlicz_from_sums(coefs, powers, sums, tol=1e-15):
    """The root r of sum_q c_q r^{-p_q} S_q = 1 (S_q = sum_i sigma_i^{p_q} > 0)."""
    coefs = np.asarray(coefs, dtype=np.float64)
    powers = np.asarray(powers, dtype=np.float64)
    sums = np.asarray(sums, dtype=np.float64)
    phi = lambda lr: float(np.sum(coefs * sums * np.exp(-powers * lr))) - 1.0
    lo, hi = -1.0, 1.0
    while phi(lo) < 0.0:
        lo -= 2.0 * (hi - lo)
    while phi(hi) > 0.0:
        hi += 2.0 * (hi - lo)
    for _ in range(400):
        mid = 0.5 * (lo + hi)
        if phi(mid) > 0.0:
            lo = mid
        else:
            hi = mid
        if hi - lo <= tol * max(1.0, abs(mid)):
            break
    return math.exp(0.5 * (lo + hi))


def orlicz_estimate(a, probes, coefs, powers, h, u_hi, ridge_solve, eps_q=1e-4, max_nodes=400):
    """|A|_g for g(s) = sum_q c_q s^{p_q}: every ||A||_{p_q}^{p_q} by the descending-node
    estimator on one shared grid (the descent stops when every sum's tail bound is below
    eps_q of that sum), then the root. Returns (estimate, standard error by the delta
    method, the Schatten sums, nodes used)."""
    g = np.asarray(probes, dtype=np.float64)
    coefs = np.asarray(coefs, dtype=np.float64)
    powers = np.asarray(powers, dtype=np.float64)
    ag = a @ g
    gg = np.sum(g * g, axis=0)
    Q, N = len(powers), g.shape[1]
    acc = np.zeros((Q, N))
    per = acc
    used = 0
    for j in range(max_nodes):
        u = u_hi - j * h
        t = math.exp(u)
        x = ridge_solve(t, g)
        T = np.sum(ag * (a @ x), axis=0)
        d = t * np.sum(g * x, axis=0)
        done = True
        per = np.empty((Q, N))
        for q in range(Q):
            c = h * math.sin(math.pi * powers[q] / 2.0) / math.pi
            acc[q] += c * math.exp(0.5 * powers[q] * u) * T
            wb = lower_tail_weight(powers[q], h, u)
            per[q] = acc[q] + wb * gg
            if float(np.mean(np.abs(d))) * wb > eps_q * abs(float(per[q].mean())):
                done = False
        used = j + 1
        if done:
            break
    sums = per.mean(axis=1)
    r = orlicz_from_sums(coefs, powers, sums)
    # delta method: per-probe values of phi(r) and its derivative in r
    vals = np.sum((coefs * r ** (-powers))[:, None] * per, axis=0)
    dphi = float(np.sum(-powers * coefs * r ** (-powers - 1.0) * sums))
    se = float(vals.std(ddof=1) / math.sqrt(N) / abs(dphi)) if N > 1 else float("nan")
    return r, se, sums, used


# ---------------------------------------------------------------------------------
# Ky Fan norms (Section 3.2 names them beside the Orlicz norms)
# ---------------------------------------------------------------------------------
# ||A||_(k) = sum_{i<=k} sigma_i(A) needs the top of the spectrum itself, which ridge solves
# (A^T A + t I)^{-1} do not isolate (every function of sigma they reach is smooth in log sigma
# with a transition width that does not shrink). It is taken from the top singular subspace:
# randomized subspace iteration on A^T A from b >= k Gaussian vectors, q steps, each
# orthonormalised, then the Rayleigh-Ritz values of A on that subspace. Ritz values interlace
# (each is at most the singular value of the same rank), so the estimate never exceeds
# ||A||_(k) and converges to it; with rank(A) <= b one step is exact.
def orthonormal_columns(z: np.ndarray, drop: float = 1e-13) -> np.ndarray:
    """An orthonormal basis of range(z) (n x b) as z V Lambda^{-1/2} from the eigenpairs of
    z^T z; directions with eigenvalue <= drop * max are left out (zero columns)."""
    g = z.T @ z
    lam, v = np.linalg.eigh(0.5 * (g + g.T))
    keep = lam > drop * lam.max()
    scale = np.zeros_like(lam)
    scale[keep] = 1.0 / np.sqrt(lam[keep])
    return (z @ v) * scale[None, :]


def kyfan_subspace(a: np.ndarray, k: int, b: int, q: int, omega: np.ndarray):
    """The Ky Fan k-norm estimate from q steps of subspace iteration started at omega
    (n x b). Returns (estimate, the b Ritz singular values in decreasing order)."""
    if not (1 <= k <= b):
        raise ValueError("1 <= k <= b")
    qm = orthonormal_columns(np.asarray(omega, dtype=np.float64))
    for _ in range(q):
        qm = orthonormal_columns(a.T @ (a @ qm))
    t = a @ qm
    lam = np.linalg.eigvalsh(t.T @ t)
    sig = np.sqrt(np.clip(lam, 0.0, None))[::-1]
    return float(sig[:k].sum()), sig
