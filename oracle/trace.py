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
