"""Seeded input recipes for the five workloads of the MSP hot path.

Every draw comes from ``numpy.random.default_rng(SeedSequence([BASE_SEED, config_id,
stream]))`` with the streams

    0  matrix / orthogonal factors      2  right-hand sides and probe vectors
    1  spectrum                         3  points of the kernel matrices
    4  sizes and lengthscales of the batched systems

The recipes follow the problem statements of the paper: a PSD matrix with k large
eigenvalues (Problem 1.1 / Theorem 1.1), RBF kernel matrices for the kernel ridge
regression application (Theorem 3.2, Section 3.1), a nonsymmetric matrix with k large
singular values for the general three-level method (Theorem 3.1) and a PSD matrix with
a harmonic spectrum for Schatten-1 estimation (Theorem 3.3).

Nothing here sketches, preconditions or iterates: these are inputs only.
"""
from __future__ import annotations

import math
import os
from concurrent.futures import ThreadPoolExecutor
from dataclasses import dataclass, field

import numpy as np

BASE_SEED = 240505865

# stream ids
_MATRIX, _SPECTRUM, _RHS, _POINTS, _SIZES = 0, 1, 2, 3, 4


def rng_for(config_id: int, stream: int) -> np.random.Generator:
    """The generator of one (config, stream) pair."""
    return np.random.default_rng(np.random.SeedSequence([BASE_SEED, int(config_id), int(stream)]))


def _threads() -> int:
    return max(1, min(16, os.cpu_count() or 1))


def gaussian(shape, config_id: int, stream: int = _RHS) -> np.ndarray:
    """Standard normal float64 array (right-hand sides, probe vectors)."""
    return rng_for(config_id, stream).standard_normal(shape)


# ----------------------------------------------------------------------------------
# PSD matrix with k large eigenvalues (Problem 1.1): A = Q diag(sigma) Q^T
# ----------------------------------------------------------------------------------
def psd_outlier(n: int, k: int, config_id: int, big=(1e2, 1e4), small=(0.5, 1.0)):
    """Q from the QR factorization of an N(0,1) matrix (columns sign-fixed by diag(R)),
    k eigenvalues log-uniform in ``big`` and n-k uniform in ``small``.

    Returns (A, eigs, Q) with eigs sorted non-increasing and A exactly symmetric.
    """
    g = rng_for(config_id, _MATRIX).standard_normal((n, n))
    q, r = np.linalg.qr(g)
    q *= np.sign(np.diag(r))[None, :]
    rs = rng_for(config_id, _SPECTRUM)
    lo, hi = math.log10(big[0]), math.log10(big[1])
    eig_big = 10.0 ** rs.uniform(lo, hi, size=k)
    eig_small = rs.uniform(small[0], small[1], size=n - k)
    eigs = np.sort(np.concatenate([eig_big, eig_small]))[::-1].copy()
    a = (q * eigs[None, :]) @ q.T
    a = 0.5 * (a + a.T)
    return a, eigs, q


def tall_outlier(n: int, d: int, k: int, config_id: int, big=(1e2, 1e4), small=(1.0, 10.0)):
    """Tall A = U diag(sv) V^T (n x d, n >= d): U from the QR factorization of an N(0,1)
    n x d matrix, V from that of a d x d one (columns sign-fixed by diag(R)), k singular
    values log-uniform in ``big`` and d-k uniform in ``small`` (the setting of the paper's
    least-squares corollary). Returns (A, sv sorted non-increasing)."""
    u, r = np.linalg.qr(rng_for(config_id, _MATRIX).standard_normal((n, d)))
    u *= np.sign(np.diag(r))[None, :]
    v, r = np.linalg.qr(rng_for(config_id, _MATRIX + 10).standard_normal((d, d)))
    v *= np.sign(np.diag(r))[None, :]
    rs = rng_for(config_id, _SPECTRUM)
    lo, hi = math.log10(big[0]), math.log10(big[1])
    sv = np.sort(np.concatenate([10.0 ** rs.uniform(lo, hi, size=k), rs.uniform(small[0], small[1], size=d - k)]))[::-1]
    return (u * sv[None, :]) @ v.T, sv.copy()


# ----------------------------------------------------------------------------------
# RBF kernel matrices (kernel ridge regression / GP regression)
# ----------------------------------------------------------------------------------
def rbf_points(n: int, dim: int, config_id: int, stream: int = _POINTS) -> np.ndarray:
    return rng_for(config_id, stream).standard_normal((n, dim))


def rbf_rows(points: np.ndarray, rows, lengthscale: float = 1.0) -> np.ndarray:
    """Rows ``rows`` of K_ab = exp(-|p_a - p_b|^2 / (2 l^2)), squared distance formed
    coordinate by coordinate (no Gram-matrix cancellation), K_aa = 1 exactly."""
    rows = np.asarray(rows, dtype=np.int64)
    pr = points[rows]
    d2 = np.zeros((rows.size, points.shape[0]))
    for c in range(points.shape[1]):
        diff = pr[:, c:c + 1] - points[None, :, c]
        d2 += diff * diff
    out = np.exp(d2 * (-0.5 / (lengthscale * lengthscale)))
    out[np.arange(rows.size), rows] = 1.0
    return out


def rbf_matrix(points: np.ndarray, lengthscale: float = 1.0, dtype=np.float64,
               block: int = 1024) -> np.ndarray:
    """The full n x n RBF kernel matrix, built in row blocks on host threads."""
    n = points.shape[0]
    out = np.empty((n, n), dtype=dtype)

    def work(r0):
        r1 = min(n, r0 + block)
        out[r0:r1] = rbf_rows(points, np.arange(r0, r1), lengthscale).astype(dtype, copy=False)

    with ThreadPoolExecutor(_threads()) as ex:
        list(ex.map(work, range(0, n, block)))
    return out


def batched_rbf_sizes(count: int, config_id: int, lo: int = 512, hi: int = 8192,
                      ls_lo: float = 0.5, ls_hi: float = 2.0):
    """Sizes n_j ~ U{lo..hi} and lengthscales l_j ~ U(ls_lo, ls_hi) of uneven systems."""
    r = rng_for(config_id, _SIZES)
    sizes = r.integers(lo, hi + 1, size=count)
    ls = r.uniform(ls_lo, ls_hi, size=count)
    return sizes, ls


def system_rng(config_id: int, stream: int, index: int) -> np.random.Generator:
    """The generator of one system of a batch (its own seed per index)."""
    return np.random.default_rng(np.random.SeedSequence([BASE_SEED, int(config_id), int(stream), int(index)]))


def batched_rbf_system(index: int, n: int, lengthscale: float, dim: int, nrhs: int, config_id: int):
    """System `index` of a batch: the F32 RBF matrix (formed in FP64, rounded to nearest
    F32: the F32 matrix is the problem) and nrhs standard normal right-hand sides."""
    pts = system_rng(config_id, _POINTS, index).standard_normal((n, dim))
    a = rbf_matrix(pts, lengthscale=lengthscale, dtype=np.float32)
    b = system_rng(config_id, _RHS, index).standard_normal((nrhs, n))
    return a, b


# ----------------------------------------------------------------------------------
# Householder-product orthogonal factors
# ----------------------------------------------------------------------------------
def householder_vectors(n: int, count: int, config_id: int, stream: int) -> np.ndarray:
    """``count`` unit vectors v_r; H_r = I - 2 v_r v_r^T."""
    v = rng_for(config_id, stream).standard_normal((count, n))
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    return v


def householder_apply(vs: np.ndarray, x: np.ndarray, transpose: bool = False) -> np.ndarray:
    """Q x with Q = H_1 H_2 ... H_count (transpose: Q^T x). ``x`` is (n,) or (n, k)."""
    y = np.array(x, dtype=np.float64, copy=True)
    order = range(len(vs)) if transpose else range(len(vs) - 1, -1, -1)
    for r in order:
        v = vs[r]
        y -= 2.0 * np.multiply.outer(v, v @ y) if y.ndim == 2 else 2.0 * v * (v @ y)
    return y


def _outer_product_matrix(u_vs, diag, v_vs, dtype, n, block=4096):
    """U diag(d) V^T with U = H_1...H_k and V = H'_1...H'_k, assembled in place by
    rank-one updates applied in row blocks (no n x n temporaries)."""
    a = np.zeros((n, n), dtype=np.float64)
    a[np.arange(n), np.arange(n)] = diag
    # A <- A V^T = ((D H'_k) H'_{k-1}) ... H'_1
    for r in range(len(v_vs) - 1, -1, -1):
        v = v_vs[r]
        w = a @ v
        for r0 in range(0, n, block):
            a[r0:r0 + block] -= 2.0 * np.outer(w[r0:r0 + block], v)
    # A <- U A = H_1 (H_2 ( ... (H_k A)))
    for r in range(len(u_vs) - 1, -1, -1):
        u = u_vs[r]
        w = u @ a
        for r0 in range(0, n, block):
            a[r0:r0 + block] -= 2.0 * np.outer(u[r0:r0 + block], w)
    return a.astype(dtype, copy=False)


def general_outlier_factors(n: int, k: int, config_id: int, reflections: int = 8,
                            big=(1e3, 1e6), small=(1.0, 10.0)):
    """The factors of general_outlier without forming A: (sv, u_vs, v_vs)."""
    u_vs = householder_vectors(n, reflections, config_id, _MATRIX)
    v_vs = householder_vectors(n, reflections, config_id, _MATRIX + 10)
    rs = rng_for(config_id, _SPECTRUM)
    sv = np.empty(n)
    sv[:k] = 10.0 ** rs.uniform(math.log10(big[0]), math.log10(big[1]), size=k)
    sv[k:] = rs.uniform(small[0], small[1], size=n - k)
    return sv, u_vs, v_vs


def outer_product_on_device(u_vs, diag, v_vs, device):
    """U diag(d) V^T on a torch device (FP64) by the rank-one updates of
    _outer_product_matrix, for sizes the host cannot assemble quickly."""
    import torch
    n = diag.shape[0]
    a = torch.zeros((n, n), dtype=torch.float64, device=device)
    a.diagonal().copy_(torch.from_numpy(np.ascontiguousarray(diag)).to(device))
    for r in range(len(v_vs) - 1, -1, -1):
        v = torch.from_numpy(np.ascontiguousarray(v_vs[r])).to(device)
        a.addr_(torch.mv(a, v), v, alpha=-2.0)
    for r in range(len(u_vs) - 1, -1, -1):
        u = torch.from_numpy(np.ascontiguousarray(u_vs[r])).to(device)
        a.addr_(u, torch.mv(a.t(), u), alpha=-2.0)
    return a


def outer_product_row(u_vs, diag, v_vs, i: int) -> np.ndarray:
    """Row i of U diag(d) V^T from the factors: ((U^T e_i) * d)^T V^T."""
    e = np.zeros(diag.shape[0])
    e[i] = 1.0
    return householder_apply(v_vs, diag * householder_apply(u_vs, e, transpose=True))


def outer_product_apply(u_vs, diag, v_vs, x: np.ndarray) -> np.ndarray:
    """U diag(d) V^T x from the factors (x of shape (n,) or (n, k))."""
    y = householder_apply(v_vs, x, transpose=True)
    y = diag * y if y.ndim == 1 else diag[:, None] * y
    return householder_apply(u_vs, y)


def general_outlier(n: int, k: int, config_id: int, reflections: int = 8,
                    big=(1e3, 1e6), small=(1.0, 10.0)):
    """Nonsymmetric A = U diag(sv) V^T with U, V products of Householder reflections,
    k singular values log-uniform in ``big`` at indices 0..k-1, the rest uniform in
    ``small``. Returns (A, sv, u_vs, v_vs)."""
    sv, u_vs, v_vs = general_outlier_factors(n, k, config_id, reflections, big, small)
    a = _outer_product_matrix(u_vs, sv, v_vs, np.float64, n)
    return a, sv, u_vs, v_vs


def schatten_psd_factors(n: int, config_id: int, reflections: int = 8):
    """The factors of schatten_psd without forming A: (sigma, q_vs)."""
    q_vs = householder_vectors(n, reflections, config_id, _MATRIX)
    sigma = 1.0 / np.arange(1, n + 1, dtype=np.float64)
    return sigma, q_vs


def schatten_psd(n: int, config_id: int, reflections: int = 8):
    """PSD A = Q diag(1/i) Q^T, Q a product of Householder reflections.
    Returns (A, sigma, q_vs)."""
    sigma, q_vs = schatten_psd_factors(n, config_id, reflections)
    a = _outer_product_matrix(q_vs, sigma, q_vs, np.float64, n)
    a = 0.5 * (a + a.T)
    return a, sigma, q_vs


# ----------------------------------------------------------------------------------
# Workload descriptions
# ----------------------------------------------------------------------------------
@dataclass
class Workload:
    name: str
    config_id: int
    n: int
    s: int
    gamma: int
    phi: int
    phi_gamma: int
    lam: float
    tol: float
    nrhs: int = 1
    structure: str = "psd"          # "psd" (two-level) or "general" (three-level)
    extra: dict = field(default_factory=dict)

    @property
    def l(self) -> int:
        """Rank parameter l of Theorem 4.1; the sketch size is s = 2 l."""
        return self.s // 2

    @property
    def seed_s(self) -> int:
        return BASE_SEED * 16 + self.config_id

    @property
    def seed_phi(self) -> int:
        return self.seed_s + 8


CONFIGS = {
    # plain MSP regularized solve, PSD with 32 outlying eigenvalues
    "psd_outlier_n1024": Workload("psd_outlier_n1024", 0, n=1024, s=64, gamma=8, phi=256, phi_gamma=8,
                                  lam=1e-3, tol=1e-10, extra={"k": 32}),
    # GP-regression-shaped RBF solve (the headline workload)
    "rbf_gp_n32768": Workload("rbf_gp_n32768", 1, n=32768, s=512, gamma=8, phi=2048, phi_gamma=8,
                              lam=1e-2, tol=1e-8, extra={"dim": 8}),
    # nonsymmetric outlier system through the three-level method
    "general_outlier_n65536": Workload("general_outlier_n65536", 2, n=65536, s=2048, gamma=8, phi=8192,
                                       phi_gamma=8, lam=0.0, tol=1e-8, nrhs=8, structure="general",
                                       extra={"k": 1024}),
    # batched differentiable GP solves (256 uneven RBF systems, 16 RHS each)
    "batched_rbf_256": Workload("batched_rbf_256", 3, n=8192, s=256, gamma=8, phi=1024, phi_gamma=8,
                                lam=1e-2, tol=1e-8, nrhs=16, extra={"count": 256, "dim": 4}),
    # Schatten-1 estimation, PSD with sigma_i = 1/i, 512 probes
    "schatten1_n16384": Workload("schatten1_n16384", 4, n=16384, s=1024, gamma=8, phi=4096, phi_gamma=8,
                                 lam=0.0, tol=1e-6, nrhs=512, structure="general"),
}


def config(name: str, n: int | None = None, s: int | None = None) -> Workload:
    """A named workload, optionally rescaled (smaller n and sketch) for tests."""
    w = CONFIGS[name]
    if n is None and s is None:
        return w
    out = Workload(**{**w.__dict__, "extra": dict(w.extra)})
    if n is not None:
        out.n = int(n)
    if s is not None:
        out.s = int(s)
        out.phi = 4 * int(s)
    return out
