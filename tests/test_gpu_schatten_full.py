"""Parity at the full size of the Schatten-1 workload (A = Q diag(1/i) Q^T, Q a product of
8 Householder reflections, n = 16384, 512 Gaussian probes as one block, s = 1024,
phi = 4096, FP32 copy of A inside MSP with FP64 refinement), in the benchmark's launches.

The whole estimate takes hours of ridge solves at this size (its smallest quadrature nodes
are unregularised problems), so the checks are the integer sketch bit for bit, 48 sampled
rows of Y against the oracle's sketch of the same rows (each row from the factors), and one
quadrature node solved to convergence: the driver's node value (h sin(pi p/2)/pi)
e^{p u/2} mean_k <A g_k, A x_k> against its closed form
sum_i (Q^T g_k)_i^2 sigma_i^2 / (sigma_i^2 + t) computed on the host from the factors.
"""
import math

import numpy as np
import pytest
import torch

import paper_2405_05865_amd as msp
import workloads as W
from oracle import rng, sketch as osk
from oracle import msp as omsp
from oracle.refine import round_f32

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")
EPS32 = float(np.finfo(np.float32).eps)


def say(*a):
    print(*a, flush=True)


@pytest.mark.timeout(600)
def test_full_size_schatten_sketch_and_one_node():
    w = W.config("schatten1_n16384")
    n, s, N = w.n, w.s, w.nrhs
    say(f"case schatten full size n={n} s={s} probes={N}")
    sig, q_vs = W.schatten_psd_factors(n, w.config_id)
    A = W.outer_product_on_device(q_vs, sig, q_vs, DEV)
    A = 0.5 * (A + A.t())
    A32 = A.float()
    g = W.gaussian((N, n), w.config_id)
    G = torch.from_numpy(g).to(DEV)
    rows, signs, Y = msp.sketch(A32, s, w.gamma, w.seed_s)
    r_o, s_o = rng.sketch_indices(w.seed_s, n, s, w.gamma)
    assert np.array_equal(rows.cpu().numpy(), r_o)
    assert np.array_equal(signs.cpu().numpy(), s_o)
    Yh = Y.cpu().numpy().astype(np.float64)
    for i in np.random.default_rng(7).choice(n, 48, replace=False):
        row = round_f32(W.outer_product_row(q_vs, sig, q_vs, int(i)))[None]
        want = osk.right_sketch(row, r_o, s_o, s)[0]
        scale = osk.right_sketch(np.abs(row), r_o, np.ones_like(s_o), s)[0]
        assert np.all(np.abs(Yh[i] - want) <= 64 * EPS32 * scale), i
    lam0 = omsp.paper_lambda0(np.sort(sig)[::-1] ** 2, s // 2)
    P = msp.Precond("general", rows, signs, Y, 1.0, lam0, w.phi, w.phi_gamma, w.seed_phi)
    t, h, p = 1e-3, 1.5, 1.0
    u = math.log(t)
    say(f"case schatten one node t={t}")
    est, se, info = msp.schatten(P, A, G, p=p, A_lo=A32, h=h, u_lo=u, u_hi=u, refine=1, tol=1e-10)
    say(est, se, info)
    assert info["code"] == "MSP_OK", info
    qg = W.householder_apply(q_vs, g.T, transpose=True)  # n x N: Q^T g_k
    per = (qg ** 2 * (sig ** 2 / (sig ** 2 + t))[:, None]).sum(axis=0)
    wgt = h * math.sin(math.pi * p / 2) / math.pi * math.exp(0.5 * p * u)
    want = wgt * per.mean()
    se_want = wgt * per.std(ddof=1) / math.sqrt(N)
    say(f"node value {est:.12g} closed form {want:.12g}")
    assert est == pytest.approx(want, rel=1e-7)
    assert se == pytest.approx(se_want, rel=1e-4)
    P.close()
