"""Least squares through msp_left_sketch + msp_lstsq (sketch-and-precondition around the
three-level MSP) against the oracle's iteration on the same sketches and against dense
least squares (within the forward error the normal-equation residual allows)."""
import numpy as np
import pytest
import torch

import paper_2405_05865_amd as msp
import workloads as W
from oracle import lstsq as olstsq
from oracle import msp as omsp
from oracle import rng, sketch as osk

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")
EPS = np.finfo(np.float64).eps


def say(*a):
    print(*a, flush=True)


def _problem(n, d, k, cid, s):
    a, sv = W.tall_outlier(n, d, k, cid)
    lam0 = omsp.paper_lambda0(sv ** 2, s // 2)
    return a, sv, lam0


def _build(A, q, s):
    rows, signs, At = msp.left_sketch(A, q, 8, 31)
    r2, s2, Y = msp.sketch(At, s, 8, 32)
    return rows, signs, At, r2, s2, Y


def _check_against_dense(a, b, x, sv, tol):
    # the host recomputes c - A^T A x with its own rounding (about u |A|^2 |x|, 1e-10 of |c|
    # here), hence the 20% margin on the library's own stop
    c = a.T @ b
    r = c - a.T @ (a @ x)
    assert np.linalg.norm(r) <= 1.2 * tol * np.linalg.norm(c)
    xs = olstsq.lstsq_dense(a, b)
    assert np.linalg.norm(x - xs) <= 1.01 * np.linalg.norm(r) / sv[-1] ** 2 + 1e-10 * np.linalg.norm(xs)


def test_left_sketch_matches_oracle():
    n, d, q = 3001, 70, 280
    say(f"case left sketch n={n} d={d} q={q}")
    a = W.gaussian((n, d), 702)
    A = torch.from_numpy(a).to(DEV)
    rows, signs, At = msp.left_sketch(A, q, 8, 41)
    r_o, s_o = rng.sketch_indices(41, n, q, 8)
    assert np.array_equal(rows.cpu().numpy(), r_o) and np.array_equal(signs.cpu().numpy(), s_o)
    want = osk.left_sketch(r_o, s_o, q, a)
    scale = osk.left_sketch(r_o, np.ones_like(s_o), q, np.abs(a))
    assert np.all(np.abs(At.cpu().numpy() - want) <= 64 * EPS * scale)


def test_lstsq_matches_oracle_iterations_and_dense():
    n, d, k, s = 4096, 128, 8, 32
    q = 4 * d
    say(f"case lstsq n={n} d={d} q={q} s={s}")
    a, sv, lam0 = _problem(n, d, k, 701, s)
    b = W.gaussian(n, 701)
    A = torch.from_numpy(a).to(DEV)
    rows, signs, At, r2, s2, Y = _build(A, q, s)
    P = msp.Precond("general", r2, s2, Y, 0.0, lam0, 4 * s, 8, 33)
    opts = dict(tol=1e-9, refine_inner_tol=1e-4, inner_tol=1e-10, level3_tol=1e-10)
    X, info = msp.lstsq(P, At, A, torch.from_numpy(b).to(DEV), **opts)
    say(info)
    assert info["code"] == "MSP_OK", info
    _check_against_dense(a, b, X.cpu().numpy(), sv, 1e-9)
    O = olstsq.LstsqMsp(a, q, 8, 31, s, 8, 32, 4 * s, 8, 33, lam0, inner_rel=1e-4,
                        opts=omsp.MspOptions(tol=1e-9, inner_tol=1e-10, level3_tol=1e-10))
    res = O.solve(b)
    say("gpu", info["outer_iters"], "oracle", res.iterations)
    assert res.status == "converged"
    assert abs(info["outer_iters"] - res.iterations) <= 2
    P.close()


@pytest.mark.parametrize("dt", [torch.float64, torch.float32])
def test_lstsq_block_of_rhs(dt):
    # k = 9 right-hand sides: the products with A on the matrix cores (FP64 arithmetic on
    # an FP32 A); the FP32 matrix is then the problem
    n, d, k, s, nrhs = 2500, 96, 6, 32, 9
    q = 4 * d
    say(f"case lstsq block n={n} d={d} k={nrhs} dtype={dt}")
    a, sv, lam0 = _problem(n, d, k, 703, s)
    A = torch.from_numpy(a).to(DEV).to(dt)
    a_p = A.double().cpu().numpy()
    sv_p = np.linalg.svd(a_p, compute_uv=False)
    bm = W.gaussian((nrhs, n), 703)
    bm[4] = 0.0  # a zero right-hand side
    rows, signs, At, r2, s2, Y = _build(A, q, s)
    P = msp.Precond("general", r2, s2, Y, 0.0, lam0, 4 * s, 8, 33)
    X, info = msp.lstsq(P, At, A, torch.from_numpy(bm).to(DEV), tol=1e-9)
    say(info)
    assert info["code"] == "MSP_OK", info
    x = X.cpu().numpy()
    assert not np.any(x[4])
    for j in range(nrhs):
        if j != 4:
            _check_against_dense(a_p, bm[j], x[j], sv_p, 1e-9)
    P.close()
