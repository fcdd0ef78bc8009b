"""GPU checks of mixed precision with FP64 refinement, the adjoint (and its autograd
wrapper), and the spectral-sum drivers, all against the oracle."""
import math

import numpy as np
import pytest
import torch

import paper_2405_05865_amd as msp
import workloads as W
from oracle import dense, trace
from oracle import msp as omsp

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")


def say(*a):
    print(*a, flush=True)


def _psd(n=1024, k=32, s=64, lam=1e-3, cid=0, dtype_lo=None, seeds=(21, 22)):
    a, eigs, q = W.psd_outlier(n, k, config_id=cid)
    lam0 = omsp.paper_lambda0(eigs, s // 2)
    A = torch.from_numpy(a).to(DEV)
    A_lo = A if dtype_lo is None else A.to(dtype_lo)
    rows, signs, Y = msp.sketch(A_lo, s, 8, seeds[0])
    P = msp.Precond("psd", rows, signs, Y, lam, lam0, 4 * s, 8, seeds[1])
    return a, eigs, q, lam0, A, A_lo, P


@pytest.mark.parametrize("dt", [torch.float32, torch.bfloat16])
def test_psd_low_precision_sweeps_refined_to_fp64(dt):
    say(f"case psd refine {dt}")
    lam = 1e-3 if dt == torch.float32 else 0.5
    a, eigs, _, lam0, A, A_lo, P = _psd(lam=lam, dtype_lo=dt)
    b = W.gaussian(a.shape[0], 0)
    X, info = msp.solve(P, A, torch.from_numpy(b).to(DEV), A_lo=A_lo, refine=1, tol=1e-10)
    say(info)
    x = X.cpu().numpy()
    assert info["status"] == "MSP_OK", info
    assert dense.rel_residual_psd(a, x, b, lam) <= 1e-10
    xs = dense.solve_psd(a, b, lam)
    assert np.linalg.norm(x - xs) <= 1e-7 * np.linalg.norm(xs)


def test_rbf_f32_problem_bf16_sweeps():
    # kernel-ridge shape: the F32 matrix is the problem, BF16 is the sweep copy
    say("case rbf f32/bf16 n=2048")
    n, s, lam = 2048, 128, 1e-2
    pts = W.rbf_points(n, 4, 3)
    a32 = W.rbf_matrix(pts, lengthscale=1.0, dtype=np.float32)
    a = a32.astype(np.float64)
    eigs = np.linalg.eigvalsh(a)[::-1]
    lam0 = omsp.paper_lambda0(eigs, s // 2)
    A = torch.from_numpy(a32).to(DEV)
    A_lo = A.to(torch.bfloat16)
    rows, signs, Y = msp.sketch(A_lo, s, 8, 5)
    P = msp.Precond("psd", rows, signs, Y, lam, lam0, 4 * s, 8, 6)
    B = W.gaussian((4, n), 3)
    X, info = msp.solve(P, A, torch.from_numpy(B).to(DEV), A_lo=A_lo, refine=1, tol=1e-8)
    say(info)
    x = X.cpu().numpy()
    assert info["status"] == "MSP_OK", info
    for j in range(4):
        assert dense.rel_residual_psd(a, x[j], B[j], lam) <= 1e-8
        xs = dense.solve_psd(a, B[j], lam)
        assert np.linalg.norm(x[j] - xs) <= 1e-6 * np.linalg.norm(xs)


def test_adjoint_matches_dense_gradients():
    say("case adjoint n=512 k=2")
    n, s, lam = 512, 32, 1e-2
    a, eigs, _, lam0, A, _, P = _psd(n=n, k=16, s=s, lam=lam, cid=301)
    B = W.gaussian((2, n), 301)
    X, _ = msp.solve(P, A, torch.from_numpy(B).to(DEV), tol=1e-12, inner_tol=1e-13)
    G = 2.0 * X  # L = sum |x|^2
    dB, dlam, dA, info = msp.solve_backward(P, A, X, G.contiguous(), want_dA=True, tol=1e-12, inner_tol=1e-13)
    x = X.cpu().numpy().T
    db_o, da_o, dl_o = dense.gradients(a, lam, x, 2.0 * x)
    assert np.linalg.norm(dB.cpu().numpy().T - db_o) <= 1e-9 * np.linalg.norm(db_o)
    assert dlam == pytest.approx(dl_o, rel=1e-9)
    assert np.linalg.norm(dA.cpu().numpy() - da_o) <= 1e-9 * np.linalg.norm(da_o)


def test_autograd_function_and_finite_differences():
    say("case autograd n=256")
    n, s, lam = 256, 32, 0.1
    a, eigs, _, lam0, A, _, P = _psd(n=n, k=8, s=s, lam=lam, cid=302)
    B = torch.from_numpy(W.gaussian(n, 302)).to(DEV).requires_grad_(True)
    Ar = A.clone().requires_grad_(True)
    lamt = torch.tensor(lam, dtype=torch.float64, device=DEV, requires_grad=True)
    X = msp.MSPSolve.apply(Ar, B, lamt, P, {"tol": 1e-12, "inner_tol": 1e-13})
    loss = (X * X).sum()
    loss.backward()
    b = B.detach().cpu().numpy()
    x = np.linalg.solve(a + lam * np.eye(n), b)
    db, da, dl = dense.gradients(a, lam, x, 2.0 * x)
    assert np.linalg.norm(B.grad.cpu().numpy() - db) <= 1e-9 * np.linalg.norm(db)
    assert np.linalg.norm(Ar.grad.cpu().numpy() - da) <= 1e-9 * np.linalg.norm(da)
    assert lamt.grad.item() == pytest.approx(dl, rel=1e-9)
    # central finite difference in lam of the oracle's dense loss
    h = 1e-6
    f = lambda l_: float(np.sum(np.linalg.solve(a + l_ * np.eye(n), b) ** 2))
    assert lamt.grad.item() == pytest.approx((f(lam + h) - f(lam - h)) / (2 * h), rel=1e-6)


def test_autograd_at_a_lambda_other_than_the_handles():
    # the solve and its adjoint take lam from the autograd input; the handle (built for
    # lam_P) is reused as the preconditioner
    say("case autograd lam != handle lam n=256")
    n, s, lam_p, lam = 256, 32, 0.1, 0.37
    a, eigs, _, lam0, A, _, P = _psd(n=n, k=8, s=s, lam=lam_p, cid=303)
    B = torch.from_numpy(W.gaussian(n, 303)).to(DEV).requires_grad_(True)
    Ar = A.clone().requires_grad_(True)
    lamt = torch.tensor(lam, dtype=torch.float64, device=DEV, requires_grad=True)
    X = msp.MSPSolve.apply(Ar, B, lamt, P, {"tol": 1e-12, "inner_tol": 1e-13})
    loss = (X * X).sum()
    loss.backward()
    b = B.detach().cpu().numpy()
    x = np.linalg.solve(a + lam * np.eye(n), b)
    assert np.linalg.norm(X.detach().cpu().numpy() - x) <= 1e-9 * np.linalg.norm(x)
    db, da, dl = dense.gradients(a, lam, x, 2.0 * x)
    assert np.linalg.norm(B.grad.cpu().numpy() - db) <= 1e-9 * np.linalg.norm(db)
    assert np.linalg.norm(Ar.grad.cpu().numpy() - da) <= 1e-9 * np.linalg.norm(da)
    assert lamt.grad.item() == pytest.approx(dl, rel=1e-9)
    assert P.lam == lam_p


def test_autograd_raises_when_the_solve_does_not_converge():
    say("case autograd cap n=256")
    n, s = 256, 32
    a, eigs, _, lam0, A, _, P = _psd(n=n, k=8, s=s, lam=1e-3, cid=304)
    B = torch.from_numpy(W.gaussian(n, 304)).to(DEV)
    lamt = torch.tensor(1e-3, dtype=torch.float64, device=DEV)
    with pytest.raises(msp.MspError) as e:
        msp.MSPSolve.apply(A, B, lamt, P, {"tol": 1e-14, "max_outer": 1})
    assert e.value.status == "MSP_ERR_NO_CONVERGENCE"


def test_solve_reports_wall_seconds():
    say("case solve seconds n=512")
    a, eigs, _, lam0, A, _, P = _psd(n=512, k=16, s=32, lam=1e-2, cid=305)
    X, info = msp.solve(P, A, torch.from_numpy(W.gaussian(512, 305)).to(DEV), tol=1e-10)
    assert info["status"] == "MSP_OK" and 0.0 < info["seconds"] < 60.0


def test_schatten1_matches_oracle_estimator(monkeypatch):
    say("case schatten-1 n=200 N=32")
    monkeypatch.setenv("MSP_LOG", "1")
    n, s, N = 200, 32, 32
    a, sig, _ = W.schatten_psd(n, config_id=200)
    g = W.gaussian((N, n), 200)
    lam0 = omsp.paper_lambda0(sig ** 2, s // 2)
    A = torch.from_numpy(a).to(DEV)
    rows, signs, Y = msp.sketch(A, s, 8, 7)
    P = msp.Precond("general", rows, signs, Y, 1.0, lam0, 4 * s, 8, 8)
    u_lo, u_hi = trace.default_range(1.0, n, eps_q=1e-2)
    h = 2.0
    est, se, info = msp.schatten(P, A, torch.from_numpy(g).to(DEV), p=1.0, h=h, u_lo=u_lo, u_hi=u_hi,
                                 tol=1e-8, inner_tol=1e-10, level3_tol=1e-10)
    nodes, w = trace.quadrature(1.0, h, u_lo, u_hi)
    ridge = lambda t, G: np.linalg.solve(a.T @ a + t * np.eye(n), G)
    est_o, se_o, _ = trace.schatten_estimate(a, g.T, 1.0, nodes, w, ridge)
    say(est, se, est_o, se_o, info)
    assert est == pytest.approx(est_o, rel=1e-6)
    assert se == pytest.approx(se_o, rel=1e-4)
    exact = dense.schatten_p(sig, 1.0)
    # Hutchinson sd for PSD A plus the quadrature error of the coarse, narrow node set
    assert abs(est - exact) < 4 * math.sqrt(2.0 * np.sum(sig ** 2) / N) + 2e-2 * exact


@pytest.mark.parametrize("pp", [0.5, 1.5])
def test_schatten_p_matches_oracle_estimator(pp):
    # p != 1 through the same driver: weights h sin(pi p/2)/pi e^{(p/2) u} and the range
    # rule in p, against the oracle's estimator on the same probes and nodes
    say(f"case schatten-p p={pp} n=160 N=24")
    n, s, N = 160, 32, 24
    a, sig, _ = W.schatten_psd(n, config_id=201)
    g = W.gaussian((N, n), 201)
    lam0 = omsp.paper_lambda0(sig ** 2, s // 2)
    A = torch.from_numpy(a).to(DEV)
    rows, signs, Y = msp.sketch(A, s, 8, 17)
    P = msp.Precond("general", rows, signs, Y, 1.0, lam0, 4 * s, 8, 18)
    u_lo, u_hi = trace.default_range(1.0, n, p=pp, eps_q=1e-2)
    h = 2.0
    est, se, info = msp.schatten(P, A, torch.from_numpy(g).to(DEV), p=pp, h=h, u_lo=u_lo, u_hi=u_hi,
                                 tol=1e-8, inner_tol=1e-10, level3_tol=1e-10)
    assert info["code"] == "MSP_OK", info
    nodes, w = trace.quadrature(pp, h, u_lo, u_hi)
    ridge = lambda t, G: np.linalg.solve(a.T @ a + t * np.eye(n), G)
    est_o, se_o, _ = trace.schatten_estimate(a, g.T, pp, nodes, w, ridge)
    say(est, se, est_o, se_o)
    assert est == pytest.approx(est_o, rel=1e-6)
    assert se == pytest.approx(se_o, rel=1e-4)
    # the quadrature of the exact spectrum with these nodes bounds what the estimator targets
    target = float(trace.quadrature_scalar(sig, pp, nodes, w).sum())
    assert abs(est - target) < 5 * se + 1e-12


def test_effective_dimension_matches_oracle():
    say("case effdim n=256 N=64")
    n, s, lam, N = 256, 32, 0.05, 64
    a, eigs, _, lam0, A, _, P = _psd(n=n, k=8, s=s, lam=lam, cid=202)
    g = W.gaussian((N, n), 202)
    est, se, info = msp.effective_dimension(P, A, torch.from_numpy(g).to(DEV), lam, tol=1e-12, inner_tol=1e-13)
    est_o, per_o = trace.effective_dimension_estimate(g.T, lam, lambda G: dense.solve_psd(a, G, lam))
    assert est == pytest.approx(est_o, rel=1e-9)
    d = dense.effective_dimension(eigs, lam)
    assert abs(est - d) < 4 * math.sqrt(2.0 * np.sum((eigs / (eigs + lam)) ** 2) / N)


def test_gaussian_probes_match_oracle_generator():
    # the integer stream is the same on both sides; the Box-Muller transform (log, sqrt,
    # cos in FP64) agrees to a few ulp
    from oracle import rng
    say("case gaussian probes n=3001 N=17")
    n, N, seed = 3001, 17, 424242
    G = msp.gaussian_probes(n, N, seed).cpu().numpy()
    want = rng.gaussian_probes(seed, n, N)
    assert np.all(np.abs(G - want) <= 1e-14 * np.maximum(1.0, np.abs(want)))


def test_schatten_generates_probes_from_a_seed():
    # G = NULL: the driver draws the probes itself; the same estimate as passing them in
    say("case schatten-1 with generated probes n=200 N=16")
    n, s, N, seed = 200, 32, 16, 77
    a, sig, _ = W.schatten_psd(n, config_id=201)
    lam0 = omsp.paper_lambda0(sig ** 2, s // 2)
    A = torch.from_numpy(a).to(DEV)
    rows, signs, Y = msp.sketch(A, s, 8, 9)
    P = msp.Precond("general", rows, signs, Y, 1.0, lam0, 4 * s, 8, 10)
    u_lo, u_hi = trace.default_range(1.0, n, eps_q=1e-2)
    kw = dict(p=1.0, h=2.0, u_lo=u_lo, u_hi=u_hi, tol=1e-8, inner_tol=1e-10, level3_tol=1e-10)
    est1, se1, _ = msp.schatten(P, A, None, nprobes=N, probe_seed=seed, **kw)
    est2, se2, _ = msp.schatten(P, A, msp.gaussian_probes(n, N, seed), **kw)
    assert est1 == est2 and se1 == se2


def test_schatten_descending_nodes_match_oracle():
    # u_lo NaN: nodes from u_hi down, the lower tail replaced by |g|^2 once its bound is
    # below 1e-4 of the estimate; the same nodes, stop and estimate as the oracle's
    say("case schatten-1 descending nodes n=200 N=16")
    n, s, N, h = 200, 32, 16, 1.5
    a, sig, _ = W.schatten_psd(n, config_id=203)
    g = W.gaussian((N, n), 203)
    lam0 = omsp.paper_lambda0(sig ** 2, s // 2)
    A = torch.from_numpy(a).to(DEV)
    rows, signs, Y = msp.sketch(A, s, 8, 27)
    P = msp.Precond("general", rows, signs, Y, 1.0, lam0, 4 * s, 8, 28)
    u_hi = trace.upper_end(1.0, 1.0)
    est, se, info = msp.schatten(P, A, torch.from_numpy(g).to(DEV), p=1.0, h=h, u_hi=u_hi, tol=1e-10,
                                 inner_tol=1e-12, level3_tol=1e-12)
    assert info["code"] == "MSP_OK", info
    ridge = lambda t, G: np.linalg.solve(a.T @ a + t * np.eye(n), G)
    est_o, se_o, _, used, bound = trace.schatten_descending(a, g.T, 1.0, h, u_hi, ridge)
    say(est, se, est_o, se_o, info["trace_nodes"], used, bound)
    assert info["trace_nodes"] == used
    assert est == pytest.approx(est_o, rel=1e-6)
    assert se == pytest.approx(se_o, rel=1e-4)
    exact = dense.schatten_p(sig, 1.0)
    assert abs(est - exact) < 4 * math.sqrt(2.0 * np.sum(sig ** 2) / N) + 2e-4 * exact


def test_orlicz_matches_oracle():
    # g(s) = s + 0.5 s^1.5: both Schatten sums from one descent, then the root of
    # sum_q c_q r^{-p_q} S_q = 1, against the oracle on the same probes
    from scipy.optimize import brentq
    say("case orlicz n=200 N=16")
    n, s, N, h = 200, 32, 16, 1.5
    a, sig, _ = W.schatten_psd(n, config_id=204)
    g = W.gaussian((N, n), 204)
    lam0 = omsp.paper_lambda0(sig ** 2, s // 2)
    A = torch.from_numpy(a).to(DEV)
    rows, signs, Y = msp.sketch(A, s, 8, 37)
    P = msp.Precond("general", rows, signs, Y, 1.0, lam0, 4 * s, 8, 38)
    coefs, powers = [1.0, 0.5], [1.0, 1.5]
    u_hi = trace.upper_end(1.0, 1.5)
    r, se, sums, info = msp.orlicz(P, A, torch.from_numpy(g).to(DEV), coefs, powers, h=h, u_hi=u_hi, tol=1e-10,
                                   inner_tol=1e-12, level3_tol=1e-12)
    assert info["code"] == "MSP_OK", info
    ridge = lambda t, G: np.linalg.solve(a.T @ a + t * np.eye(n), G)
    r_o, se_o, sums_o, used = trace.orlicz_estimate(a, g.T, coefs, powers, h, u_hi, ridge)
    say(r, se, sums, r_o, se_o, list(sums_o), info["trace_nodes"], used)
    assert info["trace_nodes"] == used
    assert r == pytest.approx(r_o, rel=1e-6)
    assert np.allclose(sums, sums_o, rtol=1e-6)
    assert se == pytest.approx(se_o, rel=1e-4)
    want = brentq(lambda x: float(np.sum(sig / x + 0.5 * (sig / x) ** 1.5)) - 1.0, 1e-3, 1e6, xtol=1e-14)
    assert abs(r - want) < 4 * se + 2e-4 * want


def _kyfan_matrix(m, n, sig, seed):
    rng_ = np.random.default_rng(seed)
    u, _ = np.linalg.qr(rng_.standard_normal((m, n)))
    v, _ = np.linalg.qr(rng_.standard_normal((n, n)))
    return (u * sig) @ v.T


@pytest.mark.parametrize("dt", [torch.float64, torch.float32])
def test_kyfan_matches_oracle_subspace(dt):
    # the same Gaussian start block (the probe generator) on both sides: the GPU's Ritz
    # values against the oracle's subspace iteration on the same (rounded) matrix, and the
    # estimate against the singular values (sigma_{b+1} / sigma_k = 1/3: converged)
    from oracle import rng
    say(f"case ky fan m=300 n=240 k=6 b=12 q=12 {dt}")
    m, n, k, b, q, seed = 300, 240, 6, 12, 12, 99
    sig = np.concatenate([np.linspace(10.0, 6.0, 8), np.linspace(2.0, 0.1, n - 8)])
    a = _kyfan_matrix(m, n, sig, 401)
    A = torch.from_numpy(a).to(DEV).to(dt).contiguous()
    est, ritz = msp.kyfan(A, k, b, q, seed)
    a_used = A.double().cpu().numpy()
    omega = rng.gaussian_probes(seed, n, b).T
    est_o, ritz_o = trace.kyfan_subspace(a_used, k, b, q, omega)
    say(est, est_o, ritz[:4], ritz_o[:4])
    assert np.allclose(ritz, ritz_o, rtol=1e-9, atol=1e-12 * ritz_o[0])
    assert est == pytest.approx(est_o, rel=1e-10)
    sv = np.linalg.svd(a_used, compute_uv=False)
    assert est <= sv[:k].sum() * (1 + 1e-12)
    assert est >= sv[:k].sum() * (1 - 1e-9)


def test_kyfan_exact_at_low_rank():
    # rank(A) = 9 <= b = 16: one step of the iteration spans range(A^T)
    say("case ky fan low rank")
    m, n, r = 200, 150, 9
    g = np.random.default_rng(402)
    a = g.standard_normal((m, r)) @ g.standard_normal((r, n))
    sv = np.linalg.svd(a, compute_uv=False)
    A = torch.from_numpy(a).to(DEV)
    for k in (1, 5, 9):
        est, ritz = msp.kyfan(A, k, 16, 1, 7)
        assert est == pytest.approx(float(sv[:k].sum()), rel=1e-10)
    assert np.allclose(ritz[:r], sv[:r], rtol=1e-10)
    assert max(ritz[r:]) <= 1e-7 * sv[0]
