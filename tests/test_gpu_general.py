"""GPU parity of the three-level path for general A (Algorithms 3-5) against the oracle."""
import numpy as np
import pytest
import torch

import paper_2405_05865_amd as msp
import workloads as W
from oracle import dense
from oracle import msp as omsp

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")


def say(*a):
    print(*a, flush=True)


def _gen(a, lam, lam0, s, seeds=(41, 43), y_dtype=None, A_sk=None):
    A = torch.from_numpy(a).to(DEV)
    rows, signs, Y = msp.sketch(A if A_sk is None else A_sk, s, 8, seeds[0], y_dtype=y_dtype)
    P = msp.Precond("general", rows, signs, Y, lam, lam0, 4 * s, 8, seeds[1])
    return A, P


def test_factors_match_oracle():
    say("case general factors n=400 s=32")
    n, s = 400, 32
    a, sv, _, _ = W.general_outlier(n, 12, config_id=103, big=(1e2, 1e4))
    lam0 = omsp.paper_lambda0(np.sort(sv)[::-1] ** 2, s // 2)
    A, P = _gen(a, 0.0, lam0, s)
    _, M3a, M3b = P.factors()
    O = omsp.GeneralMsp(a, 0.0, lam0, s, 8, 41, 4 * s, 8, 43)
    for got, want, M in ((M3a, O.m3a_inv, O.m3a), (M3b, O.m3b_inv, O.m3b)):
        kappa = np.linalg.cond(M)
        g = got.cpu().numpy()
        assert np.linalg.norm(g - want) <= kappa * 1e-12 * np.linalg.norm(want)


@pytest.mark.parametrize("form", [0, 1, 2])
def test_general_solve_matches_lu_and_oracle_iterations(form):
    # levels 2 and 3 through passes over A and A~ (form 0) or through the explicit
    # B^T B + lam~ A~^T A~ and A~^T A~ (form 1)
    say(f"case general solve n=400 k=12 s=32 level2_form={form}")
    n, k, s = 400, 12, 32
    a, sv, _, _ = W.general_outlier(n, k, config_id=103, big=(1e2, 1e4))
    lam0 = omsp.paper_lambda0(np.sort(sv)[::-1] ** 2, s // 2)
    b = W.gaussian(n, 103)
    A, P = _gen(a, 0.0, lam0, s)
    X, info = msp.solve(P, A, torch.from_numpy(b).to(DEV), tol=1e-10, inner_tol=1e-12, level3_tol=1e-12,
                        level2_form=form)
    x = X.cpu().numpy()
    say(info)
    assert info["status"] == "MSP_OK", info
    xs = dense.solve_general(a, b)
    assert np.linalg.norm(a @ x - b) <= 1e-10 * np.linalg.norm(b)
    assert np.linalg.norm(x - xs) <= 1e-7 * np.linalg.norm(xs)
    O = omsp.GeneralMsp(a, 0.0, lam0, s, 8, 41, 4 * s, 8, 43,
                        omsp.MspOptions(tol=1e-10, inner_tol=1e-12, level3_tol=1e-12))
    O.solve_system(b)
    say("gpu", info["outer_iters"], "oracle", O.info.outer_iterations)
    if form < 2:  # the same iteration as the oracle's Algorithms 3-5
        assert abs(info["outer_iters"] - O.info.outer_iterations) <= 2
    else:  # the one-level preconditioner (an explicit inverse) is a different, weaker one here
        assert info["inner_iters"] == 0 and info["level3_iters"] == 0


def test_lower_bound_example_one():
    # Section 7: A = I + e_i e_j^T - e_j e_i^T, b = 1  ->  x = 1 except x_i = 0
    say("case lower-bound example one n=96")
    n, i, j, s = 96, 5, 70, 16
    a = np.eye(n)
    a[i, j] += 1.0
    a[j, i] -= 1.0
    sv = np.array([np.sqrt(2.0)] * 2 + [1.0] * (n - 2))
    lam0 = omsp.paper_lambda0(sv ** 2, s // 2)
    A, P = _gen(a, 0.0, lam0, s)
    X, info = msp.solve(P, A, torch.ones(n, dtype=torch.float64, device=DEV), tol=1e-12, inner_tol=1e-13,
                        level3_tol=1e-13)
    want = np.ones(n)
    want[i] = 0.0
    assert np.abs(X.cpu().numpy() - want).max() <= 1e-10


def test_lower_bound_example_two():
    # Section 7: blockdiag(M, sigma_min(M) I) [x; y] = [c; 0]  ->  y = 0, x = M^{-1} c
    say("case lower-bound example two n=160")
    k, n, s = 8, 160, 32
    r = np.random.default_rng(7).standard_normal((k, k))
    m = r + 3 * np.eye(k)
    smin = np.linalg.svd(m, compute_uv=False).min()
    a = np.zeros((n, n))
    a[:k, :k] = m
    a[k:, k:] = smin * np.eye(n - k)
    b = np.zeros(n)
    b[:k] = np.random.default_rng(8).standard_normal(k)
    sv = np.sort(np.linalg.svd(a, compute_uv=False))[::-1]
    lam0 = omsp.paper_lambda0(sv ** 2, s // 2)
    A, P = _gen(a, 0.0, lam0, s)
    X, info = msp.solve(P, A, torch.from_numpy(b).to(DEV), tol=1e-12, inner_tol=1e-13, level3_tol=1e-13)
    x = X.cpu().numpy()
    assert np.abs(x[k:]).max() <= 1e-10 * np.linalg.norm(b)
    assert np.linalg.norm(x[:k] - np.linalg.solve(m, b[:k])) <= 1e-9 * np.linalg.norm(b)


def test_ridge_normal_equations_multi_rhs():
    say("case general normal mode n=300 k=3")
    n, s, lam = 300, 32, 0.5
    a, sv, _, _ = W.general_outlier(n, 6, config_id=104, big=(1e1, 1e3))
    lam0 = omsp.paper_lambda0(np.sort(sv)[::-1] ** 2, s // 2)
    c = W.gaussian((3, n), 104)
    A, P = _gen(a, lam, lam0, s)
    X, info = msp.solve(P, A, torch.from_numpy(c).to(DEV), normal=1, tol=1e-11, inner_tol=1e-12, level3_tol=1e-12)
    assert info["status"] == "MSP_OK", info
    x = X.cpu().numpy()
    for j in range(3):
        xs = dense.solve_ridge(a, c[j], lam)
        assert np.linalg.norm(x[j] - xs) <= 1e-8 * np.linalg.norm(xs)


def test_general_f32_sweeps_with_fp64_refinement():
    # FP32-stored A inside MSP, FP64 residuals on the FP64 A
    say("case general refine f32 n=512")
    n, s = 512, 32
    a, sv, _, _ = W.general_outlier(n, 8, config_id=105, big=(1e2, 1e3))
    lam0 = omsp.paper_lambda0(np.sort(sv)[::-1] ** 2, s // 2)
    b = W.gaussian(n, 105)
    A = torch.from_numpy(a).to(DEV)
    A32 = A.float()
    rows, signs, Y = msp.sketch(A32, s, 8, 41)
    P = msp.Precond("general", rows, signs, Y, 0.0, lam0, 4 * s, 8, 43)
    X, info = msp.solve(P, A, torch.from_numpy(b).to(DEV), A_lo=A32, refine=1, tol=1e-10, inner_tol=1e-8,
                        level3_tol=1e-8)
    say(info)
    x = X.cpu().numpy()
    assert info["status"] == "MSP_OK", info
    assert np.linalg.norm(a @ x - b) <= 1e-10 * np.linalg.norm(b)
    xs = dense.solve_general(a, b)
    assert np.linalg.norm(x - xs) <= 1e-7 * np.linalg.norm(xs)
    assert info["refine_steps"] >= 1


def test_unsupported_adjoint_for_general():
    n, s = 64, 16
    a, sv, _, _ = W.general_outlier(n, 4, config_id=106, big=(1e1, 1e2))
    A, P = _gen(a, 0.0, 1.0, s)
    X = torch.zeros(n, dtype=torch.float64, device=DEV)
    with pytest.raises(msp.MspError) as e:
        msp.solve_backward(P, A, X, X.clone())
    assert e.value.status == "MSP_ERR_UNSUPPORTED"


def test_general_block_rhs_matrix_core_sweeps():
    # k >= 8: both A and A^T products of the three-level path on blocks
    say("case general block rhs n=300 k=9")
    n, s, k = 300, 32, 9
    a, sv, _, _ = W.general_outlier(n, 6, config_id=107, big=(1e1, 1e3))
    lam0 = omsp.paper_lambda0(np.sort(sv)[::-1] ** 2, s // 2)
    bm = W.gaussian((k, n), 107)
    A, P = _gen(a, 0.0, lam0, s)
    X, info = msp.solve(P, A, torch.from_numpy(bm).to(DEV), tol=1e-10, inner_tol=1e-12, level3_tol=1e-12)
    say(info)
    assert info["status"] == "MSP_OK", info
    x = X.cpu().numpy()
    for j in range(k):
        assert np.linalg.norm(a @ x[j] - bm[j]) <= 1e-10 * np.linalg.norm(bm[j])


def test_general_graph_replayed_level3_steps_match_eager():
    # the level-3 step chunks of both product-form solves replayed as graphs (one per
    # operator and chunk length) give the eager solution bit for bit
    say("case general graph-replayed level-3 steps n=400")
    n, k, s = 400, 12, 32
    a, sv, _, _ = W.general_outlier(n, k, config_id=103, big=(1e2, 1e4))
    lam0 = omsp.paper_lambda0(np.sort(sv)[::-1] ** 2, s // 2)
    b = torch.from_numpy(W.gaussian(n, 103)).to(DEV)
    A, P = _gen(a, 0.0, lam0, s)
    out = []
    for g in (0, 1, 0, 1):
        X, info = msp.solve(P, A, b, tol=1e-10, inner_tol=1e-12, level3_tol=1e-12, use_graph=g)
        assert info["status"] == "MSP_OK", info
        out.append((X.cpu().numpy(), info))
    for x, info in out[1:]:
        assert np.array_equal(x, out[0][0])
        assert info["level3_iters"] == out[0][1]["level3_iters"]


@pytest.mark.parametrize("n,s,nrhs", [(400, 32, 1), (1300, 300, 9), (1300, 300, 16)])
def test_two_kernel_level3_steps_match_the_generic_step(n, s, nrhs):
    # the level-3 solves as two kernels per step (direct FP64 row products over the formed
    # A~^T A~ and M3^{-1}) against the generic step kernels: the same iteration, so both
    # converge to the same solution with level-3 counts that differ only by rounding;
    # s = 300 spans two reduction chunks and ends in a partial block of rows
    say(f"case two-kernel level-3 steps n={n} s={s} nrhs={nrhs}")
    a, sv, _, _ = W.general_outlier(n, 12, config_id=109, big=(1e2, 1e4))
    lam0 = omsp.paper_lambda0(np.sort(sv)[::-1] ** 2, s // 2)
    bm = W.gaussian((nrhs, n), 109)
    A, P = _gen(a, 0.0, lam0, s)
    B = torch.from_numpy(bm if nrhs > 1 else bm[0]).to(DEV)
    got = {}
    for l3k in (2, 0, 2):
        X, info = msp.solve(P, A, B, tol=1e-10, inner_tol=1e-12, level3_tol=1e-12, level3_kernels=l3k)
        say(l3k, info)
        assert info["status"] == "MSP_OK", info
        x = X.cpu().numpy().reshape(nrhs, n)
        for j in range(nrhs):
            assert np.linalg.norm(a @ x[j] - bm[j]) <= 1e-10 * np.linalg.norm(bm[j])
        if l3k in got:  # deterministic: the repeated two-kernel solve gives the same bits
            assert np.array_equal(x, got[l3k][0])
        got[l3k] = (x, info)
    x2, i2 = got[2]
    x0, i0 = got[0]
    xs = np.linalg.solve(a, bm.T).T
    for j in range(nrhs):
        assert np.linalg.norm(x2[j] - xs[j]) <= 1e-7 * np.linalg.norm(xs[j])
    assert abs(i2["level3_iters"] - i0["level3_iters"]) <= 0.05 * i0["level3_iters"] + 4
    assert abs(i2["outer_iters"] - i0["outer_iters"]) <= 2


@pytest.mark.parametrize("n,s,nrhs", [(1100, 1025, 8), (2100, 2048, 8), (1700, 1600, 12), (700, 513, 16)])
def test_two_kernel_level3_steps_at_large_s(n, s, nrhs):
    # the two-kernel level-3 step over several 512-column segments: s = 1025 (three segments,
    # the last one column wide, one row per wavefront), s = 2048 (four segments, four rows per
    # wavefront), s = 1600 with 12 right-hand sides (four segments, two rows per wavefront,
    # two passes of 8 and 4 columns) and s = 513 with 16 (a one-column second segment, two
    # full passes), against the generic step; phi = n keeps the matrix small
    say(f"case two-kernel level-3 steps n={n} s={s} k={nrhs}")
    # a milder spread (singular values 1 .. 100) keeps the full solves to seconds
    a, sv, _, _ = W.general_outlier(n, 64, config_id=110, big=(1e1, 1e2))
    lam0 = omsp.paper_lambda0(np.sort(sv)[::-1] ** 2, s // 2)
    bm = W.gaussian((nrhs, n), 110)
    A = torch.from_numpy(a).to(DEV)
    rows, signs, Y = msp.sketch(A, s, 8, 41)
    P = msp.Precond("general", rows, signs, Y, 0.0, lam0, n, 8, 43)
    B = torch.from_numpy(bm).to(DEV)
    xs = {}
    # the first three level-1 steps of both forms: the same iteration, so the same inner and
    # level-3 counts up to rounding
    part = {}
    for l3k in (2, 0):
        X, info = msp.solve(P, A, B, tol=1e-6, inner_tol=1e-10, level3_tol=1e-10, level3_kernels=l3k, max_outer=3)
        say("three steps", l3k, info)
        part[l3k] = info
    assert abs(part[2]["level3_iters"] - part[0]["level3_iters"]) <= 0.02 * part[0]["level3_iters"] + 4
    assert abs(part[2]["inner_iters"] - part[0]["inner_iters"]) <= 2
    for l3k in (2, 0):
        X, info = msp.solve(P, A, B, tol=1e-6, inner_tol=1e-10, level3_tol=1e-10, level3_kernels=l3k)
        say(l3k, info)
        assert info["status"] == "MSP_OK", info
        x = X.cpu().numpy()
        for j in range(nrhs):
            assert np.linalg.norm(a @ x[j] - bm[j]) <= 1e-6 * (1 + 1e-6) * np.linalg.norm(bm[j])
        xs[l3k] = (x, info)
    # both residuals are at most 1e-6 |b|, so the solutions differ by at most 2e-6 |b| / sigma_min
    for j in range(nrhs):
        assert np.linalg.norm(xs[2][0][j] - xs[0][0][j]) <= 2.02e-6 * np.linalg.norm(bm[j]) / sv.min()
    assert abs(xs[2][1]["outer_iters"] - xs[0][1]["outer_iters"]) <= 2
    assert xs[2][1]["level3_iters"] > 0


def test_refinement_stops_on_a_stall():
    # kappa(A) ~ 1e6 (so kappa(A)^4 is far beyond FP64) with an FP32 copy inside MSP and the
    # one-level form, whose explicit level-2 matrix B^T B loses the small directions: the
    # refinement either converges or stops with the best iterate within a few steps (a
    # stall is two steps that fail to halve the residual; the one-level form has no inner
    # level to tighten, so it stops at the first stall)
    form = 2
    say(f"case general refinement stall n=512 level2_form={form}")
    n, s = 512, 64
    a, sv, _, _ = W.general_outlier(n, 16, config_id=108)
    lam0 = omsp.paper_lambda0(np.sort(sv)[::-1] ** 2, s // 2)
    b = W.gaussian(n, 108)
    A = torch.from_numpy(a).to(DEV)
    A32 = A.float()
    rows, signs, Y = msp.sketch(A32, s, 8, 41)
    P = msp.Precond("general", rows, signs, Y, 0.0, lam0, 4 * s, 8, 43)
    tol = 1e-11
    X, info = msp.solve(P, A, torch.from_numpy(b).to(DEV), A_lo=A32, refine=1, tol=tol, level2_form=form,
                        max_outer=20000, max_refine=30)
    say(info)
    assert info["code"] in ("MSP_OK", "MSP_ERR_NO_CONVERGENCE"), info
    assert info["refine_steps"] <= 12, info
    x = X.cpu().numpy()
    bn = np.linalg.norm(b)
    host = np.linalg.norm(b - a @ x) / bn
    # the two FP64 residuals differ by rounding: n eps (|A| |x| + |b|) relative to |b|
    floor = n * np.finfo(np.float64).eps * np.linalg.norm(np.abs(a) @ np.abs(x) + np.abs(b)) / bn
    say(f"host {host:.3e} library {info['rel_residual_max']:.3e} rounding floor {floor:.1e}")
    assert np.isfinite(host) and host < 1.0
    assert abs(info["rel_residual_max"] - host) <= 1e-8 * host + floor
    if info["code"] == "MSP_OK":
        assert host <= tol + floor


def test_refinement_level1_budget_across_steps():
    # max_outer caps the level-1 steps of all inner solves of one refined solve together
    say("case general refinement budget n=512")
    n, s = 512, 64
    a, sv, _, _ = W.general_outlier(n, 16, config_id=108)
    lam0 = omsp.paper_lambda0(np.sort(sv)[::-1] ** 2, s // 2)
    b = W.gaussian(n, 108)
    A = torch.from_numpy(a).to(DEV)
    A32 = A.float()
    rows, signs, Y = msp.sketch(A32, s, 8, 41)
    P = msp.Precond("general", rows, signs, Y, 0.0, lam0, 4 * s, 8, 43)
    X, info = msp.solve(P, A, torch.from_numpy(b).to(DEV), A_lo=A32, refine=1, tol=1e-14, max_outer=7)
    say(info)
    assert info["code"] == "MSP_ERR_NO_CONVERGENCE", info
    assert info["outer_iters"] <= 7
