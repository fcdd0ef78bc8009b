"""GPU parity of the two-level PSD path (Algorithms 1-2) against the FP64 oracle.

Every case prints its name before touching the GPU. Inputs come from `workloads`;
expected values come from `oracle` only.
"""
import numpy as np
import pytest
import torch

import paper_2405_05865_amd as msp
import workloads as W
from oracle import dense, rng, sketch as osk
from oracle import msp as omsp

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")
EPS = np.finfo(np.float64).eps


def say(*a):
    print(*a, flush=True)


def _abs_sketch(a, rows, s):
    """sum_i |A[r, i]| |S[j, i]|: the scale of the rounding error of Y[r, j]."""
    return osk.right_sketch(np.abs(a), rows, np.ones_like(rows, dtype=np.int8), s)


@pytest.mark.parametrize("m,n,s,gamma,seed", [(1000, 1000, 64, 8, 5), (777, 777, 50, 3, 6), (300, 300, 300, 1, 8),
                                              (130, 2100, 200, 8, 9), (4096, 4096, 512, 8, 7)])
def test_sketch_bitwise_indices_and_values(m, n, s, gamma, seed):
    say(f"case sketch m={m} n={n} s={s} gamma={gamma}")
    a = np.random.default_rng(seed).standard_normal((m, n))
    A = torch.from_numpy(a).to(DEV)
    rows, signs, Y = msp.sketch(A, s, gamma, seed)
    r_o, s_o = rng.sketch_indices(seed, n, s, gamma)
    assert np.array_equal(rows.cpu().numpy(), r_o)
    assert np.array_equal(signs.cpu().numpy(), s_o)
    y_o = osk.right_sketch(a, r_o, s_o, s)
    bound = 64 * EPS * _abs_sketch(a, r_o, s) + 1e-300
    assert np.all(np.abs(Y.cpu().numpy() - y_o) <= bound)


@pytest.mark.parametrize("dt", [torch.float32, torch.bfloat16])
def test_sketch_low_precision(dt):
    say(f"case sketch dtype={dt}")
    m, n, s, gamma, seed = 513, 1030, 128, 8, 3
    a = np.random.default_rng(1).standard_normal((m, n))
    A = torch.from_numpy(a).to(DEV).to(dt)
    a_lo = A.float().cpu().double().numpy()   # the stored values
    rows, signs, Y = msp.sketch(A, s, gamma, seed)
    assert Y.dtype == torch.float32
    r_o, s_o = rng.sketch_indices(seed, n, s, gamma)
    y_o = osk.right_sketch(a_lo, r_o, s_o, s)
    bound = 64 * np.finfo(np.float32).eps * _abs_sketch(a_lo, r_o, s)
    assert np.all(np.abs(Y.cpu().double().numpy() - y_o) <= bound)


def _psd_case(n, k, s, cid, lam):
    a, eigs, _ = W.psd_outlier(n, k, config_id=cid)
    return a, eigs, msp_lam0(eigs, s)


def msp_lam0(eigs, s):
    return omsp.paper_lambda0(eigs, s // 2)


def test_nystrom_factors_match_oracle():
    say("case nystrom factors n=1024 s=64")
    n, s, lam = 1024, 64, 1e-3
    a, eigs, lam0 = _psd_case(n, 32, s, 0, lam)
    A = torch.from_numpy(a).to(DEV)
    rows, signs, Y = msp.sketch(A, s, 8, 101)
    P = msp.Precond("psd", rows, signs, Y, lam, lam0, 4 * s, 8, 102)
    Wg, Mi, _ = P.factors()
    O = omsp.PsdMsp(a, lam, lam0, s, 8, 101, 4 * s, 8, 102)
    w_o = O.w
    assert np.linalg.norm(Wg.cpu().numpy() - w_o) <= 1e-13 * np.linalg.norm(w_o)
    # the GPU and the oracle form M2 from Y with different summation orders; that
    # relative perturbation (well below 1e-12) is amplified by kappa(M2) in the inverse
    kappa = np.linalg.cond(O.m2)
    mi = Mi.cpu().numpy()
    assert np.linalg.norm(mi - O.m2inv) <= kappa * 1e-12 * np.linalg.norm(O.m2inv)
    assert np.array_equal(mi, mi.T)


def _solve_case(n, k, s, cid, lam, tol, inner_tol, b=None, seeds=(11, 12), **opts):
    a, eigs, lam0 = _psd_case(n, k, s, cid, lam)
    if b is None:
        b = W.gaussian(n, cid)
    A = torch.from_numpy(a).to(DEV)
    bt = torch.from_numpy(np.ascontiguousarray(b)).to(DEV)
    rows, signs, Y = msp.sketch(A, s, 8, seeds[0])
    P = msp.Precond("psd", rows, signs, Y, lam, lam0, 4 * s, 8, seeds[1])
    X, info = msp.solve(P, A, bt, tol=tol, inner_tol=inner_tol, **opts)
    return a, eigs, lam0, b, X.cpu().numpy(), info, P, A


@pytest.mark.parametrize("form", [0, 1, 2])
def test_solve_outlier_n1024_matches_dense_and_oracle_iterations(form):
    # the plain MSP regularized solve: n = 1024, 32 outliers, lam = 1e-3, tol 1e-10; the
    # level-2 operator through the sketch (form 0) or through C^T C + lam~ W (form 1)
    say(f"case solve psd_outlier n=1024 level2_form={form}")
    w = W.config("psd_outlier_n1024")
    a, eigs, lam0, b, x, info, _, _ = _solve_case(w.n, 32, w.s, w.config_id, w.lam, w.tol, 1e-12,
                                                  seeds=(w.seed_s, w.seed_phi), level2_form=form)
    assert info["status"] == "MSP_OK", info
    xs = dense.solve_psd(a, b, w.lam)
    assert dense.rel_residual_psd(a, x, b, w.lam) <= w.tol
    assert np.linalg.norm(x - xs) <= 1e-7 * np.linalg.norm(xs)
    O = omsp.PsdMsp(a, w.lam, lam0, w.s, w.gamma, w.seed_s, w.phi, w.phi_gamma, w.seed_phi,
                    omsp.MspOptions(tol=w.tol, inner_tol=1e-12))
    O.solve(b)
    say("gpu", info["outer_iters"], info["inner_iters"], "oracle", O.info.outer_iterations, O.info.inner_iterations)
    assert abs(info["outer_iters"] - O.info.outer_iterations) <= 2


def test_solve_rbf_shape_n4096():
    # the GP-regression shape at n/8: RBF kernel over N(0, I_8) points, s/n = 1/64
    say("case solve rbf n=4096 s=64")
    w = W.config("rbf_gp_n32768", n=4096, s=64)
    pts = W.rbf_points(w.n, 8, w.config_id)
    a = W.rbf_matrix(pts)
    eigs = np.linalg.eigvalsh(a)[::-1]
    lam0 = omsp.paper_lambda0(eigs, w.l)
    b = W.gaussian(w.n, w.config_id)
    A = torch.from_numpy(a).to(DEV)
    rows, signs, Y = msp.sketch(A, w.s, w.gamma, w.seed_s)
    P = msp.Precond("psd", rows, signs, Y, w.lam, lam0, w.phi, w.phi_gamma, w.seed_phi)
    X, info = msp.solve(P, A, torch.from_numpy(b).to(DEV), tol=w.tol, inner_tol=1e-10)
    x = X.cpu().numpy()
    assert info["status"] == "MSP_OK", info
    assert dense.rel_residual_psd(a, x, b, w.lam) <= w.tol
    xs = dense.solve_psd(a, b, w.lam)
    assert np.linalg.norm(x - xs) <= 1e-7 * np.linalg.norm(xs)
    O = omsp.PsdMsp(a, w.lam, lam0, w.s, w.gamma, w.seed_s, w.phi, w.phi_gamma, w.seed_phi,
                    omsp.MspOptions(tol=w.tol, inner_tol=1e-10))
    O.solve(b)
    say("gpu", info["outer_iters"], "oracle", O.info.outer_iterations)
    assert abs(info["outer_iters"] - O.info.outer_iterations) <= max(2, 0.02 * O.info.outer_iterations)


def test_multi_rhs_ragged_with_zero_column():
    say("case solve multi-rhs n=1001 s=48 k=3")
    n, k, s, lam = 1001, 10, 48, 1e-2
    a, eigs, lam0 = _psd_case(n, k, s, 300, lam)
    bm = W.gaussian((3, n), 300)
    bm[1] = 0.0
    A = torch.from_numpy(a).to(DEV)
    rows, signs, Y = msp.sketch(A, s, 8, 31)
    P = msp.Precond("psd", rows, signs, Y, lam, lam0, 4 * s, 8, 32)
    X, info = msp.solve(P, A, torch.from_numpy(bm).to(DEV), tol=1e-10, inner_tol=1e-12)
    x = X.cpu().numpy()
    assert info["status"] == "MSP_OK", info
    assert np.all(x[1] == 0.0)
    for j in (0, 2):
        xs = dense.solve_psd(a, bm[j], lam)
        assert np.linalg.norm(x[j] - xs) <= 1e-8 * np.linalg.norm(xs)
    # the same columns solved one at a time give the same answers
    X0, _ = msp.solve(P, A, torch.from_numpy(bm[0].copy()).to(DEV), tol=1e-10, inner_tol=1e-12)
    assert np.linalg.norm(X0.cpu().numpy() - x[0]) <= 1e-9 * np.linalg.norm(x[0])


def test_deterministic():
    say("case determinism n=1024")
    n, s, lam = 1024, 64, 1e-3
    a, eigs, lam0 = _psd_case(n, 32, s, 0, lam)
    A = torch.from_numpy(a).to(DEV)
    b = torch.from_numpy(W.gaussian(n, 0)).to(DEV)
    outs = []
    for _ in range(2):
        rows, signs, Y = msp.sketch(A, s, 8, 5)
        P = msp.Precond("psd", rows, signs, Y, lam, lam0, 4 * s, 8, 6)
        X, _ = msp.solve(P, A, b, tol=1e-10, inner_tol=1e-12)
        outs.append((Y.cpu().numpy(), X.cpu().numpy()))
    assert np.array_equal(outs[0][0], outs[1][0]) and np.array_equal(outs[0][1], outs[1][1])


def test_set_lambda_refactors():
    say("case set_lambda n=512")
    n, s = 512, 32
    a, eigs, lam0 = _psd_case(n, 16, s, 301, 1e-3)
    A = torch.from_numpy(a).to(DEV)
    b = W.gaussian(n, 301)
    rows, signs, Y = msp.sketch(A, s, 8, 7)
    P = msp.Precond("psd", rows, signs, Y, 1e-3, lam0, 4 * s, 8, 8)
    P.set_lambda(0.5)
    X, info = msp.solve(P, A, torch.from_numpy(b).to(DEV), tol=1e-10, inner_tol=1e-12)
    xs = dense.solve_psd(a, b, 0.5)
    assert np.linalg.norm(X.cpu().numpy() - xs) <= 1e-8 * np.linalg.norm(xs)


def test_iteration_cap_reports_no_convergence():
    say("case cap n=512")
    n, s = 512, 32
    a, eigs, lam0 = _psd_case(n, 16, s, 302, 1e-3)
    A = torch.from_numpy(a).to(DEV)
    rows, signs, Y = msp.sketch(A, s, 8, 9)
    P = msp.Precond("psd", rows, signs, Y, 1e-3, lam0, 4 * s, 8, 10)
    X, info = msp.solve(P, A, torch.from_numpy(W.gaussian(n, 302)).to(DEV), tol=1e-12, max_outer=3)
    assert info["code"] == "MSP_ERR_NO_CONVERGENCE"
    assert info["outer_iters"] == 3


@pytest.mark.parametrize("k", [20, 40])
def test_block_rhs_matrix_core_sweep_f64(k):
    # k >= 8 right-hand sides take the matrix-core block sweep; ragged n, a zero column
    say(f"case block rhs f64 n=777 k={k}")
    n, s, lam = 777, 48, 1e-2
    a, eigs, lam0 = _psd_case(n, 10, s, 310, lam)
    bm = W.gaussian((k, n), 310)
    bm[3] = 0.0
    A = torch.from_numpy(a).to(DEV)
    rows, signs, Y = msp.sketch(A, s, 8, 33)
    P = msp.Precond("psd", rows, signs, Y, lam, lam0, 4 * s, 8, 34)
    X, info = msp.solve(P, A, torch.from_numpy(bm).to(DEV), tol=1e-10, inner_tol=1e-12)
    say(info)
    assert info["status"] == "MSP_OK", info
    x = X.cpu().numpy()
    assert np.all(x[3] == 0.0)
    for j in range(k):
        if j == 3:
            continue
        assert dense.rel_residual_psd(a, x[j], bm[j], lam) <= 1e-10
        xs = dense.solve_psd(a, bm[j], lam)
        assert np.linalg.norm(x[j] - xs) <= 1e-8 * np.linalg.norm(xs)


@pytest.mark.parametrize("dt", [torch.float32, torch.bfloat16])
def test_block_rhs_low_precision_refined(dt):
    # F32 / BF16 block sweeps inside MSP, FP64 residuals on the FP64 matrix (k >= 8)
    say(f"case block rhs refine {dt} n=640 k=12")
    n, s, k = 640, 48, 12
    lam = 1e-2 if dt == torch.float32 else 0.5
    a, eigs, lam0 = _psd_case(n, 10, s, 320, lam)
    bm = W.gaussian((k, n), 320)
    A = torch.from_numpy(a).to(DEV)
    A_lo = A.to(dt)
    rows, signs, Y = msp.sketch(A.float(), s, 8, 35)
    P = msp.Precond("psd", rows, signs, Y, lam, lam0, 4 * s, 8, 36)
    X, info = msp.solve(P, A, torch.from_numpy(bm).to(DEV), A_lo=A_lo, refine=1, tol=1e-10)
    say(info)
    assert info["status"] == "MSP_OK", info
    x = X.cpu().numpy()
    for j in range(k):
        assert dense.rel_residual_psd(a, x[j], bm[j], lam) <= 1e-10


@pytest.mark.parametrize("n,pad", [(1000, 0), (1000, 2), (1000, 1), (513, 3), (256, 0)])
def test_lower_triangle_sweep(n, pad):
    # the level-1 sweep of a symmetric A from its lower triangle (256 x 256 tiles): ragged
    # n, padded leading dimensions; an FP64 lda that is not a multiple of two elements is
    # not 16-byte aligned and takes the full sweep instead. Both sweeps must give the
    # dense solution, and the triangle sweep streams n(n+1)/2 elements per level-1 sweep.
    say(f"case lower-triangle sweep n={n} pad={pad}")
    s, lam, tol = 64, 1e-3, 1e-10
    a, eigs, lam0 = _psd_case(n, 32, s, 3, lam)
    b = W.gaussian(n, 3)
    big = torch.zeros((n, n + pad), dtype=torch.float64, device=DEV)
    big[:, :n] = torch.from_numpy(a).to(DEV)
    if pad:
        big[:, n:] = float("nan")  # padding must never be read
    A = big[:, :n]
    bt = torch.from_numpy(b).to(DEV)
    rows, signs, Y = msp.sketch(A, s, 8, 41)
    P = msp.Precond("psd", rows, signs, Y, lam, lam0, 4 * s, 8, 42)
    xs = dense.solve_psd(a, b, lam)
    res = {}
    for sym in (1, 0):
        X, info = msp.solve(P, A, bt, tol=tol, inner_tol=1e-12, sym_sweep=sym)
        x = X.cpu().numpy()
        assert info["status"] == "MSP_OK", info
        assert dense.rel_residual_psd(a, x, b, lam) <= tol
        assert np.linalg.norm(x - xs) <= 1e-7 * np.linalg.norm(xs)
        res[sym] = info
    aligned = ((n + pad) * 8) % 16 == 0
    full = res[1]["sweeps"] * float(n) * n * 8
    if aligned:
        assert res[1]["sweep_bytes"] < 0.6 * full
    else:
        assert res[1]["sweep_bytes"] == full
    assert abs(res[1]["outer_iters"] - res[0]["outer_iters"]) <= 2
    P.close()


def test_lower_triangle_sweep_refined_f32():
    # the FP32 A_lo sweep from its lower triangle inside FP64 refinement
    say("case lower-triangle sweep f32 refinement n=1000")
    n, s, lam, tol = 1000, 64, 1e-2, 1e-10
    a, eigs, lam0 = _psd_case(n, 32, s, 4, lam)
    b = W.gaussian(n, 4)
    A = torch.from_numpy(a).to(DEV)
    A32 = A.float()
    rows, signs, Y = msp.sketch(A32, s, 8, 43)
    P = msp.Precond("psd", rows, signs, Y, lam, lam0, 4 * s, 8, 44)
    X, info = msp.solve(P, A, torch.from_numpy(b).to(DEV), A_lo=A32, refine=1, tol=tol, sym_sweep=1)
    x = X.cpu().numpy()
    assert info["status"] == "MSP_OK", info
    assert dense.rel_residual_psd(a, x, b, lam) <= tol
    xs = dense.solve_psd(a, b, lam)
    assert np.linalg.norm(x - xs) <= 1e-7 * np.linalg.norm(xs)
    P.close()


def test_graph_replayed_inner_steps_match_eager():
    # the predicted inner steps of every SolveM1 call as one replayed HIP graph: the same
    # kernels in the same order, so the solution is bitwise the eager one; the graph is
    # replayed hundreds of times per solve with eager kernels and host syncs in between,
    # and a second solve in a row replays fresh graphs
    say("case graph-replayed inner steps n=1024")
    w = W.config("psd_outlier_n1024")
    runs = []
    for g in (0, 1, 1, 0):
        a, eigs, lam0, b, x, info, P, _ = _solve_case(w.n, 32, w.s, w.config_id, w.lam, w.tol, 1e-12,
                                                      seeds=(w.seed_s, w.seed_phi), use_graph=g)
        assert info["status"] == "MSP_OK", info
        runs.append((x, info))
        P.close()
    for x, info in runs[1:]:
        assert np.array_equal(x, runs[0][0])
        assert info["outer_iters"] == runs[0][1]["outer_iters"]
        assert info["inner_iters"] == runs[0][1]["inner_iters"]


@pytest.mark.parametrize("case", ["outlier", "rbf", "bf16"])
def test_lambda0_estimator_matches_oracle(case):
    # lambda0 < 0: the GPU estimates lam0 = (2/l) max(tr A - tr(W^+ C^T C), 0) from the
    # handle's sketch and A's diagonal; the oracle's estimator on the same sketch
    say(f"case lambda0 estimator {case}")
    if case == "outlier":
        n, s, lam = 1024, 64, 1e-3
        a, eigs, _ = W.psd_outlier(n, 32, config_id=0)
    else:
        n, s, lam = 2048, 128, 1e-2
        a = W.rbf_matrix(W.rbf_points(n, 8, 11))
    A = torch.from_numpy(a).to(DEV)
    A_sk = A.to(torch.bfloat16) if case == "bf16" else A
    rows, signs, Y = msp.sketch(A_sk, s, 8, 31)
    P = msp.Precond("psd", rows, signs, Y, lam, None, 4 * s, 8, 32, A=A_sk)
    a_sk = A_sk.double().cpu().numpy()
    r_o, s_o = rng.sketch_indices(31, n, s, 8)
    c = osk.right_sketch(a_sk, r_o, s_o, s)
    w = osk.left_sketch(r_o, s_o, s, c)
    want = omsp.lambda0_estimate(a_sk, c, w, s // 2)
    scale = 2.0 / (s // 2) * float(np.trace(a_sk))
    tol = (1e-9 if case != "bf16" else 1e-5) * scale  # BF16: the FP32 sketch's rounding
    say(f"gpu lam0 {P.lam0:.12e} oracle {want:.12e}")
    assert abs(P.lam0 - want) <= tol
    if case == "outlier":
        b = W.gaussian(n, 0)
        X, info = msp.solve(P, A, torch.from_numpy(b).to(DEV), tol=1e-10, inner_tol=1e-12)
        assert info["status"] == "MSP_OK", info
        assert dense.rel_residual_psd(a, X.cpu().numpy(), b, lam) <= 1e-10


def test_lambda0_estimator_low_rank_needs_lambda():
    # rank(A) <= s: the estimate is 0; with lam = 0 there is no regulariser left
    say("case lambda0 estimator low rank")
    n, r, s = 300, 20, 32
    g = np.random.default_rng(3).standard_normal((n, r))
    A = torch.from_numpy(g @ g.T).to(DEV)
    rows, signs, Y = msp.sketch(A, s, 8, 5)
    P = msp.Precond("psd", rows, signs, Y, 1e-2, None, 4 * s, 8, 6, A=A)
    assert P.lam0 == 0.0
    with pytest.raises(msp.MspError) as e:
        msp.Precond("psd", rows, signs, Y, 0.0, None, 4 * s, 8, 6, A=A)
    assert e.value.status == "MSP_ERR_INVALID_ARG"
