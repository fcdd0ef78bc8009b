"""GPU parity of the batched solve (one launch for many PSD systems of uneven size)
against dense LAPACK solves and the oracle's two-level iteration counts."""
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


def _system(n, cid, lam=1e-2, dtype=np.float64, lengthscale=1.0, seeds=(11, 12)):
    """One RBF kernel system of the batched-GP shape (points in 4 dimensions)."""
    pts = W.rbf_points(n, 4, cid)
    a = W.rbf_matrix(pts, lengthscale=lengthscale, dtype=dtype)
    a64 = a.astype(np.float64)
    s = max(8, min(64, n // 2))
    lam0 = omsp.paper_lambda0(np.linalg.eigvalsh(a64)[::-1], s // 2)
    return dict(n=n, a=a, a64=a64, s=s, phi=min(4 * s, n), lam=lam, lam0=lam0, seeds=(seeds[0] + cid, seeds[1] + cid))


def _padded(a, dt, pad):
    """Device copy of a with leading dimension n + pad (row-major view of a wider buffer)."""
    n = a.shape[0]
    buf = torch.zeros((n, n + pad), dtype=dt, device=DEV)
    buf[:, :n] = torch.from_numpy(a).to(DEV).to(dt)
    return buf[:, :n]


def _build(sy, A, y_dtype=None):
    rows, signs, Y = msp.sketch(A, sy["s"], 8, sy["seeds"][0], y_dtype=y_dtype)
    return msp.Precond("psd", rows, signs, Y, sy["lam"], sy["lam0"], sy["phi"], 8, sy["seeds"][1])


def test_batched_f64_matches_dense_and_oracle():
    sizes = [130, 257, 400, 64, 515, 333, 97]
    k = 3
    say(f"case batched f64 sizes={sizes} k={k}")
    syss, args, Bs = [], [], []
    for i, n in enumerate(sizes):
        sy = _system(n, 500 + i, lengthscale=0.5 + 0.25 * i)
        A = _padded(sy["a"], torch.float64, pad=i % 3)
        P = _build(sy, A)
        Bm = W.gaussian((k, n), 500 + i)
        Bm[1] = 0.0  # a zero right-hand side
        syss.append((sy, P))
        Bs.append(Bm)
        args.append((P, A, None, torch.from_numpy(Bm).to(DEV)))
    Xs, infos = msp.solve_batched(args, tol=1e-10, inner_tol=1e-10)
    for (sy, P), Bm, X, info in zip(syss, Bs, Xs, infos):
        say(sy["n"], info["status"], info["outer_iters"], info["inner_iters"], info["rel_residual_max"])
        assert info["status"] == "MSP_OK", info
        x = X.cpu().numpy()
        assert np.all(x[1] == 0.0)
        for j in (0, 2):
            assert dense.rel_residual_psd(sy["a64"], x[j], Bm[j], sy["lam"]) <= 1e-10
            xs = dense.solve_psd(sy["a64"], Bm[j], sy["lam"])
            assert np.linalg.norm(x[j] - xs) <= 1e-7 * np.linalg.norm(xs)
        # level-1 steps: the oracle's two-level solve on the same sketches, per column
        O = omsp.PsdMsp(sy["a64"], sy["lam"], sy["lam0"], sy["s"], 8, sy["seeds"][0], sy["phi"], 8, sy["seeds"][1],
                        omsp.MspOptions(tol=1e-10, inner_tol=1e-10))
        its = []
        for j in (0, 2):
            O.solve(Bm[j])
            its.append(O.info.outer_iterations)
        assert abs(info["outer_iters"] - max(its)) <= max(2, 0.03 * max(its)), (info["outer_iters"], its)


@pytest.mark.parametrize("lo,hi", [(torch.float32, torch.float32), (torch.bfloat16, torch.float32),
                                   (torch.float32, torch.float64), (torch.bfloat16, torch.float64)])
def test_batched_low_precision_refined(lo, hi):
    sizes = [300, 96, 513, 200]
    k = 4
    say(f"case batched refine lo={lo} hi={hi}")
    syss, args, Bs = [], [], []
    for i, n in enumerate(sizes):
        # BF16 sweeps pay off only where lam dominates the rounding perturbation of A
        lam = 0.5 if lo == torch.bfloat16 else 1e-2
        sy = _system(n, 600 + i, lam=lam, dtype=np.float32, lengthscale=1.0 + 0.3 * i)
        A_hi = _padded(sy["a"], hi, pad=(8 if i % 2 else 0))
        A_lo = torch.empty_strided(A_hi.shape, A_hi.stride(), dtype=lo, device=DEV)
        A_lo.copy_(A_hi)
        # the preconditioner comes from the problem matrix (BF16 rounding is not PSD);
        # the low-precision copy is what the inner MSP sweeps
        P = _build(sy, torch.from_numpy(sy["a"]).to(DEV))
        Bm = W.gaussian((k, n), 600 + i)
        syss.append(sy)
        Bs.append(Bm)
        args.append((P, A_hi, A_lo, torch.from_numpy(Bm).to(DEV)))
    Xs, infos = msp.solve_batched(args, tol=1e-8, refine=1)
    for sy, Bm, X, info in zip(syss, Bs, Xs, infos):
        say(sy["n"], info)
        assert info["status"] == "MSP_OK", info
        x = X.cpu().numpy()
        for j in range(k):
            assert dense.rel_residual_psd(sy["a64"], x[j], Bm[j], sy["lam"]) <= 1e-8
        assert info["refine_steps"] >= 1


def test_batched_bf16_sweeps_at_the_workload_lambda():
    # the BF16 sweep variant of the batched GP workload at its own lam = 1e-2 (RBF kernels in
    # 4 dimensions, the F32 matrix is the problem): BF16 rounding moves A by far more than
    # lam, so the refinement runs Krylov steps around the BF16 solves; every system must still
    # reach a relative residual of 1e-8 on the F32 matrix, and x is compared with the dense
    # FP64 solution of that matrix
    sizes = [300, 96, 513, 200]
    k = 4
    say("case batched bf16 sweeps lam=1e-2")
    syss, args, Bs = [], [], []
    for i, n in enumerate(sizes):
        sy = _system(n, 650 + i, lam=1e-2, dtype=np.float32, lengthscale=0.5 + 0.5 * i)
        A_hi = _padded(sy["a"], torch.float32, pad=(8 if i % 2 else 0))
        A_lo = torch.empty_strided(A_hi.shape, A_hi.stride(), dtype=torch.bfloat16, device=DEV)
        A_lo.copy_(A_hi)
        P = _build(sy, torch.from_numpy(sy["a"]).to(DEV))
        Bm = W.gaussian((k, n), 650 + i)
        syss.append(sy)
        Bs.append(Bm)
        args.append((P, A_hi, A_lo, torch.from_numpy(Bm).to(DEV)))
    # the Krylov refinement takes tens of steps here (30 is the default cap)
    Xs, infos = msp.solve_batched(args, tol=1e-8, refine=1, max_refine=300)
    for sy, Bm, X, info in zip(syss, Bs, Xs, infos):
        say(sy["n"], info)
        assert info["status"] == "MSP_OK", info
        x = X.cpu().numpy()
        xs = dense.solve_psd(sy["a64"], Bm.T, sy["lam"]).T
        err = max(np.linalg.norm(x[j] - xs[j]) / np.linalg.norm(xs[j]) for j in range(k))
        say(f"n={sy['n']}: max_j |x - x*| / |x*| = {err:.3e}")
        for j in range(k):
            rel = dense.rel_residual_psd(sy["a64"], x[j], Bm[j], sy["lam"])
            assert rel <= 1e-8 * (1 + 1e-6)
            # A + lam I >= lam I: the forward error the residual allows
            assert np.linalg.norm(x[j] - xs[j]) <= 1.01 * rel * np.linalg.norm(Bm[j]) / sy["lam"] + 1e-10 * np.linalg.norm(xs[j])


def test_batched_deterministic_and_chunks_of_16():
    sizes = [150, 77, 260]
    k = 20  # two launches: 16 + 4 right-hand sides
    say(f"case batched determinism k={k}")
    args, syss = [], []
    for i, n in enumerate(sizes):
        sy = _system(n, 700 + i)
        A = torch.from_numpy(sy["a"]).to(DEV)
        P = _build(sy, A)
        syss.append(sy)
        args.append((P, A, None, torch.from_numpy(W.gaussian((k, n), 700 + i)).to(DEV)))
    X1, i1 = msp.solve_batched(args, tol=1e-9)
    X2, i2 = msp.solve_batched(args, tol=1e-9)
    for a_, b_, inf in zip(X1, X2, i1):
        assert inf["status"] == "MSP_OK", inf
        assert torch.equal(a_, b_)
    for (P, A, _, Bv), X, sy in zip(args, X1, syss):
        x = X.cpu().numpy()
        b = Bv.cpu().numpy()
        for j in range(k):
            assert dense.rel_residual_psd(sy["a64"], x[j], b[j], sy["lam"]) <= 1e-9


def test_batched_iteration_cap_reports_no_convergence():
    say("case batched cap")
    sy = _system(300, 800)
    A = torch.from_numpy(sy["a"]).to(DEV)
    P = _build(sy, A)
    Bv = torch.from_numpy(W.gaussian((2, 300), 800)).to(DEV)
    _, infos = msp.solve_batched([(P, A, None, Bv)], tol=1e-12, max_outer=2)
    assert infos[0]["status"] == "MSP_ERR_NO_CONVERGENCE"


@pytest.mark.parametrize("lo", [None, torch.float32])
def test_batched_adjoint_matches_dense_gradients(lo):
    # forward plus adjoint of the batched GP solves under L = sum_i |X_i|_F^2: G_i = 2 X_i,
    # dB_i = (A_i + lam I)^{-1} G_i, dlam_i = -sum_j <dB_ij, X_ij>, dA_i = -dB_i X_i^T
    sizes = [300, 517, 128, 1024]
    k = 4
    say(f"case batched adjoint sizes={sizes} k={k} lo={lo}")
    args, syss = [], []
    for i, n in enumerate(sizes):
        if lo is None:
            sy = _system(n, 700 + i, lengthscale=0.6 + 0.3 * i)
            A = _padded(sy["a"], torch.float64, pad=(i % 2) * 2)
            A_lo, P = None, _build(sy, A)
        else:
            sy = _system(n, 700 + i, lengthscale=0.6 + 0.3 * i, dtype=np.float32)
            A = _padded(sy["a"], torch.float32, pad=(i % 2) * 4)
            A_lo, P = A, _build(sy, A, y_dtype=torch.float32)
        Bm = W.gaussian((k, n), 700 + i)
        syss.append((sy, Bm))
        args.append((P, A, A_lo, torch.from_numpy(Bm).to(DEV)))
    opts = dict(tol=1e-10, inner_tol=1e-10)
    if lo is not None:
        opts.update(refine=1)
    Xs, infos = msp.solve_batched(args, **opts)
    assert all(i["status"] == "MSP_OK" for i in infos), infos
    Gs = [2.0 * X for X in Xs]
    dBs, dlams, dAs, binfos = msp.solve_batched_backward(args, Xs, Gs, want_dA=True, **opts)
    for (sy, Bm), X, dB, dl, dA, info in zip(syss, Xs, dBs, dlams, dAs, binfos):
        say(sy["n"], info["status"], info["outer_iters"], info["rel_residual_max"], dl)
        assert info["status"] == "MSP_OK", info
        a, lam = sy["a64"], sy["lam"]
        xd = np.stack([dense.solve_psd(a, Bm[j], lam) for j in range(k)])
        gd = 2.0 * xd
        dbd = np.stack([dense.solve_psd(a, gd[j], lam) for j in range(k)])
        dbg = dB.cpu().numpy()
        for j in range(k):
            assert np.linalg.norm(dbg[j] - dbd[j]) <= 1e-7 * np.linalg.norm(dbd[j])
        dld = -float(np.sum(dbd * xd))
        assert abs(dl - dld) <= 1e-7 * abs(dld)
        dad = -dbd.T @ xd
        assert np.linalg.norm(dA.cpu().numpy() - dad) <= 1e-7 * np.linalg.norm(dad)
        # dlam against a central difference of L(lam) = sum |(A + lam I)^{-1} B|^2
        h = 1e-5 * lam
        lp = sum(np.sum(dense.solve_psd(a, Bm[j], lam + h) ** 2) for j in range(k))
        lm = sum(np.sum(dense.solve_psd(a, Bm[j], lam - h) ** 2) for j in range(k))
        assert abs(dl - (lp - lm) / (2 * h)) <= 1e-5 * abs(dld)


def test_batched_teams_same_bits_as_single_workgroups():
    # finished workgroups help the A-sweeps of the larger systems (row chunks with their
    # own partials, summed in chunk order): the solutions are the same bits as without
    # helpers, for several launches in a row
    sizes = [3000, 2600, 2100, 300, 200, 180, 160, 150, 140, 130, 120, 110]
    k = 4
    say(f"case batched teams sizes={sizes} k={k}")
    args, syss = [], []
    for i, n in enumerate(sizes):
        sy = _system(n, 900 + i, lengthscale=0.7 + 0.1 * i, dtype=np.float32)
        A = _padded(sy["a"], torch.float32, pad=(i % 2) * 4)
        P = _build(sy, A, y_dtype=torch.float32)
        Bm = W.gaussian((k, n), 900 + i)
        syss.append(sy)
        args.append((P, A, A, torch.from_numpy(Bm).to(DEV)))
    runs = []
    for teams in (0, 1, 1, 0):
        Xs, infos = msp.solve_batched(args, tol=1e-10, refine=1, batch_teams=teams)
        assert all(d["status"] == "MSP_OK" for d in infos), infos
        runs.append([X.cpu().numpy() for X in Xs])
    for r in runs[1:]:
        for x0, x1 in zip(runs[0], r):
            assert np.array_equal(x0, x1)
    for sy, x, (_, _, _, Bt) in zip(syss, runs[1], args):
        Bm = Bt.cpu().numpy()
        for j in range(k):
            assert dense.rel_residual_psd(sy["a64"], x[j], Bm[j], sy["lam"]) <= 1e-10
