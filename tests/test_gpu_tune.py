"""The block-sweep autotuner (msp_solve_opts.autotune): the tuned segment count is one of
the admissible ones, the solution still matches the dense solve, a second solve reuses
the cached choice (same bits), and the choice is written to the MSP_TUNE_CACHE file once."""
import json

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


def test_autotuned_block_sweep(tmp_path, monkeypatch):
    cache = tmp_path / "tune.jsonl"
    monkeypatch.setenv("MSP_TUNE_CACHE", str(cache))
    n, k, s, lam = 2048, 12, 64, 1e-3
    say(f"case autotune psd n={n} k={k} s={s}")
    a, eigs, _ = W.psd_outlier(n, 32, config_id=401)
    lam0 = omsp.paper_lambda0(eigs, s // 2)
    bm = W.gaussian((k, n), 401)
    A = torch.from_numpy(a).to(DEV)
    B = torch.from_numpy(bm).to(DEV)
    rows, signs, Y = msp.sketch(A, s, 8, 21)
    P = msp.Precond("psd", rows, signs, Y, lam, lam0, 4 * s, 8, 22)
    X0, i0 = msp.solve(P, A, B, tol=1e-10, inner_tol=1e-12)
    X1, i1 = msp.solve(P, A, B, tol=1e-10, inner_tol=1e-12, autotune=1)
    X2, i2 = msp.solve(P, A, B, tol=1e-10, inner_tol=1e-12, autotune=1)
    say("built-in", i0["sweep_segments"], "tuned", i1["sweep_segments"], i2["sweep_segments"])
    for info in (i0, i1, i2):
        assert info["status"] == "MSP_OK", info
    assert i0["sweep_segments"] in (1, 2, 4, 8, 16, 32, 64)
    assert i1["sweep_segments"] in (1, 2, 4, 8, 16, 32)  # 64 leaves segments under 64 columns
    assert i2["sweep_segments"] == i1["sweep_segments"]
    assert np.array_equal(X1.cpu().numpy(), X2.cpu().numpy())
    x1 = X1.cpu().numpy()
    for j in range(k):
        xs = dense.solve_psd(a, bm[j], lam)
        assert np.linalg.norm(x1[j] - xs) <= 1e-8 * np.linalg.norm(xs)
    assert abs(i1["outer_iters"] - i0["outer_iters"]) <= 2
    lines = [json.loads(l) for l in cache.read_text().splitlines() if l.strip()]
    assert len(lines) == 1, lines
    rec = lines[0]
    assert rec["kernel"] == "block_sweep" and rec["rows"] == n and rec["cols"] == n and rec["k"] == k
    assert rec["nseg"] == i1["sweep_segments"] and rec["ms"] > 0
    P.close()


@pytest.mark.parametrize("dt,n,s", [(torch.float64, 4096, 256), (torch.float32, 3000, 300)])
def test_autotuned_sketch_rows_per_block(tmp_path, monkeypatch, dt, n, s):
    # msp_sketch_autotune times every admissible number of rows of A per block on the
    # caller's matrix and keeps the fastest for the shape; the rows per block change only the
    # work split, not the order of any sum, so Y is the same bits as the built-in choice's,
    # and a second call takes the cached choice without timing again
    cache = tmp_path / "tune.jsonl"
    monkeypatch.setenv("MSP_TUNE_CACHE", str(cache))
    say(f"case sketch autotune n={n} s={s} {dt}")
    g = torch.Generator(device=DEV)
    g.manual_seed(402)
    A = torch.randn((n, n), dtype=dt, device=DEV, generator=g)
    r0, g0, Y0 = msp.sketch(A, s, 8, 31)
    r1, g1, Y1, R = msp.sketch(A, s, 8, 31, autotune=True)
    say("rows per block", R)
    assert R in (2, 4, 8, 16, 32)
    assert torch.equal(r0, r1) and torch.equal(g0, g1)
    assert torch.equal(Y0, Y1)
    _, _, Y2, R2 = msp.sketch(A, s, 8, 31, autotune=True)
    _, _, Y3 = msp.sketch(A, s, 8, 31)
    assert R2 == R and torch.equal(Y2, Y0) and torch.equal(Y3, Y0)
    lines = [json.loads(l) for l in cache.read_text().splitlines() if l.strip()]
    assert len(lines) == 1, lines
    rec = lines[0]
    assert rec["kernel"] == "sketch_apply" and rec["n"] == n and rec["s"] == s and rec["gamma"] == 8
    assert rec["rows_per_block"] == R and rec["ms"] > 0
