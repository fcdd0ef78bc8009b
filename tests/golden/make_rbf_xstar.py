"""Writes rbf_gp_n32768_xstar.npy: x* = (A + lam I)^{-1} b for the n = 32768 RBF kernel
matrix and right-hand side of the GP-regression workload, by the oracle's dense LU solve
(oracle.dense.solve_general on A + lam I; the Cholesky routine of this image's OpenBLAS
stops with a segmentation fault at n = 32768, LU does not), plus rbf_gp_n32768_xstar.json
with the sizes, the FP64 residual of x* and its norm. Calls only `workloads` and `oracle`.
Needs about 20 GB of host memory and a few minutes.

    python tests/golden/make_rbf_xstar.py
"""
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import workloads as W  # noqa: E402
from oracle import dense  # noqa: E402


def main():
    name = "rbf_gp_n32768"
    w = W.config(name)
    t0 = time.time()
    a = W.rbf_matrix(W.rbf_points(w.n, w.extra["dim"], w.config_id))
    b = W.gaussian(w.n, w.config_id)
    t1 = time.time()
    a[np.diag_indices_from(a)] += w.lam  # A + lam I, in place
    x = dense.solve_general(a, b)
    t2 = time.time()
    rr = float(np.linalg.norm(b - a @ x) / np.linalg.norm(b))
    here = os.path.dirname(os.path.abspath(__file__))
    np.save(os.path.join(here, f"rbf_gp_n{w.n}_xstar.npy"), x)
    out = {
        "workload": name, "n": w.n, "lambda": w.lam, "method": "oracle.dense.solve_general on A + lam I (dense LU, FP64)",
        "rel_residual": rr, "x_norm": float(np.linalg.norm(x)), "b_norm": float(np.linalg.norm(b)),
        "x_sha256": hashlib.sha256(np.ascontiguousarray(x).tobytes()).hexdigest(),
        "seconds_matrix": t1 - t0, "seconds_solve": t2 - t1,
    }
    with open(os.path.join(here, f"rbf_gp_n{w.n}_xstar.json"), "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
