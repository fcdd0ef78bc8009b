"""Writes rbf_gp_n32768_lambda0.json: lam0 = (2/l) sum_{i>l} lambda_i (Theorem 4.1) of the
n = 32768 RBF kernel matrix of the GP-regression workload, from tr(A) = n and its l
largest eigenvalues (ARPACK Lanczos on the host). Calls only `workloads` and `oracle`.

    python tests/golden/make_rbf_lambda0.py [n]
"""
import json
import os
import sys
import time

import numpy as np
import scipy.sparse.linalg as sla

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import workloads as W  # noqa: E402
from oracle import msp  # noqa: E402


def main():
    name = "rbf_gp_n32768"
    w = W.config(name)
    n = int(sys.argv[1]) if len(sys.argv) > 1 else w.n
    if n != w.n:
        w = W.config(name, n=n, s=max(8, n // 64))
    t0 = time.time()
    pts = W.rbf_points(w.n, w.extra["dim"], w.config_id)
    a = W.rbf_matrix(pts)
    tr = float(np.trace(a))
    top = sla.eigsh(a, k=w.l + 1, which="LA", return_eigenvectors=False, tol=1e-10)
    top = np.sort(top)[::-1]
    lam0 = msp.paper_lambda0_from_top(tr, top[:w.l], w.l)
    out = {
        "workload": name, "n": w.n, "s": w.s, "l": w.l, "trace": tr,
        "lambda_1": float(top[0]), "lambda_l": float(top[w.l - 1]), "lambda_l_plus_1": float(top[w.l]),
        "tail_sum": tr - float(top[:w.l].sum()), "lambda0": lam0,
        "method": "tr(A) - sum of the l largest eigenvalues (scipy eigsh, tol 1e-10)",
        "seconds": time.time() - t0,
    }
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), f"rbf_gp_n{w.n}_lambda0.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
