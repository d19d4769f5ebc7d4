"""Writes fullsize_oracle.json: the dense oracle's residual and test-set error
at the full size of the 2D approximation workloads and at the largest sizes of
the 2D Poisson family that a host can factor.

Calls only ``oracle`` (dense A entry by entry, LAPACK truncated SVD at
tau = 1e-12 relative to sigma_1) and ``workloads`` (problem data).  Usage,
from the repository root:

    python tests/golden/make_fullsize_oracle.py [case ...]

Cases: c3a128 (disk R = 0.8, n = 128, eps*h = 0.5), c3_128 (the same at
eps*h = 1), c4_96 and c4_128 (Poisson star, weak Dirichlet rows),
ellipse128x64 (the ellipse x^2 + 4 y^2 <= 1 on the anisotropic box
[-1.4, 1.4] x [-0.7, 0.7], 128 x 64 centres), flower128 (the multiply
connected flower of section 6.3 with a manufactured solution: Helmholtz
k^2 = 4, Neumann data on the outer curve, Dirichlet data on the hole),
flower100 (the same at the paper's 100 x 100 centres).  Each case
is written as soon as it finishes, so a long run can be resumed by naming the
remaining cases.  The test-set error uses the 200 x 200 cell-centred lattice
restricted to the domain, as the full-size GPU tests do.
"""
import json
import os
import platform
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import workloads as W  # noqa: E402
from oracle import dense, evaluate, lstsq  # noqa: E402

OUT = os.path.join(HERE, "fullsize_oracle.json")
M2D = 200

CASES = {
    "ellipse128x64": lambda: W.config_ellipse(128, 64),
    "flower128": lambda: W.config_flower(128, manufactured=True),
    "flower100": lambda: W.config_flower(100, manufactured=True),
    "c3a128": lambda: W.config_c3a(128),
    "c3_128": lambda: W.config_c3(128),
    "c4_96": lambda: W.config_c4(96),
    "c4_128": lambda: W.config_c4(128),
}


def run(name):
    prob = CASES[name]()
    t0 = time.perf_counter()
    A, idx, pts, bpts = dense.system_matrix(prob)
    B = dense.rhs(prob, pts, bpts)
    t1 = time.perf_counter()
    X, rank = lstsq.tsvd_solve(A, B, 1e-12)
    t2 = time.perf_counter()
    rel = evaluate.relres(A, X, B)
    del A
    tp = W.test_points(prob, m2d=M2D)
    f = np.stack([g(*tp.T) for g in (prob.exact or prob.rhs)], axis=1)
    err = np.max(np.abs(evaluate.eval_dense(prob, X, tp) - f), axis=0)
    return {
        "config": prob.name, "n": prob.n, "ny": prob.n_y, "N": prob.N, "M": int(idx.size), "Mb": int(bpts.shape[0]),
        "eh": prob.eh, "s": prob.s, "domain": prob.domain.name, "tau": 1e-12,
        "rank": int(rank), "relres": [float(v) for v in np.atleast_1d(rel)],
        "maxerr": [float(v) for v in err], "test_lattice": M2D,
        "seconds": {"assembly": round(t1 - t0, 1), "svd_solve": round(t2 - t1, 1)},
    }


def main(names):
    data = {}
    if os.path.exists(OUT):
        with open(OUT) as fh:
            data = json.load(fh)
    data["host"] = {"machine": platform.machine(), "cores": len(os.sched_getaffinity(0))}
    for name in names:
        print(f"[oracle] {name} ...", flush=True)
        data.setdefault("cases", {})[name] = dict(run(name), command="python tests/golden/make_fullsize_oracle.py " + name)
        print(f"[oracle] {name}: {json.dumps(data['cases'][name])}", flush=True)
        with open(OUT, "w") as fh:
            json.dump(data, fh, indent=1)


if __name__ == "__main__":
    main(sys.argv[1:] or list(CASES))
