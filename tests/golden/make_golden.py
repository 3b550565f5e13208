"""Writes the stored expected values of the full-size parity tests.

Every number written here comes from the FP64 oracle (``oracle/``) run on the
seeded synthetic workloads of ``genios_data``; nothing is taken from the GPU
path.  Run from the repository root:

    python tests/golden/make_golden.py [name ...]

Files written (one JSON per workload, under tests/golden/):
  lasso_1000x10000.json   certified Lasso optimum of the 1000 x 10000
                          decaying-spectrum workload (Sec. 5 dense Lasso
                          experiment shape): F*, duality gap, support, signs,
                          the nonzero values of x*, ||x*||.
  lasso_20000x40000.json  the same for the 20000 x 40000 workload (the large
                          dense Lasso), by the oracle's working-set route
                          (restricted certified solves, full KKT check, full
                          duality gap).
  logreg_20000x5000.json  certified optimum of the l1-logistic workload
                          (Sec. 4.2 shape) by the same working-set route.
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import genios_data  # noqa: E402
from oracle import adjoint as oadj  # noqa: E402
from oracle import lasso as olasso  # noqa: E402
from oracle import logreg as ologreg  # noqa: E402


def lasso_1000x10000():
    P = genios_data.config("lasso_1000x10000")
    t0 = time.time()
    sol = olasso.solve(P["A"], P["b"], P["lam"])
    dt = time.time() - t0
    x = sol["x"]
    S = sol["support"]
    return {
        "workload": "lasso_1000x10000",
        "generator": "genios_data.config('lasso_1000x10000')",
        "lam": P["lam"],
        "F": sol["F"],
        "gap": sol["gap"],
        "polished": bool(sol["polished"]),
        "oracle_iters": int(sol["iters"]),
        "support": [int(i) for i in S],
        "signs": [int(v) for v in np.sign(x[S])],
        "x_support": [float(v) for v in x[S]],
        "x_norm": float(np.linalg.norm(x)),
        "strict_complementarity_margin": float(
            oadj.strict_complementarity_margin(P["A"], P["b"], P["lam"], x)),
        "oracle_seconds": round(dt, 1),
    }


def lasso_20000x40000():
    P = genios_data.config("lasso_20000x40000")
    t0 = time.time()
    sol = olasso.solve_working_set(P["A"], P["b"], P["lam"])
    dt = time.time() - t0
    assert sol["certified"], sol["gap"]
    x = sol["x"]
    S = sol["support"]
    g = olasso.rmatvec_rows(P["A"], P["A"][:, S].astype(np.float64) @ x[S] - P["b"])
    off = np.ones(x.size, bool)
    off[S] = False
    return {
        "workload": "lasso_20000x40000",
        "generator": "genios_data.config('lasso_20000x40000')",
        "lam": P["lam"],
        "F": sol["F"],
        "gap": sol["gap"],
        "polished": bool(sol["polished"]),
        "working_set": sol["working_set"],
        "outer_rounds": sol["outer"],
        "support": [int(i) for i in S],
        "signs": [int(v) for v in np.sign(x[S])],
        "x_support": [float(v) for v in x[S]],
        "x_norm": float(np.linalg.norm(x)),
        "strict_complementarity_margin": float(np.min(P["lam"] - np.abs(g[off])) / P["lam"]),
        "oracle_seconds": round(dt, 1),
    }


def logreg_20000x5000():
    P = genios_data.config("logreg_20000x5000")
    t0 = time.time()
    sol = ologreg.solve_working_set(P["A"], P["y"], P["lam"])
    dt = time.time() - t0
    assert sol["certified"], sol["gap"]
    x = sol["x"]
    S = np.flatnonzero(x)
    return {
        "workload": "logreg_20000x5000",
        "generator": "genios_data.config('logreg_20000x5000')",
        "lam": P["lam"],
        "F": sol["F"],
        "gap": sol["gap"],
        "polished": bool(sol["polished"]),
        "working_set": sol["working_set"],
        "outer_rounds": sol["outer"],
        "support": [int(i) for i in S],
        "signs": [int(v) for v in np.sign(x[S])],
        "x_support": [float(v) for v in x[S]],
        "x_norm": float(np.linalg.norm(x)),
        "oracle_seconds": round(dt, 1),
    }


GOLDEN = {"lasso_1000x10000": lasso_1000x10000, "lasso_20000x40000": lasso_20000x40000,
          "logreg_20000x5000": logreg_20000x5000}


def main(names):
    for name in names or list(GOLDEN):
        rec = GOLDEN[name]()
        path = os.path.join(HERE, name + ".json")
        with open(path, "w") as f:
            json.dump(rec, f, indent=1)
            f.write("\n")
        print(f"{path}: F={rec['F']:.12g} gap={rec['gap']:.3g} |S|={len(rec['support'])} "
              f"({rec['oracle_seconds']} s)")


if __name__ == "__main__":
    main(sys.argv[1:])
