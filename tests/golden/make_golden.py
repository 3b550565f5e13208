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
  oracle_timing_lasso_20000x40000.json
                          the oracle timed on the whole 20000 x 40000 Lasso
                          workload (same A, b, lambda): the set-up of its
                          exact x-step (Cholesky of rho I + A A^T), its ADMM
                          iterations per second, its time to r_kkt <= 1e-4 on
                          its own iterates, and the time of its certified
                          optimum; with the host's core count.
"""
import json
import os
import platform
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


def _host():
    import threadpoolctl
    info = threadpoolctl.threadpool_info()
    threads = max([d.get("num_threads", 1) for d in info] or [os.cpu_count() or 1])
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"blas_threads": int(threads), "cpu_count": os.cpu_count(), "cpu_model": model,
            "python": platform.python_version(), "numpy": np.__version__}


def oracle_timing_lasso_20000x40000():
    P = genios_data.config("lasso_20000x40000")
    A64 = P["A"].astype(np.float64)
    b64 = P["b"].astype(np.float64)
    # set-up of the exact x-step alone (the same factorisation admm() starts with)
    t0 = time.perf_counter()
    olasso.ShiftedGramSolve(A64, 1.0 + 1e-6)
    t_setup = time.perf_counter() - t0
    # the oracle's GeNIOS ADMM (alpha 1.6, sigma 1e-6, the paper's penalty rule) to
    # r_kkt <= 1e-4, each iteration's residual from the exact FP64 gradient
    t0 = time.perf_counter()
    x, z, u, rho, hist = olasso.admm(A64, b64, P["lam"], rho=1.0, alpha=1.6, sigma=1e-6,
                                     max_iter=1000, eps=1e-4, rho_update_every=25)
    t_admm = time.perf_counter() - t0
    iters = len(hist)
    per_iter = (t_admm - t_setup) / iters
    F = olasso.objective(A64, b64, P["lam"], z)
    del A64
    t0 = time.perf_counter()
    sol = olasso.solve_working_set(P["A"], P["b"], P["lam"])
    t_cert = time.perf_counter() - t0
    return {
        "workload": "lasso_20000x40000",
        "generator": "genios_data.config('lasso_20000x40000')",
        "host": _host(),
        "setup_s": round(t_setup, 2),
        "admm_iters_to_1e-4": iters,
        "admm_final_r_kkt": float(hist[-1, 3]),
        "admm_s_per_iter": round(per_iter, 3),
        "admm_iters_per_s": round(1.0 / per_iter, 4),
        "time_to_1e-4_s": round(t_admm, 2),
        "rel_obj_err_at_1e-4": (F - sol["F"]) / sol["F"],
        "time_to_certified_optimum_s": round(t_cert, 2),
        "certified_by": "working-set route: certified restricted solves, full KKT check, "
                        "full App. A duality gap",
        "F": sol["F"],
        "gap": sol["gap"],
        "support": [int(i) for i in sol["support"]],
        "oracle_seconds": round(t_setup + t_admm + t_cert, 1),
    }


GOLDEN = {"lasso_1000x10000": lasso_1000x10000, "lasso_20000x40000": lasso_20000x40000,
          "logreg_20000x5000": logreg_20000x5000,
          "oracle_timing_lasso_20000x40000": oracle_timing_lasso_20000x40000}


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
