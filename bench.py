"""Benchmark of the GeNIOS hot path on one MI355X.

    python bench.py [--gpus 1] [--steps K (5)] [--warmup W (1)] [--workload NAME]

A step is one pass of the whole hot path over the workload: a cold-start Lasso
solve in BF16-A + FP32-refinement precision (BF16 rounding of A, A^T b, the
Nystrom sketch, the ADMM loop with Nystrom-preconditioned CG, the FP32 phase
and its certification) followed by the adjoint (masked Nystrom PCG) of the loss
||z* - x0||^2.  The data are synthetic and resident in HBM before timing.

Prints one JSON line: value = ADMM iterations per second over the timed steps,
plus time-to-1e-4 for BF16-A + refine and for plain FP32 A, the dominant
kernel's bandwidth against the HBM roofline (the fused one-pass Hessian-vector
product on the BF16 copy, timed with HIP events on the solver's stream; its
measured HBM traffic per launch comes from the rocprofv3 counter summary under
profiles/), and the CPU FP64 oracle on a bounded sample of the same workload.

    python bench.py --probe-traffic

runs only a plain copy of known size and a few fused products on the workload,
for the two counter passes (FETCH_SIZE, WRITE_SIZE) that calibrate and measure
the traffic.

    python bench.py --probe-sketch

runs only a few Nystrom builds of the workload's BF16 operator (the sketch
products on the matrix cores), for counter passes over those kernels.

    python bench.py --probe-shared

runs only a few H p of 32 problems sharing the workload's matrix on the matrix
cores (BF16 copy, then the FP32 matrix), for the kernel trace and counter
passes over those kernels.

After the timed steps, `next_rows` times (once warm, outside the timed region)
the elastic net, the duality-gap termination and the adaptive sketch size on the
same workload, Huber fitting at n = 16000 under the paper's stopping rule and
the bounded least squares ablation at 32000 x 16000, the logistic workload and the
batch of 64 Lasso problems (--no-next skips them).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import statistics
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
MFMA_BF16_PEAK_TFLOPS = 2500.0  # dense BF16 matrix-core peak
METRIC = "time-to-1e-4 KKT resid & ADMM iters/s: FP32 vs BF16-A; matvec HBM GB/s"


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "hvp_fused_bf16_lasso_20000x40000_traffic.txt")
KERNEL_SOURCE = os.path.join(ROOT, "paper_2310_08333_amd", "csrc", "gemv.hip")


def measured_traffic():
    """HBM bytes per fused-product launch from the committed counter summary, or
    None when the summary is missing or the kernel source changed since."""
    try:
        with open(TRAFFIC_FILE) as f:
            kv = dict(line.split(":", 1) for line in f if ":" in line and not line.startswith("#"))
        kv = {k.strip(): v.strip() for k, v in kv.items()}
        with open(KERNEL_SOURCE, "rb") as f:
            sha = hashlib.sha256(f.read()).hexdigest()
        if kv.get("kernel_source_sha256") != sha:
            return None
        return int(float(kv["traffic_bytes_per_launch"]))
    except (OSError, KeyError, ValueError):
        return None


def probe_traffic(workload):
    """A plain device copy of known size, then fused products on the workload."""
    import torch

    import genios_data
    import paper_2310_08333_amd as g
    dev = torch.device("cuda:0")
    nbytes = 1 << 30
    src = torch.ones(nbytes // 4, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    dst.copy_(src)
    torch.cuda.synchronize()
    log(f"copy of {nbytes} bytes done")
    del src, dst
    P = genios_data.config(workload)
    A = torch.from_numpy(P["A"]).to(dev)
    A16 = g.cast_bf16(A)
    p = torch.from_numpy(np.random.default_rng(0).standard_normal(P["A"].shape[1])
                         .astype(np.float32)).to(dev)
    for i in range(3):
        g.hvp(A, p, A16=A16)
    torch.cuda.synchronize()
    log("3 fused products done")


def probe_sketch(workload):
    """A few Nystrom builds on the workload's BF16 copy at its sketch rank."""
    import torch

    import genios_data
    import paper_2310_08333_amd as g
    dev = torch.device("cuda:0")
    P = genios_data.config(workload)
    A = torch.from_numpy(P["A"]).to(dev)
    for i in range(3):
        U, lam, info = g.nystrom_build(A, P["s"], precision="bf16_only", profile_kernels=1)
        torch.cuda.synchronize()
        log(f"sketch {i}: rank {info[0]['precond_rank']} products "
            f"{1e3 * info[0]['t_sketch_mc']:.3f} ms on the matrix cores")


def probe_shared(workload, B=32):
    """A few H p of B problems sharing the workload's matrix, on the matrix cores, with
    the BF16 copy and with the FP32 matrix."""
    import torch

    import genios_data
    import paper_2310_08333_amd as g
    dev = torch.device("cuda:0")
    P = genios_data.config(workload)
    A = torch.from_numpy(P["A"]).to(dev)
    m, n = A.shape
    A16 = g.cast_bf16(A)
    Pm = torch.randn(B, n, device=dev, dtype=torch.float32)
    for name, a16 in (("bf16", A16.expand(B, m, n)), ("fp32", None)):
        for i in range(3):
            g.hvp(A.expand(B, m, n), Pm, A16=a16, batch_mfma=1)
            torch.cuda.synchronize()
        log(f"shared H p {name}: 3 products of {B} problems")


ORACLE_TIMING_FILE = os.path.join(ROOT, "tests", "golden", "oracle_timing_lasso_20000x40000.json")


def cpu_baseline(P, iters=3):
    """The oracle on the benchmark workload itself (same A, b, lambda), timed on this
    host: its GeNIOS ADMM (exact x-steps through the Cholesky factor of
    rho I + A A^T, alpha 1.6, sigma 1e-6) for `iters` iterations after its set-up.
    value = ADMM iterations per second after the set-up.  The whole run of the same
    oracle to r_kkt <= 1e-4 and its certified optimum take minutes; their figures,
    from the committed record tests/golden/oracle_timing_lasso_20000x40000.json
    (written by tests/golden/make_golden.py), ride along as `full_run`."""
    import threadpoolctl

    from oracle import lasso as olasso
    info = threadpoolctl.threadpool_info()
    cores = max([d.get("num_threads", 1) for d in info] or [os.cpu_count() or 1])
    A64 = P["A"].astype(np.float64)
    b64 = P["b"].astype(np.float64)
    clock = []
    olasso.admm(A64, b64, P["lam"], rho=1.0, alpha=1.6, sigma=1e-6, max_iter=iters,
                rho_update_every=25, clock=clock)
    del A64
    setup = clock[1] - clock[0]
    per_iter = (clock[-1] - clock[1]) / iters
    rec = {"value": round(1.0 / per_iter, 4), "unit": "ADMM iters/s", "cores": int(cores),
           "kind": "oracle",
           "sample": f"oracle GeNIOS ADMM (FP64, exact x-step) on the whole "
                     f"{P['A'].shape[0]}x{P['A'].shape[1]} workload (same A, b, lambda): "
                     f"set-up {setup:.1f} s (Cholesky of rho I + A A^T), then {iters} "
                     f"iterations at {per_iter:.2f} s each",
           "setup_s": round(setup, 2), "s_per_iter": round(per_iter, 3)}
    try:
        with open(ORACLE_TIMING_FILE) as f:
            full = json.load(f)
        rec["full_run"] = {k: full[k] for k in (
            "setup_s", "admm_iters_to_1e-4", "admm_s_per_iter", "time_to_1e-4_s",
            "rel_obj_err_at_1e-4", "time_to_certified_optimum_s", "certified_by", "host")}
    except (OSError, KeyError, ValueError):
        rec["full_run"] = None
    return rec


def _hvp_rate(info):
    """Event-timed bandwidth of the fused H p launches of one solve (BF16 and master copy)."""
    t = info["t_hvp"] + info["t_hvp_hi"]
    by = info["bytes_hvp"] + info["bytes_hvp_hi"]
    if t <= 0:
        return None, None
    gbs = by / t / 1e9
    return round(gbs, 1), round(gbs / HBM_PEAK_GBS, 4)


def _solve_record(info, target_key="t_to_target"):
    gbs, frac = _hvp_rate(info)
    return {"status_ok": info["status"] == 0, "time_s": round(info[target_key], 4),
            "iters": info["iters"], "cg_iters": info["cg_iters"],
            "iters_per_s": round(info["iters"] / info["t_total"], 2),
            "linsys_ms_per_iter": round(1e3 * info["t_linsys"] / max(info["iters"], 1), 3),
            "hvp_GBps": gbs, "hvp_frac_of_peak": frac}


def next_rows(g, torch, A, b, lam, s):
    """The rows built after the headline path, each measured once warm:
    elastic net (Sec. 4.1's lambda2 = lambda1), duality-gap termination and the
    adaptive sketch size (Sec. 2.2; sizes 8, 16, ... up to 128, kappa bound <= 10 and
    <= 1.2) on
    the headline workload, FP32 against BF16-A + refinement time to 1e-4 on the
    1000 x 10000 and the logistic workloads, Huber fitting at the paper's largest size (n = 16000,
    N = 8000, no preconditioner) under its own stopping rule, dist(0, dF(z)) <= 1e-4,
    bounded least squares at the size of its ablation (N = 32000, n = 16000,
    eps 1e-5) with and without the preconditioner and inexact solves, the
    l1-logistic workload (20000 x 5000, to 1e-4; a 16-value lambda path of it on
    its one matrix, each point to 1e-4), the batch of 64 Lasso
    problems with their adjoints, and 32 problems sharing the headline matrix (their
    H p on the matrix cores, and a lambda path)."""
    import genios_data
    out = {}
    # the 1000 x 10000 gene-expression-shaped workload: time to r_kkt <= 1e-4, FP32 A
    # against BF16-A + FP32 refinement (median of 5 after a warm-up)
    C2 = genios_data.config("lasso_1000x10000")
    A2 = torch.from_numpy(C2["A"]).to(A.device)
    b2 = torch.from_numpy(C2["b"]).to(A.device)
    for prec in ("bf16_refine", "f32"):
        runs = [g.lasso_solve(A2, b2, C2["lam"], precision=prec, eps=1e-4, sketch_rank=C2["s"])
                ["info"][0] for _ in range(6)][1:]
        r2 = sorted(runs, key=lambda i: i["t_to_target"])[len(runs) // 2]
        out[f"lasso_1000x10000_{prec}"] = {
            "status_ok": all(i["status"] == 0 for i in runs),
            "time_to_1e-4_s": round(r2["t_to_target"], 5), "iters": r2["iters"],
            "cg_iters": r2["cg_iters"], "phase_switch_iter": r2["phase_switch_iter"],
            "iters_per_s": round(r2["iters"] / r2["t_solve"], 1)}
        log(f"lasso 1000x10000 {prec}: {out[f'lasso_1000x10000_{prec}']}")
    del A2, b2
    kw = dict(precision="bf16_refine", sketch_rank=s, profile_kernels=1)
    for _ in range(2):
        en = g.lasso_solve(A, b, lam, eps=1e-4, lambda2=lam, **kw)["info"][0]
    out["elastic_net"] = dict(_solve_record(en), lambda2=lam, eps=1e-4,
                              rel_gap=en["rel_gap"], precond_s=round(en["t_precond"], 4))
    log(f"elastic net: {out['elastic_net']}")
    # (thousands of iterations here: one run, the kernels are warm from the one above)
    gp = g.lasso_solve(A, b, lam, termination=1, eps_gap=1e-4, **kw)["info"][0]
    out["gap_termination"] = dict(_solve_record(gp), eps_gap=1e-4, rel_gap=gp["rel_gap"],
                                  gap_checks=gp["gap_checks"])
    log(f"gap termination: {out['gap_termination']}")
    for target in (10.0, 1.2):
        for _ in range(2):
            ad = g.lasso_solve(A, b, lam, eps=1e-4, precision="bf16_refine", profile_kernels=1,
                               adaptive_sketch=1, sketch_rank=128, sketch_rank_init=8,
                               sketch_kappa=target)["info"][0]
        key = f"adaptive_sketch_kappa{target:g}"
        out[key] = dict(_solve_record(ad), rank_cap=128, rank_init=8, kappa_target=target,
                        chosen_rank=ad["precond_rank"], sizes_tried=ad["sketch_rounds"],
                        kappa_bound=ad["kappa_bound"], sketch_err=ad["sketch_err"],
                        precond_s=round(ad["t_precond"], 4))
        log(f"{key}: {out[key]}")
    t0 = time.time()
    H = genios_data.huber_outliers(16000, seed=6)
    Ah = torch.from_numpy(H["A"]).to(A.device)
    bh = torch.from_numpy(H["b"]).to(A.device)
    log(f"generated {H['name']} in {time.time() - t0:.1f}s")
    for prec in ("bf16_refine", "f32"):
        for _ in range(2):
            hu = g.huber_solve(Ah, bh, H["lam"], precision=prec, precondition=0, termination=2,
                               eps_gap=1e-4, profile_kernels=1, max_iter=5000)["info"][0]
        out[f"huber_{prec}"] = dict(_solve_record(hu), workload=H["name"],
                                    subgrad_dist=hu["subgrad_dist"], obj=hu["obj"])
        log(f"huber {prec}: {out[f'huber_{prec}']}")
    del Ah, bh
    # a batch sharing the headline matrix: the H p of 32 problems at once on the matrix
    # cores against one fused product per problem, and a 32-value lambda path
    Bsh = 32
    m = A.shape[0]
    Ash, A16sh = A.expand(Bsh, m, A.shape[1]), g.cast_bf16(A).expand(Bsh, m, A.shape[1])
    Psh = torch.randn(Bsh, A.shape[1], device=A.device, dtype=torch.float32)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    for name, a16, e_a in (("bf16", A16sh, 2), ("fp32", None, 4)):
        t_sh = {}
        for mf in (1, 0):
            g.hvp(Ash, Psh, A16=a16, batch_mfma=mf)
            torch.cuda.synchronize()
            ev0.record()
            for _ in range(3):
                g.hvp(Ash, Psh, A16=a16, batch_mfma=mf)
            ev1.record()
            torch.cuda.synchronize()
            t_sh[mf] = ev0.elapsed_time(ev1) / 3 / 1e3
        a_bytes = m * A.shape[1] * e_a
        out[f"shared_matrix_hvp_32_{name}"] = {
            "matrix_cores_ms": round(1e3 * t_sh[1], 3),
            "per_problem_fused_ms": round(1e3 * t_sh[0], 3), "speedup": round(t_sh[0] / t_sh[1], 2),
            "matrix_cores_GBps": round((2 * a_bytes + Bsh * A.shape[1] * 8) / t_sh[1] / 1e9, 1),
            "matrix_cores_TFLOPs": round(4 * m * A.shape[1] * Bsh / t_sh[1] / 1e12, 1),
            "per_problem_equivalent_GBps": round(Bsh * a_bytes / t_sh[1] / 1e9, 1)}
        log(f"shared hvp {name}: {out[f'shared_matrix_hvp_32_{name}']}")
    lams = [float(lam) * 2.0 ** ((j - 16) / 8.0) for j in range(Bsh)]
    bsh = b.expand(Bsh, m).contiguous()
    for mf in (1, 0):
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        op = g.lasso_solve(Ash, bsh, lams, A16=A16sh, precision="bf16_refine", eps=1e-4, sketch_rank=s,
                           batch_mfma=mf, profile_kernels=1)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        its = [i["iters"] for i in op["info"]]
        out[f"lasso_path_32_batch_mfma{mf}"] = {
            "all_ok": all(i["status"] == 0 for i in op["info"]), "solve_s": round(t2 - t1, 4),
            "admm_iters_total": int(sum(its)), "admm_iters_max": int(max(its)),
            "hvp_launches_matrix_cores": op["info"][0]["n_hvp_mrhs"],
            "phase_switch_iter": op["info"][0]["phase_switch_iter"]}
        log(f"lasso path 32 batch_mfma={mf}: {out[f'lasso_path_32_batch_mfma{mf}']}")
    del Ash, A16sh, Psh, bsh
    # l1-logistic regression at the paper's settings (re-sketch every 20, eps 1e-4) from
    # the workload's initial penalty (the mean Hessian eigenvalue at x = 0): time to
    # r_kkt <= 1e-4, FP32 against BF16-A + FP32 refinement (median of 5 after a warm-up)
    Lg = genios_data.config("logreg_20000x5000")
    Al = torch.from_numpy(Lg["A"]).to(A.device)
    yl = torch.from_numpy(Lg["y"]).to(A.device)
    for prec in ("bf16_refine", "f32"):
        runs = []
        for _ in range(6):
            runs.append(g.logreg_solve(Al, yl, Lg["lam"], rho=Lg["rho"], precision=prec,
                                       eps=1e-4, sketch_rank=Lg["s"], resketch_every=20,
                                       profile_kernels=1)["info"][0])
        runs = runs[1:]
        lo = sorted(runs, key=lambda i: i["t_to_target"])[len(runs) // 2]
        gbs, frac = _hvp_rate(lo)
        out[f"logreg_20000x5000_{prec}"] = {
            "status_ok": all(i["status"] == 0 for i in runs), "rho0": round(Lg["rho"], 3),
            "time_to_1e-4_s": round(lo["t_to_target"], 4), "iters": lo["iters"],
            "cg_iters": lo["cg_iters"], "resketches": lo["resketches"],
            "phase_switch_iter": lo["phase_switch_iter"],
            "iters_per_s": round(lo["iters"] / lo["t_solve"], 1), "r_kkt": lo["r_kkt"],
            "precond_s": round(lo["t_precond"], 4), "hvp_GBps": gbs, "hvp_frac_of_peak": frac}
        log(f"logreg {prec}: {out[f'logreg_20000x5000_{prec}']}")
    # a 16-value lambda path of that workload on its one matrix, each point to 1e-4
    Bl = 16
    Alb = Al.expand(Bl, *Al.shape)
    ylb = yl.expand(Bl, yl.shape[0]).contiguous()
    lams_l = [float(Lg["lam"]) * 2.0 ** ((j - 8) / 4.0) for j in range(Bl)]
    for mf in (1, 0):
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        ol = g.logreg_solve(Alb, ylb, lams_l, rho=Lg["rho"], precision="bf16_refine", eps=1e-4,
                            sketch_rank=Lg["s"], resketch_every=20, max_iter=1000,
                            batch_mfma=mf, profile_kernels=1)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        out[f"logreg_path_16_batch_mfma{mf}"] = {
            "all_ok": all(i["status"] == 0 for i in ol["info"]),
            "solve_s": round(t2 - t1, 4), "admm_iters_total": int(sum(i["iters"] for i in ol["info"])),
            "cg_iters_max": int(max(i["cg_iters"] for i in ol["info"])),
            "hvp_launches_matrix_cores": ol["info"][0]["n_hvp_mrhs"]}
        log(f"logreg path 16 batch_mfma={mf}: {out[f'logreg_path_16_batch_mfma{mf}']}")
    del Al, yl, Alb, ylb
    # the batch of 64 Lasso problems (2000 x 8000 each) and their adjoints
    t0 = time.time()
    Pb = genios_data.config("lasso_batch_64x2000x8000")
    Ab = torch.from_numpy(Pb["A"]).to(A.device)
    bb = torch.from_numpy(Pb["b"]).to(A.device)
    x0b = torch.from_numpy(Pb["x0"]).to(A.device, torch.float32)
    log(f"generated {Pb['name']} in {time.time() - t0:.1f}s")
    for _ in range(2):
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        ob = g.lasso_solve(Ab, bb, Pb["lam"], precision="bf16_refine", eps=1e-4,
                           sketch_rank=Pb["s"], profile_kernels=1)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        gzb = (2.0 * (ob["z"] - x0b)).contiguous()
        _, _, binf = g.lasso_backward(Ab, ob["z"], gzb, Pb["lam"], sketch_rank=Pb["s"])
        torch.cuda.synchronize()
        t3 = time.perf_counter()
    its = [i["iters"] for i in ob["info"]]
    gbs, frac = _hvp_rate(ob["info"][0])
    out["lasso_batch_64x2000x8000"] = {
        "problems": len(its), "all_ok": all(i["status"] == 0 for i in ob["info"]) and
        all(i["status"] == 0 for i in binf),
        "solve_s": round(t2 - t1, 4), "adjoint_s": round(t3 - t2, 4),
        "admm_iters_total": int(sum(its)), "admm_iters_max": int(max(its)),
        "admm_iters_per_s": round(sum(its) / (t2 - t1), 1),
        "problems_per_s": round(len(its) / (t3 - t1), 1),
        "hvp_GBps": gbs, "hvp_frac_of_peak": frac}
    log(f"batch: {out['lasso_batch_64x2000x8000']}")
    del Ab, bb, x0b
    # bounded least squares at the size of the paper's ablation (N = 32000, n = 16000),
    # eps 1e-5, with and without the preconditioner and inexact solves
    t0 = time.time()
    Q = genios_data.boxls_decay(32000, 16000, seed=8, s=50)
    Aq = torch.from_numpy(Q["A"]).to(A.device)
    bq = torch.from_numpy(Q["b"]).to(A.device)
    log(f"generated {Q['name']} in {time.time() - t0:.1f}s")
    variants = [("bf16_refine", 1, 1), ("f32", 1, 1), ("f32", 0, 1), ("f32", 1, 0), ("f32", 0, 0)]
    for prec, pc, inexact in variants:
        for _ in range(2 if (pc and inexact) else 1):
            bx = g.boxls_solve(Aq, bq, 0.0, 1.0, precision=prec, eps=1e-5, sketch_rank=Q["s"],
                               precondition=pc, inexact=inexact, profile_kernels=1,
                               max_iter=5000)["info"][0]
        key = f"boxls_{prec}" + ("" if pc else "_nopc") + ("" if inexact else "_exact")
        out[key] = dict(_solve_record(bx), workload=Q["name"], eps=1e-5,
                        precond_s=round(bx["t_precond"], 4), obj=bx["obj"])
        log(f"{key}: {out[key]}")
    del Aq, bq
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="lasso_20000x40000")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp32", action="store_true")
    ap.add_argument("--no-backward", action="store_true")
    ap.add_argument("--no-next", action="store_true")
    ap.add_argument("--probe-traffic", action="store_true")
    ap.add_argument("--probe-sketch", action="store_true")
    ap.add_argument("--probe-shared", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU: the library has no multi-GPU path "
              f"(--gpus {args.gpus} requested)", file=sys.stderr)
        sys.exit(2)

    if args.probe_traffic:
        probe_traffic(args.workload)
        return
    if args.probe_sketch:
        probe_sketch(args.workload)
        return
    if args.probe_shared:
        probe_shared(args.workload)
        return

    import torch

    import genios_data
    import paper_2310_08333_amd as g

    t0 = time.time()
    P = genios_data.config(args.workload)
    log(f"generated {P['name']} in {time.time() - t0:.1f}s")
    dev = torch.device("cuda:0")
    A = torch.from_numpy(P["A"]).to(dev)
    b = torch.from_numpy(P["b"]).to(dev)
    x0 = torch.from_numpy(P["x0"]).to(dev, torch.float32)
    lam, s = P["lam"], P["s"]
    m, n = P["A"].shape
    torch.cuda.synchronize()
    opts = dict(eps=1e-4, sketch_rank=s)

    def step(profile):
        out = g.lasso_solve(A, b, lam, precision="bf16_refine", profile_kernels=profile, **opts)
        bw = None
        if not args.no_backward:
            gz = (2.0 * (out["z"] - x0)).contiguous()
            bw = g.lasso_backward(A, out["z"], gz, lam, sketch_rank=s, profile_kernels=profile)
        return out, bw

    for i in range(args.warmup):
        out, _ = step(0)
        log(f"warmup {i}: status {out['status']} iters {out['info'][0]['iters']}")
    torch.cuda.synchronize()
    iters, ttt, infos, binfos = [], [], [], []
    t_start = time.perf_counter()
    for i in range(args.steps):
        out, bw = step(1)
        inf = out["info"][0]
        infos.append(inf)
        if bw is not None:
            binfos.append(bw[2][0])
        iters.append(inf["iters"])
        ttt.append(inf["t_to_target"])
        log(f"step {i}: status {out['status']} iters {inf['iters']} cg {inf['cg_iters']} "
            f"switch {inf['phase_switch_iter']} t_to_1e-4 {inf['t_to_target']:.4f}s "
            f"r_kkt {inf['r_kkt']:.2e}")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start
    ms_per_step = 1e3 * elapsed / args.steps

    # The dominant kernel: the fused Hessian-vector product on the BF16 copy,
    # timed with HIP events on the solver's stream inside the timed steps.
    allinf = infos + binfos
    tot = lambda key: sum(i[key] for i in allinf)
    t_h, n_h, b_h = tot("t_hvp"), tot("n_hvp"), tot("bytes_hvp")
    t_hh, n_hh, b_hh = tot("t_hvp_hi"), tot("n_hvp_hi"), tot("bytes_hvp_hi")
    ach = b_h / t_h / 1e9 if t_h > 0 else None
    per = b_h / max(n_h, 1)
    traffic = measured_traffic()
    # the read rate a plain streaming kernel reaches on this GPU (the FP32 master,
    # 3.2 GB, read 10 times): the attainable HBM rate for a bandwidth-bound kernel
    read_s = g.stream_read_seconds(A, reps=10)
    attainable = 10 * A.numel() * 4 / read_s / 1e9
    log(f"streaming read: {attainable:.0f} GB/s")
    roofline = {
        "bound": "hbm", "kernel": "k_hvp_fused: H p = A^T A p, BF16 A, one pass over A",
        "achieved": round(ach, 1) if ach else None, "peak": HBM_PEAK_GBS, "unit": "GB/s",
        "frac": round(ach / HBM_PEAK_GBS, 4) if ach else None, "traffic": traffic,
        "attainable_read_GBps": round(attainable, 1),
        "frac_of_attainable": round(ach / attainable, 4) if ach else None,
        "bytes_per_launch": int(per), "launches": n_h,
        "avg_us": round(1e6 * t_h / max(n_h, 1), 2),
        "two_stream_equivalent_GBps": round(2 * m * n * 2 / (t_h / max(n_h, 1)) / 1e9, 1)
        if t_h > 0 else None,
        "master_copy_hvp": {"achieved_GBps": round(b_hh / t_hh / 1e9, 1) if t_hh > 0 else None,
                            "launches": n_hh,
                            "avg_us": round(1e6 * t_hh / max(n_hh, 1), 2)},
    }

    # The sketch products W = A Omega, Y = A^T W on the matrix cores: algorithmic
    # flops 4 m n s per sketch over their event-timed duration, against the BF16
    # matrix-core peak and against the HBM bound of two BF16 streams of A.
    t_sk, f_sk, n_sk = tot("t_sketch_mc"), tot("flops_sketch_mc"), tot("n_sketch_mc")
    sketch = None
    if t_sk > 0 and n_sk > 0:
        tfl = f_sk / t_sk / 1e12
        intensity = (4.0 * m * n * s) / (2.0 * m * n * 2)  # flop per byte of A read
        attainable = min(MFMA_BF16_PEAK_TFLOPS, intensity * HBM_PEAK_GBS / 1e3)
        sketch = {"kernels": "k_sketch_w_mfma + k_sketch_y_mfma (v_mfma_f32_16x16x32_bf16)",
                  "achieved_TFLOPs": round(tfl, 1), "peak_TFLOPs": MFMA_BF16_PEAK_TFLOPS,
                  "mfma_utilisation": round(tfl / MFMA_BF16_PEAK_TFLOPS, 4),
                  "bound": "hbm", "attainable_TFLOPs": round(attainable, 1),
                  "frac_of_attainable": round(tfl / attainable, 4),
                  "flop_per_byte": intensity, "sketches": n_sk,
                  "avg_ms": round(1e3 * t_sk / n_sk, 3),
                  "hbm_GBps": round(n_sk * 2.0 * m * n * 2 / t_sk / 1e9, 1)}

    # per-phase iteration rates from one solve with the iteration history (outside
    # the timed steps): the BF16-A phase from the end of set-up to its last
    # iteration, the FP32 phase from there to the last iteration
    hs = g.lasso_solve(A, b, lam, precision="bf16_refine", history=400, **opts)
    hist, hinf = hs["history"][0], hs["info"][0]
    k_tot = hinf["iters"]
    rows = hist[:k_tot]
    ph0 = rows[rows[:, 7] == 0]
    ph1 = rows[rows[:, 7] == 1]
    t0_end = ph0[-1, 8] if len(ph0) else hinf["t_setup"]
    phases = {
        "setup_s": round(hinf["t_setup"], 4),
        "bf16_A": {"iters": int(len(ph0)),
                   "iters_per_s": round(float(len(ph0) / max(t0_end - hinf["t_setup"], 1e-9)), 1)},
        "fp32_A": {"iters": int(len(ph1)),
                   "iters_per_s": round(float(len(ph1) / max(ph1[-1, 8] - t0_end, 1e-9)), 1)
                   if len(ph1) else None},
    }
    # the plain matrix-vector kernels of the step (set-up A^T b, duality gap, adjoint)
    t_n, b_n, n_n = tot("t_matvec_n"), tot("bytes_matvec_n"), tot("n_matvec_n")
    t_t, b_t, n_t = tot("t_matvec_t"), tot("bytes_matvec_t"), tot("n_matvec_t")
    matvecs = {"A_v": {"launches": n_n, "GBps": round(b_n / t_n / 1e9, 1) if t_n > 0 else None},
               "At_w": {"launches": n_t, "GBps": round(b_t / t_t / 1e9, 1) if t_t > 0 else None}}
    log(f"phases: {phases} matvecs: {matvecs}")

    fp32 = None
    if not args.no_fp32:
        o32 = g.lasso_solve(A, b, lam, precision="f32", **opts)["info"][0]
        o32 = g.lasso_solve(A, b, lam, precision="f32", **opts)["info"][0]
        fp32 = {"time_to_1e-4_s": round(o32["t_to_target"], 4), "iters": o32["iters"],
                "cg_iters": o32["cg_iters"], "iters_per_s": round(o32["iters"] / o32["t_total"], 2)}
        log(f"fp32: {fp32}")

    nxt = None
    if not args.no_next:
        nxt = next_rows(g, torch, A, b, lam, s)

    cpu = None
    if not args.no_cpu_baseline:
        log("cpu baseline: the oracle's set-up and 3 ADMM iterations on the whole workload")
        cpu = cpu_baseline(P)
        log(f"cpu baseline: {cpu}")

    value = sum(iters) / elapsed
    rec = {
        "metric": METRIC, "value": round(value, 3), "unit": "ADMM iters/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "bf16",
        "data": "synthetic",
        "config": {"workload": P["name"], "m": m, "n": n, "sketch_rank": s,
                   "precision": "bf16_refine", "step": "lasso solve + adjoint" if not args.no_backward else "lasso solve",
                   "eps": 1e-4},
        "time_to_1e-4_s": {"bf16_refine": round(statistics.median(ttt), 4),
                           "fp32": fp32["time_to_1e-4_s"] if fp32 else None},
        "admm_iters": statistics.median(iters),
        "time_to_1e-4_min_s": round(min(ttt), 4),
        "phases": phases,
        "matvecs": matvecs,
        "precond_s": round(statistics.median(i["t_precond"] for i in infos), 4),
        "fp32": fp32,
        "roofline": roofline,
        "sketch_gemm": sketch,
        "next_rows": nxt,
        "cpu_baseline": cpu,
    }
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
