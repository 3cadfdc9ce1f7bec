#!/usr/bin/env python3
"""Benchmark of the NysPCG hot path on one MI355X.

Workload (default): the batched lambda-grid problem at n = 1e6 points, d = 16,
RBF kernel sigma = 4, 64 right-hand sides b_c = sign(X w_c) times 8 lambdas
log-spaced over [1e-7 n, 1e-3 n] (512 independent columns), one shared Nystrom
sketch of rank 500, F16X3_D6 kernel products (fp16 K V split over the six-term
bf16 distance), block PCG in float32 with float64 residual refinement, tolerance 1e-6
on the float64 true relative residual.

One step = sketch + preconditioner build + PCG to tolerance for every column
(the paper counts the preconditioner build in the solve time, section "Large-Scale
Ridge Regression with NysPCG").  Data generation, device placement and the
Gaussian test matrix are outside the timer; one warm-up capped at 10 iterations
precedes the timed steps and the clock stops after a device synchronisation
(section "Hardware, Timing, and Solver Settings").

One step at n = 1e6 takes minutes, so --steps and --warmup are upper bounds under a
wall-clock budget (--budget-s, counted from process start): at most one warm-up, the
first timed step always, and a further one only when its projected end (the slowest
step so far, plus the time the report needs) fits the budget.  The JSON line reports
the counts actually run.  Progress goes to stderr, one line per phase.

Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import platform
import statistics
import sys
import time

T_START = time.monotonic()
ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "NysPCG time-to-1e-6 rel. residual + kernel_matvec TFLOP/s, n=1e6 d=16"
PEAK_BF16_TFLOPS = 2500.0      # MI355X dense bf16 / fp16 MFMA (published)
PEAK_F64_TFLOPS = 78.6         # MI355X float64 MFMA (published)
HBM_GBS = 8000.0


def phase(msg: str) -> None:
    print(f"[bench {time.monotonic() - T_START:7.1f}s] {msg}", file=sys.stderr, flush=True)


def elapsed() -> float:
    return time.monotonic() - T_START


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1, help="timed steps (upper bound under --budget-s)")
    ap.add_argument("--warmup", type=int, default=1, help="warm-up steps (at most one is run)")
    ap.add_argument("--budget-s", type=float, default=540.0,
                    help="wall-clock budget from process start; no timed step starts that would end past it")
    ap.add_argument("--n", type=int, default=1_000_000)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--seeds", default="",
                    help="comma-separated data seeds, one timed step each in turn (default: --seed)")
    ap.add_argument("--refine-every", type=int, default=0)
    ap.add_argument("--refine-mode", type=int, default=1)
    ap.add_argument("--refine-reduction", type=float, default=1e-3,
                    help="first cycle factor of the float64 refinement cycles")
    ap.add_argument("--no-block", action="store_true",
                    help="headline: column-independent PCG instead of block PCG over the 64 right-hand sides "
                         "of each lambda")
    ap.add_argument("--kmv-reps", type=int, default=3)
    ap.add_argument("--cpu-seconds", type=float, default=15.0, help="target CPU time of the oracle sample")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-m1", action="store_true", help="skip the single right-hand-side solve")
    ap.add_argument("--no-probe", action="store_true", help="skip the ceiling probes")
    ap.add_argument("--kmv-only", action="store_true", help="time the kernel product only (profiling)")
    ap.add_argument("--kmv-fp64", default="",
                    help="with --kmv-only: also time the float64 product (the refinement residual) at these "
                         "comma-separated column counts")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="with --kmv-only: first run one plain 1 GiB device copy, whose HBM counter readings "
                         "scale the kernel's (rocprofv3 --pmc FETCH_SIZE / WRITE_SIZE)")
    ap.add_argument("--verbose", action="store_true")
    ap.add_argument("--ridge-n", type=int, default=65536, help="ridge_ratio: rows of X")
    ap.add_argument("--ridge-p", type=int, default=0, help="ridge_ratio: columns of X (0: = rows)")
    ap.add_argument("--ridge-alpha", type=float, default=2.0, help="ridge_ratio: spectral decay")
    ap.add_argument("--ridge-lambda", type=float, default=1e-6, help="ridge_ratio: regularisation")
    ap.add_argument("--ridge-rank", type=int, default=128, help="ridge_ratio: Nystrom rank")
    ap.add_argument("--en-n", type=int, default=400_000, help="elastic_net: rows")
    ap.add_argument("--en-d", type=int, default=100, help="elastic_net: raw inputs per row")
    ap.add_argument("--en-p", type=int, default=1000, help="elastic_net: random features (columns of X)")
    ap.add_argument("--en-eps", type=float, default=1e-7, help="elastic_net: eps_abs = eps_rel")
    ap.add_argument("--en-max-iters", type=int, default=5000, help="elastic_net: ADMM iteration cap")
    ap.add_argument("--prec", default="f16x3_d6",
                    choices=["bf16x3", "bf16x3_d6", "bf16x3_d10", "f16x3_d10", "f16x3_d6", "fp32"],
                    help="kernel-product precision of the batched workload")
    ap.add_argument("--no-autotune", action="store_true",
                    help="skip the tile autotuner (heuristic chunk widths)")
    ap.add_argument("--tile-cache", default=os.path.expanduser("~/.cache/paper_2609_08136_amd/tiles.json"),
                    help="JSON cache of autotuned chunk widths")
    ap.add_argument("--workload", default="batched_lambda_grid",
                    choices=["batched_lambda_grid", "plain_fp64", "matrix_free_fp32", "precision_variant",
                             "differentiation", "grid_vs_fp32", "cg_ratio", "ridge_ratio", "elastic_net"],
                    help="batched_lambda_grid is the headline workload; the others are recorded separately")
    return ap.parse_args()


# ----------------------------------------------------------------------------- other workloads

def _timed(torch, fn):
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    res = fn()
    torch.cuda.synchronize()
    return res, time.perf_counter() - t0


def _solve_once(nys, torch, X, B, w, Om0, prec, sketch_prec, **opts):
    """sketch + build + solve; returns (Xsol, info, rc, P, seconds)."""
    def run():
        P = nys.build_preconditioner(X, Om0, w.kind, w.sigma, sketch_prec)
        x, info, rc = nys.nyspcg_solve(X, B, w.lambdas, w.kind, w.sigma, P, tol=w.tol, prec=prec, **opts)
        return x, info, rc, P
    (x, info, rc, P), t = _timed(torch, run)
    return x, info, rc, P, t


def run_other(args):
    import numpy as np
    import torch

    import nys_inputs as ni
    import paper_2609_08136_amd as nys

    nys.load()
    dev = torch.device("cuda:0")
    T = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    wl = args.workload
    out = {"n_gpus": 1, "steps": 1, "warmup": 1, "higher_is_better": False, "scaling": "weak",
           "vs_baseline": None, "data": "synthetic", "unit": "s", "device": device_label(torch)}

    if wl == "plain_fp64":
        w = ni.plain_fp64(args.seed)
        X, B, Om0 = T(w.X), T(w.B), T(ni.gaussian_test_matrix(w.n, w.r, args.seed))
        _solve_once(nys, torch, X, B, w, Om0, nys.FP64, nys.FP64, max_iters=10)          # warmup
        x, info, rc, P, t = _solve_once(nys, torch, X, B, w, Om0, nys.FP64, nys.FP64, check_true=True)
        cpu = cpu_baseline_plain(w, x.cpu().numpy().reshape(-1), ni.gaussian_test_matrix(w.n, w.r, args.seed))
        out.update(metric="NysPCG time-to-1e-8 rel. residual, n=2000 d=10, FP64", value=round(t, 5),
                   ms_per_step=round(t * 1e3, 3), dtype="f64",
                   config={"workload": "plain_fp64", "n": w.n, "d": w.d, "rank": w.r, "lambda": w.lambdas[0],
                           "sigma": w.sigma, "tol": w.tol},
                   solve={"status": rc, "iters": info[0]["iters"], "relres_true": info[0]["relres_true"],
                          "rel_error_vs_cholesky": cpu.pop("rel_error_vs_cholesky")},
                   cpu_baseline=cpu)
    elif wl == "matrix_free_fp32":
        w = ni.matrix_free_fp32(args.seed)
        X, B = T(w.X), T(w.B)
        g = torch.Generator(device=dev)
        g.manual_seed(args.seed + ni.OMEGA_SEED_OFFSET)
        Om0 = torch.randn((w.n, w.r), generator=g, device=dev, dtype=torch.float64)
        _solve_once(nys, torch, X, B, w, Om0, nys.FP32, nys.FP32, max_iters=10, refine_every=0)
        x, info, rc, P, t = _solve_once(nys, torch, X, B, w, Om0, nys.FP32, nys.FP32, refine_every=0,
                                        refine_mode=1)
        x2, info2, rc2, _, t2 = _solve_once(nys, torch, X, B, w, Om0, nys.FP32, nys.FP32, refine_every=-1,
                                            check_true=True)
        V = torch.randn((w.n, 1), generator=g, device=dev, dtype=torch.float32)
        nys.kernel_matvec(X, X, V, w.kind, w.sigma, nys.FP32)
        _, tk = _timed(torch, lambda: nys.kernel_matvec(X, X, V, w.kind, w.sigma, nys.FP32))
        out.update(metric="NysPCG time-to-1e-6 float64 rel. residual, n=2e5 d=20, FP32 matrix-free",
                   value=round(t, 3), ms_per_step=round(t * 1e3, 1), dtype="f32",
                   config={"workload": "matrix_free_fp32", "n": w.n, "d": w.d, "rank": w.r,
                           "lambda": w.lambdas[0], "sigma": w.sigma, "tol": w.tol},
                   solve={"status": rc, "iters": info[0]["iters"], "refinements": info[0]["refinements"],
                          "relres_true": info[0]["relres_true"]},
                   without_refinement={"seconds": round(t2, 3), "status": rc2, "iters": info2[0]["iters"],
                                       "relres_recursive": info2[0]["relres_recursive"],
                                       "relres_true": info2[0]["relres_true"]},
                   kernel_matvec_m1_ms=round(tk * 1e3, 3))
    elif wl == "precision_variant":
        w = ni.precision_variant(args.seed)
        X, B = T(w.X), T(w.B)
        g = torch.Generator(device=dev)
        g.manual_seed(args.seed + ni.OMEGA_SEED_OFFSET)
        Om0 = torch.randn((w.n, w.r), generator=g, device=dev, dtype=torch.float64)
        res = {}
        for name, prec in (("bf16x3", nys.BF16X3), ("fp32", nys.FP32)):
            _solve_once(nys, torch, X, B, w, Om0, prec, prec, max_iters=10, refine_every=20)
            x, info, rc, P, t = _solve_once(nys, torch, X, B, w, Om0, prec, prec, refine_every=20, refine_mode=1)
            res[name] = {"seconds": round(t, 3), "status": rc, "iters": info[0]["iters"],
                         "refinements": info[0]["refinements"], "relres_true": info[0]["relres_true"]}
            if args.verbose:
                print(name, res[name], file=sys.stderr, flush=True)
        out.update(metric="NysPCG time-to-1e-6 float64 rel. residual, n=5e5 d=32, BF16X3 + FP64 refinement",
                   value=res["bf16x3"]["seconds"], ms_per_step=round(res["bf16x3"]["seconds"] * 1e3, 1),
                   dtype="bf16x3",
                   config={"workload": "precision_variant", "n": w.n, "d": w.d, "rank": w.r,
                           "lambda": w.lambdas[0], "sigma": w.sigma, "tol": w.tol, "refine_every": 20},
                   runs=res, speedup_vs_fp32=round(res["fp32"]["seconds"] / res["bf16x3"]["seconds"], 3))
    elif wl in ("grid_vs_fp32", "cg_ratio"):
        out.update(grid_or_cg(args, nys, torch, ni, dev, T))
    elif wl == "ridge_ratio":
        out.update(ridge_ratio(args, nys, torch, ni, dev))
    elif wl == "elastic_net":
        out.update(elastic_net(args, nys, torch, ni, dev, T))
    else:  # differentiation
        from paper_2609_08136_amd import autograd as ag
        w = ni.differentiation(args.seed)
        X, y, Xv, yv = T(w.X), T(w.B[:, 0]), T(w.Xval), T(w.yval)
        g = torch.Generator(device=dev)
        g.manual_seed(args.seed + ni.OMEGA_SEED_OFFSET)
        Om0 = torch.randn((w.n, w.r), generator=g, device=dev, dtype=torch.float64)
        opts = dict(tol=1e-10, prec=nys.FP64)

        def loss_grad(theta):
            P = nys.build_preconditioner(X, Om0, w.kind, math.exp(theta[1]), nys.FP64)
            tl = torch.tensor(theta[0], dtype=torch.float64, device=dev, requires_grad=True)
            ts = torch.tensor(theta[1], dtype=torch.float64, device=dev, requires_grad=True)
            L = ag.validation_loss(X, y, Xv, yv, tl, ts, w.kind, P, opts)
            L.backward()
            return float(L), np.array([float(tl.grad), float(ts.grad)])

        theta = np.array([math.log(w.lambdas[0]), math.log(w.sigma)])
        loss_grad(theta)                                                              # warmup
        (L, gr), t_one = _timed(torch, lambda: loss_grad(theta))
        eta, hist = 0.05, [L]
        t0 = time.perf_counter()
        for _ in range(20):
            while True:
                cand = theta - eta * gr
                Lc, gc = loss_grad(cand)
                if Lc <= L or eta < 1e-6:
                    break
                eta *= 0.5
            theta, L, gr = cand, Lc, gc
            hist.append(L)
        t_gd = time.perf_counter() - t0
        out.update(metric="validation loss + adjoint gradient time, n=1e5 train / 2e4 val, d=16, Laplacian, FP64",
                   value=round(t_one, 3), ms_per_step=round(t_one * 1e3, 1), dtype="f64",
                   config={"workload": "differentiation", "n_train": w.n, "n_val": w.Xval.shape[0], "d": w.d,
                           "rank": w.r, "lambda0": w.lambdas[0], "sigma0": w.sigma, "kernel": "laplacian"},
                   gradient_descent={"steps": 20, "eta_final": eta, "seconds": round(t_gd, 2),
                                     "loss": [round(v, 8) for v in hist],
                                     "lambda": math.exp(theta[0]), "sigma": math.exp(theta[1])})
    print(json.dumps(out))


def cpu_baseline_plain(w, x_gpu, Omega):
    """The oracle on the whole plain float64 workload (dense K, Nystrom, textbook
    PCG), timed on the host, plus the GPU solution's error against its Cholesky
    solve."""
    import numpy as np
    import oracle as o

    t0 = time.perf_counter()
    o.nyspcg_dense(w.X, w.B, w.lambdas, w.kind, w.sigma, Omega, tol=w.tol)
    t_cpu = time.perf_counter() - t0
    K = o.kernel_matrix(w.X, w.X, w.kind, w.sigma)
    ref = o.direct_solve(K, w.B[:, 0], w.lambdas[0])
    return {"value": t_cpu, "unit": "s", "cores": os.cpu_count(), "kind": "oracle",
            "sample": "the whole workload: dense K, Nystrom, textbook PCG (float64 NumPy)",
            "rel_error_vs_cholesky": float(np.linalg.norm(x_gpu - ref) / np.linalg.norm(ref))}


def grid_or_cg(args, nys, torch, ni, dev, T):
    """grid_vs_fp32: the lambda-grid recipe (64 rhs x 8 lambdas) at a reduced n with the
    mixed-precision product against plain float32 products, both to the float64-checked
    tolerance.  cg_ratio: the float32 matrix-free workload (n = 2e5, d = 20) with NysPCG
    against plain CG (no preconditioner), the ratio the paper reports for its ridge
    problems (section "Large-Scale Ridge Regression with NysPCG")."""
    def solve(w, X, B, Om0, prec, P_on, max_iters=1000):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        P = nys.build_preconditioner(X, Om0, w.kind, w.sigma, prec) if P_on else None
        x, info, rc = nys.nyspcg_solve(X, B, w.lambdas, w.kind, w.sigma, P, tol=w.tol, max_iters=max_iters,
                                       prec=prec, refine_every=0, refine_mode=1,
                                       block=not args.no_block and B.shape[1] > 1)
        torch.cuda.synchronize()
        t = time.perf_counter() - t0
        rel = [c["relres_true"] for c in info]
        return {"seconds": round(t, 3), "status": rc, "max_iters": max(c["iters"] for c in info),
                "sum_iters": sum(c["iters"] for c in info), "sum_refinements": sum(c["refinements"] for c in info),
                "max_relres_true": max(rel), "accepted_fp64": rc == nys.OK and all(0 <= v <= w.tol for v in rel)}

    seeds = [int(s) for s in args.seeds.split(",") if s.strip()] or [args.seed]
    res = {}
    for seed in seeds:
        if args.workload == "grid_vs_fp32":
            n = args.n if args.n != 1_000_000 else 200_000
            w = ni.batched_lambda_grid(seed, n=n)
        else:
            w = ni.matrix_free_fp32(seed)
        X, B = T(w.X), T(w.B)
        g = torch.Generator(device=dev)
        g.manual_seed(seed + ni.OMEGA_SEED_OFFSET)
        Om0 = torch.randn((w.n, w.r), generator=g, device=dev, dtype=torch.float64)
        if args.workload == "grid_vs_fp32":
            arms = ((args.prec, nys.PREC_BY_NAME[args.prec], True), ("fp32", nys.FP32, True))
        else:
            arms = (("nyspcg", nys.FP32, True), ("cg", nys.FP32, False))
        for name, prec, P_on in arms:
            solve(w, X, B, Om0, prec, P_on, max_iters=10)                          # warm-up
            r = solve(w, X, B, Om0, prec, P_on, max_iters=1000 if P_on else 20000)
            res.setdefault(name, []).append(r)
            phase(f"seed {seed} {name}: {r}")
    names = list(res)
    med = {k: statistics.median(r["seconds"] for r in v) for k, v in res.items()}
    if args.workload == "grid_vs_fp32":
        return {"metric": f"lambda-grid time-to-1e-6 float64 rel. residual, n={w.n} d=16, 64 rhs x 8 lambdas",
                "value": round(med[names[0]], 3), "ms_per_step": round(med[names[0]] * 1e3, 1),
                "dtype": args.prec, "steps": len(seeds),
                "config": {"workload": "grid_vs_fp32", "n": w.n, "d": w.d, "rank": w.r, "tol": w.tol,
                           "lambdas": [float(v) for v in w.lambdas],
                           "solver": "column PCG" if args.no_block else "block PCG per lambda"},
                "runs": res, "median_s": med, "speedup_vs_fp32": round(med["fp32"] / med[args.prec], 3)}
    return {"metric": "CG time / NysPCG time, n=2e5 d=20 float32 matrix-free, float64-checked 1e-6",
            "value": round(med["cg"] / med["nyspcg"], 3), "unit": "ratio", "higher_is_better": True,
            "ms_per_step": round(med["nyspcg"] * 1e3, 1), "dtype": "f32", "steps": len(seeds),
            "config": {"workload": "cg_ratio", "n": w.n, "d": w.d, "rank": w.r, "tol": w.tol,
                       "lambda": w.lambdas[0]},
            "runs": res, "median_s": med}


def ridge_ratio(args, nys, torch, ni, dev):
    """CG time / NysPCG time on the paper's ridge problem (section "Large-Scale Ridge
    Regression with NysPCG": X = U Sigma V^T from SORF factors, y = U g / |g|), normal
    matrix applied through X and X^T, tolerance 1e-6 (the paper's calibrated ridge
    tolerance), rank-128 Nystrom preconditioner built inside the timed NysPCG region,
    median and min-max over the seeds (three by default)."""
    import numpy as np

    n = args.ridge_n
    p = args.ridge_p or n
    alpha, lam, rank, tol = args.ridge_alpha, args.ridge_lambda, args.ridge_rank, 1e-6
    seeds = [int(v) for v in args.seeds.split(",") if v.strip()] or [0, 1, 2]
    runs = {"nyspcg": [], "cg": []}

    def nyspcg(X, y, seed, max_iters):
        Y, Q = nys.nys_ridge_sketch(X, None, seed=seed, r=rank)
        P = nys.nys_precond_build(Y, Q, with_fp32=False)
        del Y, Q
        return nys.nys_ridge_solve(X, y, lam, P, tol=tol, max_iters=max_iters, check_true=True)

    def cg(X, y, seed, max_iters):
        return nys.nys_ridge_solve(X, y, lam, None, tol=tol, max_iters=max_iters, check_true=True)

    for seed in seeds:
        (X, y), t_gen = _timed(torch, lambda: ni.ridge_problem_device(n, p, alpha, seed, dev))
        phase(f"ridge seed {seed}: X {n} x {p} built on the device in {t_gen:.1f} s")
        for name, fn, cap in (("nyspcg", nyspcg, 5000), ("cg", cg, 20000)):
            fn(X, y, seed, 3)                                                          # warm-up
            (W, info, rc), t = _timed(torch, lambda: fn(X, y, seed, cap))
            r = {"seed": seed, "seconds": round(t, 4), "iters": info[0]["iters"], "status": rc,
                 "relres_recursive": info[0]["relres_recursive"], "relres_true": info[0]["relres_true"]}
            runs[name].append(r)
            phase(f"ridge seed {seed} {name}: {r}")
            del W
        del X, y
        torch.cuda.empty_cache()
    med = {k: statistics.median(r["seconds"] for r in v) for k, v in runs.items()}
    rng = {k: [min(r["seconds"] for r in v), max(r["seconds"] for r in v)] for k, v in runs.items()}
    cg_capped = any(r["status"] != nys.OK for r in runs["cg"])
    out = {"metric": f"CG time / NysPCG time, ridge n={n} p={p} alpha={alpha:g} lambda={lam:g}, rel. residual 1e-6",
           "value": round(med["cg"] / med["nyspcg"], 3), "unit": "ratio", "higher_is_better": True,
           "ms_per_step": round(med["nyspcg"] * 1e3, 2), "dtype": "f64", "steps": len(seeds),
           "config": {"workload": "ridge_ratio", "n": n, "p": p, "alpha": alpha, "lambda": lam, "rank": rank,
                      "tol": tol, "seeds": seeds},
           "median_s": med, "min_max_s": rng, "runs": runs,
           "cg_lower_bound": cg_capped,
           "paper_context": "7.23x on one H200 at n = p = 2^16, alpha 2, lambda 1e-6 (another machine)"}
    if not args.no_cpu:
        import oracle as o

        pr = ni.ridge_problem(4096, 4096, alpha, seed=seeds[0])
        t0 = time.perf_counter()
        U, lh, _ = o.nystrom(o.ridge_normal_apply(pr.X), ni.gaussian_test_matrix(4096, rank, seeds[0]))
        A = o.ridge_normal_apply(pr.X)
        b = pr.X.T @ pr.y
        _, it, _ = o.pcg(lambda v: A(v) + lam * v, b, lambda r: o.precond_apply(U, lh, lam, r), tol=tol,
                         max_iters=5000)
        t_cpu = time.perf_counter() - t0
        out["cpu_baseline"] = {"value": round(t_cpu, 3), "unit": "s", "cores": os.cpu_count(), "kind": "oracle",
                               "sample": f"oracle NysPCG (rank {rank}, float64 NumPy) on the same recipe at "
                                         f"n = p = 4096 on the host: {it} iterations"}
    return out


def elastic_net(args, nys, torch, ni, dev, T):
    """NysADMM on the bounded elastic net (section "Bounded Elastic Net with NysADMM")
    on a synthetic dense random-feature problem of the shape of the paper's yolanda-rf
    (4e5 rows, 100 standardised inputs, 1000 Gaussian random features; the dataset
    itself is not used), lam1 = lam2 = 0.1 lam_max, at the paper's calibrated NysADMM
    tolerance 1e-7 and otherwise the default configuration.  The answer is checked by
    its stationarity (the distance from 0 to the subdifferential, infinity norm,
    computed here in float64 with torch) and its box feasibility."""
    n, d_in, p, eps = args.en_n, args.en_d, args.en_p, args.en_eps
    t0 = time.perf_counter()
    pr = ni.elastic_net_problem(n, d_in, p, seed=args.seed)
    phase(f"elastic net: X {n} x {p} generated on the host in {time.perf_counter() - t0:.1f} s")
    X, y = T(pr.X), T(pr.y)
    cfg = dict(eps_abs=eps, eps_rel=eps, seed=args.seed, max_iters=args.en_max_iters)
    nys.nys_admm_elastic_net(X, y, pr.lam1, pr.lam2, **dict(cfg, max_iters=2))           # warm-up
    (w, info, rc), t = _timed(torch, lambda: nys.nys_admm_elastic_net(X, y, pr.lam1, pr.lam2, **cfg))
    phase(f"elastic net: {t:.2f} s, {info['iters']} ADMM iterations, {info['pcg_iters']} PCG iterations, rc={rc}")
    # stationarity of w (intercept at its optimum): -grad of the smooth part against
    # lam1 * subdifferential of |.| plus the normal cone of [0, 1]
    Xc = X - X.mean(dim=0)
    g = Xc.T @ (Xc @ w - (y - y.mean())) / n + pr.lam2 * w
    t_ = -g
    lo_s = torch.where(w > 0, torch.full_like(w, pr.lam1), torch.full_like(w, -pr.lam1))
    hi_s = torch.full_like(w, pr.lam1)
    lo_s = torch.where(w <= 0.0, torch.full_like(w, -math.inf), lo_s)
    hi_s = torch.where(w >= 1.0, torch.full_like(w, math.inf), hi_s)
    viol = torch.where(t_ < lo_s, lo_s - t_, torch.where(t_ > hi_s, t_ - hi_s, torch.zeros_like(t_)))
    stationarity = float(viol.abs().max())
    feas = float(torch.clamp(torch.maximum(-w, w - 1.0), min=0.0).max())
    del Xc
    return {"metric": f"NysADMM bounded elastic net time to eps {eps:g}, dense n={n} p={p}",
            "value": round(t, 3), "unit": "s", "higher_is_better": False, "ms_per_step": round(t * 1e3, 1),
            "dtype": "f64", "steps": 1,
            "config": {"workload": "elastic_net", "n": n, "d_in": d_in, "p": p, "lam1": pr.lam1, "lam2": pr.lam2,
                       "eps_abs": eps, "eps_rel": eps, "rank": 50, "admm_defaults": "table tab:rlaopt-admm-config"},
            "status": rc, "info": info, "stationarity_inf": stationarity, "box_violation": feas,
            "accepted": rc == nys.OK and stationarity < 1e-4 and feas <= 1e-6,
            "nonzeros": int((w > 0).sum()), "at_upper": int((w >= 1.0).sum()),
            "paper_context": "the paper's checks: stationarity < 1e-4, feasibility < 1e-6 (its datasets are not used)"}


def log(args, *a):
    if args.verbose:
        print(*a, file=sys.stderr, flush=True)


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor()


# Kernel sources whose hash a committed HBM-counter summary must match to be reported.
KERNEL_SOURCES = ["kmv_common.h", "kmv_kernels.h", "kmv_host.hip", "gen_dispatch.py"]


def device_label(torch) -> str:
    """Marketing name of GPU 0, else its gfx architecture (the name can be empty)."""
    props = torch.cuda.get_device_properties(0)
    arch = getattr(props, "gcnArchName", "") or ""
    name = props.name or ""
    return f"{name} ({arch})" if name and arch else (name or arch)


def kernel_source_hash() -> str:
    import hashlib
    h = hashlib.sha256()
    base = os.path.join(os.path.dirname(os.path.abspath(__file__)), "paper_2609_08136_amd", "csrc")
    for f in KERNEL_SOURCES:
        with open(os.path.join(base, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def counted_traffic(prec_name: str, n: int, m: int):
    """HBM bytes per launch of the dominant kernel, from the committed rocprofv3 --pmc
    summary (FETCH_SIZE and WRITE_SIZE, each scaled by a 1 GiB copy's reading), or None
    when there is none for this configuration or the kernel sources changed since."""
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "profiles",
                        f"kmv_traffic_{prec_name}_n{n}_m{m}.md")
    if not os.path.exists(path):
        return None
    fields = {}
    with open(path) as fh:
        for line in fh:
            if ":" in line and line.startswith("- "):
                k, v = line[2:].split(":", 1)
                fields[k.strip()] = v.strip().strip("`")
    if fields.get("kernel_source_sha256") != kernel_source_hash():
        return None
    try:
        return int(fields["traffic_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def time_kernel_matvec(nys, torch, X, sigma, m, prec, reps):
    """Average duration of one kernel_matvec call, from HIP events recorded on the
    stream the product is launched on (torch's current stream)."""
    g = torch.Generator(device=X.device)
    g.manual_seed(1234)
    dt = torch.float64 if prec == nys.FP64 else torch.float32
    V = torch.randn((X.shape[0], m), generator=g, device=X.device, dtype=dt)
    out = torch.empty_like(V)
    nys.kernel_matvec(X, X, V, nys.RBF, sigma, prec, out=out)     # untimed first call
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    s = torch.cuda.Event(enable_timing=True)
    e = torch.cuda.Event(enable_timing=True)
    s.record(stream)
    for _ in range(reps):
        nys.kernel_matvec(X, X, V, nys.RBF, sigma, prec, out=out)
    e.record(stream)
    torch.cuda.synchronize()
    t = s.elapsed_time(e) / 1e3 / reps
    del V, out
    return t


def cpu_baseline(args, w, Xs_host, seconds, gpu_info):
    """The oracle's float64 K V (NumPy) on a bounded row sample of the headline run:
    V is the GPU's own solution (n x 512), so the same product also gives an
    independent float64 residual estimate on the sampled rows.  The time is scaled to
    a full time-to-solution estimate with the GPU run's product count."""
    import numpy as np
    import oracle as o

    n, m = w.n, Xs_host.shape[1]
    nrhs = w.B.shape[1]
    cores = os.cpu_count() or 1
    rng = np.random.default_rng(11)
    order = rng.permutation(n)
    rows = 8
    t0 = time.perf_counter()
    KX = [o.kernel_matvec_rows(w.X[order[:rows]], w.X, Xs_host, w.kind, w.sigma)]
    t_small = time.perf_counter() - t0
    more = max(0, min(n - rows, int(rows * seconds / max(t_small, 1e-3)) - rows))
    if more:
        KX.append(o.kernel_matvec_rows(w.X[order[rows:rows + more]], w.X, Xs_host, w.kind, w.sigma))
    t_rows = time.perf_counter() - t0
    rows += more
    sel = order[:rows]
    KX = np.concatenate(KX, axis=0)
    lam_col = np.array([w.lambdas[c // nrhs] for c in range(m)])
    Bcol = w.B[sel][:, [c % nrhs for c in range(m)]]
    res = Bcol - KX - lam_col * Xs_host[sel]
    relres_rows = float((np.linalg.norm(res, axis=0) / np.linalg.norm(Bcol, axis=0)).max())
    t_kv = t_rows * n / rows                       # one full m-column K V, extrapolated
    kv_equiv = gpu_info["kv_equivalents"]
    est = t_kv * kv_equiv
    return {
        "value": round(est, 1), "unit": "s", "cores": cores, "kind": "oracle",
        "sample": (f"oracle float64 K(X[S], X) V for {rows} random rows S of the n={n} point set with V the "
                   f"GPU solution (n x {m}) took {t_rows:.1f} s ({cores} host threads, {cpu_model()}); "
                   f"extrapolated x{n / rows:.0f} to one full {m}-column product ({t_kv:.0f} s) and "
                   f"x{kv_equiv:.1f} to the GPU run's products (sum of column iterations plus 5 x float64 "
                   f"refinements, / {m})"),
        "kernel_matvec_tflops": round(n * n * (2 * w.d + 2 * m) / t_kv / 1e12, 4),
        "oracle_sampled_rows_max_relres": relres_rows,
        "rows": rows,
    }


def probes(nys, torch, dev):
    """Sustained ceilings of the units the product uses (nys_peak_probe)."""
    ws = torch.empty(2 << 30, dtype=torch.uint8, device=dev)
    out = {
        "bf16_mfma_tflops": nys.nys_peak_probe(nys.PROBE_BF16_MFMA, workspace=ws) / 1e12,
        "f16_mfma_tflops": nys.nys_peak_probe(nys.PROBE_F16_MFMA, workspace=ws) / 1e12,
        "f64_mfma_tflops": nys.nys_peak_probe(nys.PROBE_F64_MFMA, workspace=ws) / 1e12,
        "exp2_f32_gexp_s": nys.nys_peak_probe(nys.PROBE_EXP2, workspace=ws) / 1e9,
        "copy_gbs": nys.nys_peak_probe(nys.PROBE_COPY, 4, workspace=ws) / 1e9,
    }
    del ws
    return {k: round(v, 1) for k, v in out.items()}


def headline(args):
    phase("loading torch and libnys")
    import numpy as np
    import torch

    import nys_inputs as ni
    import paper_2609_08136_amd as nys

    nys.load()
    dev = torch.device("cuda:0")
    budget = args.budget_s
    seeds = [int(s) for s in args.seeds.split(",") if s.strip()] or [args.seed]
    prec = nys.PREC_BY_NAME[args.prec]

    state = {}

    def load_seed(seed):
        if state.get("seed") == seed:
            return state
        state.clear()
        w = ni.batched_lambda_grid(seed, n=args.n)
        g = torch.Generator(device=dev)
        g.manual_seed(seed + ni.OMEGA_SEED_OFFSET)
        state.update(seed=seed, w=w, X=torch.from_numpy(w.X).to(dev), B=torch.from_numpy(w.B).to(dev),
                     Omega0=torch.randn((w.n, w.r), generator=g, device=dev, dtype=torch.float64))
        return state

    st = load_seed(seeds[0])
    w, X = st["w"], st["X"]
    n, d, r = w.n, w.d, w.r
    nrhs, nlam = w.B.shape[1], len(w.lambdas)
    m = nrhs * nlam
    phase(f"inputs ready: n={n} d={d} r={r} columns={m} ({nrhs} rhs x {nlam} lambdas) prec={args.prec}")

    t_tune, tiles, f64_tiles = 0.0, None, None
    if not args.no_autotune:
        t0 = time.perf_counter()
        tiles = nys.autotune(X, w.kind, w.sigma, prec, m, cache=args.tile_cache, n_rows=min(n, 262144))
        # the float64 refinement products: per-chunk costs of every width on this shape
        f64_tiles = nys.autotune_fp64_costs(X, w.kind, w.sigma, n_rows=min(n, 16384))
        t_tune = time.perf_counter() - t0
        phase(f"autotune {t_tune:.1f} s: " + ", ".join(f"{k}: {v['tm']}" for k, v in tiles.items())
              + f"; float64 cost table measured, {f64_tiles['tm_at_256']} columns at 256")
    if args.kmv_only and args.copy_calibration:
        src = torch.ones(1 << 28, dtype=torch.float32, device=dev)      # 1 GiB
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        phase("copy calibration: 1 GiB device-to-device copy done")
        del src, dst
    ceilings = None
    if not args.no_probe and not args.kmv_only:
        ceilings = probes(nys, torch, dev)
        phase(f"ceiling probes: {ceilings}")
    # ---- dominant kernel: the m-column product (the solve's first product width)
    t_kmv = time_kernel_matvec(nys, torch, X, w.sigma, m, prec, args.kmv_reps)
    flops = n * n * (2 * d + 2 * m)
    kmv_tflops = flops / t_kmv / 1e12
    phase(f"kernel_matvec m={m}: {t_kmv * 1e3:.1f} ms, {kmv_tflops:.1f} TFLOP/s")
    t_kmv1 = time_kernel_matvec(nys, torch, X, w.sigma, 1, prec, args.kmv_reps)
    phase(f"kernel_matvec m=1: {t_kmv1 * 1e3:.1f} ms")
    if args.kmv_only:
        res = {"kernel_matvec_ms": t_kmv * 1e3, "tflops": kmv_tflops, "m1_ms": t_kmv1 * 1e3}
        for mc in [int(c) for c in args.kmv_fp64.split(",") if c.strip()]:
            t64 = time_kernel_matvec(nys, torch, X, w.sigma, mc, nys.FP64, args.kmv_reps)
            phase(f"float64 kernel_matvec m={mc}: {t64 * 1e3:.1f} ms")
            res[f"fp64_m{mc}_ms"] = t64 * 1e3
        print(json.dumps(res), flush=True)
        return

    ws = torch.empty(nys.nys_workspace_bytes(nys.OP_SOLVE, n, 0, d, r, m, prec), dtype=torch.uint8, device=dev)

    def step(st, max_iters, B=None, lambdas=None):
        Xd = st["X"]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        Y, Q = nys.nys_sketch(Xd, st["Omega0"], w.kind, w.sigma, prec)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        P = nys.nys_precond_build(Y, Q, prec, with_fp32=True)
        del Y, Q
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        Xs, info, rc = nys.nyspcg_solve(Xd, st["B"] if B is None else B, w.lambdas if lambdas is None else lambdas,
                                        w.kind, w.sigma, P, tol=w.tol, max_iters=max_iters, prec=prec,
                                        refine_every=args.refine_every, refine_mode=args.refine_mode,
                                        refine_reduction=args.refine_reduction, workspace=ws,
                                        block=not args.no_block and (B is None or B.shape[-1] > 1))
        torch.cuda.synchronize()
        t3 = time.perf_counter()
        return Xs, info, rc, P, (t1 - t0, t2 - t1, t3 - t2, t3 - t0)

    n_warm = 0
    if args.warmup > 0:
        step(st, 10)
        n_warm = 1
        phase("warm-up step (10 iterations) done")
    # time the report needs after the last step: single-RHS solve, acceptance, oracle sample
    reserve = (0 if args.no_m1 else 25.0) + (0 if args.no_cpu else args.cpu_seconds + 10.0) + 10.0
    runs = []
    for k in range(max(1, args.steps)):
        if k > 0:
            worst = max(rn["phases"][3] for rn in runs)
            if elapsed() + 1.05 * worst + reserve > budget:
                phase(f"budget: next step would end past {budget:.0f} s; stopping after {k} timed step(s)")
                break
        seed = seeds[k % len(seeds)]
        st = load_seed(seed)
        Xs, info, rc, P, ph = step(st, 1000)
        rel_true = [c["relres_true"] for c in info]
        runs.append({"seed": seed, "phases": ph, "rc": rc, "info": info, "rank": P.rank, "nu": P.nu,
                     "accepted": rc == nys.OK and all(0 <= v <= w.tol for v in rel_true),
                     "max_relres_true": max(rel_true)})
        phase(f"timed step {k + 1} (seed {seed}): sketch {ph[0]:.2f} s, build {ph[1]:.2f} s, solve {ph[2]:.2f} s, "
              f"total {ph[3]:.2f} s, rc={rc}, max true relres {max(rel_true):.3e}")
        del P
    last = runs[-1]
    st = load_seed(last["seed"])
    w = st["w"]
    info = last["info"]
    times = [rn["phases"][3] for rn in runs]
    t_step = statistics.median(times)
    iters = [c["iters"] for c in info]
    refs = [c["refinements"] for c in info]
    per_lambda = {f"{w.lambdas[l]:.3g}": max(iters[l * nrhs:(l + 1) * nrhs]) for l in range(nlam)}

    # ---- independent acceptance check (after the timer) on 8192 sampled rows:
    # r_S = b_S - (K x)_S - lambda x_S with the float64 product
    rows = torch.from_numpy(np.sort(np.random.default_rng(3).choice(n, min(n, 8192), replace=False))).to(dev)
    KX = nys.kernel_matvec(st["X"][rows].contiguous(), st["X"], Xs, w.kind, w.sigma, nys.FP64)
    lam_col = torch.tensor([w.lambdas[c // nrhs] for c in range(m)], dtype=torch.float64, device=dev)
    Bcol = st["B"][:, [c % nrhs for c in range(m)]]
    res = Bcol[rows] - KX - lam_col * Xs[rows]
    sampled = (res.norm(dim=0) / Bcol[rows].norm(dim=0)).max().item()
    del KX, res, Bcol
    phase(f"sampled-row float64 check: max relres {sampled:.3e}")

    # ---- single right-hand side (m = 1) at lambda = 1e-3 n: sketch + build + solve
    single = None
    if not args.no_m1 and elapsed() + 30.0 + (0 if args.no_cpu else args.cpu_seconds + 10.0) < budget:
        b1 = st["B"][:, :1].contiguous()
        _, info1, rc1, P1, ph1 = step(st, 1000, B=b1, lambdas=[w.lambdas[-1]])
        single = {"lambda": float(w.lambdas[-1]), "seconds": round(ph1[3], 3),
                  "phases_s": {"sketch": round(ph1[0], 3), "build": round(ph1[1], 3), "solve": round(ph1[2], 3)},
                  "iters": info1[0]["iters"], "refinements": info1[0]["refinements"],
                  "relres_true": info1[0]["relres_true"], "status": rc1}
        del P1
        phase(f"single right-hand side: {ph1[3]:.2f} s, {info1[0]['iters']} iterations, "
              f"true relres {info1[0]['relres_true']:.3e}")

    kv_equiv = (sum(iters) + sum(refs) * 5) / m   # a float64 column product costs ~5 low-precision ones
    cpu = None
    if not args.no_cpu:
        secs = max(2.0, min(args.cpu_seconds, budget - elapsed() - 10.0))
        phase(f"oracle sample on the host ({secs:.0f} s target)")
        cpu = cpu_baseline(args, w, Xs.cpu().numpy(), secs, {"kv_equivalents": kv_equiv})
        phase(f"oracle sample: {cpu['rows']} rows, sampled-row relres {cpu['oracle_sampled_rows_max_relres']:.3e}")

    three = PEAK_BF16_TFLOPS / 3.0
    out = {
        "metric": METRIC,
        "value": round(t_step, 3),
        "unit": "s",
        "n_gpus": 1,
        "steps": len(runs),
        "warmup": n_warm,
        "ms_per_step": round(t_step * 1e3, 1),
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.prec,
        "data": "synthetic",
        "config": {
            "workload": "batched_lambda_grid",
            "n": n, "d": d, "kernel": "rbf", "sigma": w.sigma, "nrhs": nrhs, "nlam": nlam,
            "lambdas": [float(v) for v in w.lambdas], "rank": r, "tol": w.tol,
            "precision": f"{args.prec} K V, fp32 CG, fp64 residual refinement",
            "refine_every": args.refine_every, "refine_mode": args.refine_mode,
            "solver": ("column-independent PCG sharing each product" if args.no_block else
                       "block PCG (O'Leary): the 64 right-hand sides of each lambda share a block Krylov space; "
                       "the 8 blocks share each product"),
        },
        "steps_requested": args.steps, "warmup_requested": args.warmup, "budget_s": budget,
        "seeds": [rn["seed"] for rn in runs],
        "step_s": {"median": round(t_step, 3), "min": round(min(times), 3), "max": round(max(times), 3),
                   "all": [round(t, 3) for t in times]},
        "tiles": {"autotune_s": round(t_tune, 1), "widths": {k: v["tm"] for k, v in (tiles or {}).items()},
                  "fp64_cost_table": f64_tiles},
        "kernel_matvec_tflops": round(kmv_tflops, 1),
        "kernel_matvec": {"m": m, "ms": round(t_kmv * 1e3, 2), "tflops": round(kmv_tflops, 1),
                          "m1_ms": round(t_kmv1 * 1e3, 2),
                          "m1_gpairs_per_s": round(n * n / t_kmv1 / 1e9, 1)},
        "roofline": {
            "bound": "mfma",
            "achieved": round(kmv_tflops, 1),
            "peak": PEAK_BF16_TFLOPS,
            "unit": "TFLOP/s",
            "frac": round(kmv_tflops / PEAK_BF16_TFLOPS, 4),
            "traffic": counted_traffic(args.prec, n, m),
            "three_product_roof": {"peak": round(three, 1), "frac": round(kmv_tflops / three, 4),
                                   "note": "each multiply of the split product is three MFMA products"},
            "measured_ceilings": ceilings,
        },
        "phases_s": {"sketch": round(last["phases"][0], 3), "build": round(last["phases"][1], 3),
                     "solve": round(last["phases"][2], 3)},
        "solve": {"status": last["rc"], "accepted_fp64": all(rn["accepted"] for rn in runs),
                  "max_relres_true": max(rn["max_relres_true"] for rn in runs),
                  "sampled_rows_max_relres": sampled, "max_iters_per_lambda": per_lambda,
                  "sum_column_iters": sum(iters), "sum_refinements": sum(refs), "rank": last["rank"],
                  "nu": last["nu"]},
        "single_rhs": single,
        "cpu_baseline": cpu,
        "device": device_label(torch),
        "wall_s": round(elapsed(), 1),
    }
    print(json.dumps(out), flush=True)


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU: this build has no multi-GPU path (asked for --gpus {args.gpus})",
              file=sys.stderr)
        sys.exit(2)
    if args.workload != "batched_lambda_grid":
        run_other(args)
        return
    headline(args)


if __name__ == "__main__":
    main()
