#!/usr/bin/env python3
"""Benchmark of the NysPCG hot path on one MI355X.

Workload (default): the batched lambda-grid problem at n = 1e6 points, d = 16,
RBF kernel sigma = 4, 64 right-hand sides b_c = sign(X w_c) times 8 lambdas
log-spaced over [1e-7 n, 1e-3 n] (512 independent columns), one shared Nystrom
sketch of rank 500, BF16X3 kernel products, float32 CG with float64 residual
refinement, tolerance 1e-6 on the float64 true relative residual.

One step = sketch + preconditioner build + PCG to tolerance for every column
(the paper counts the preconditioner build in the solve time, section "Large-Scale
Ridge Regression with NysPCG").  Data generation, device placement and the
Gaussian test matrix are outside the timer; one warmup capped at 10 iterations
precedes the timed steps (section "Hardware, Timing, and Solver Settings").

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

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "NysPCG time-to-1e-6 rel. residual + kernel_matvec TFLOP/s, n=1e6 d=16"
PEAK_BF16_TFLOPS = 2500.0      # MI355X dense bf16 MFMA
HBM_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=1_000_000)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--refine-every", type=int, default=0)
    ap.add_argument("--refine-mode", type=int, default=1)
    ap.add_argument("--refine-reduction", type=float, default=1e-3,
                    help="first cycle factor of the float64 refinement cycles")
    ap.add_argument("--kmv-reps", type=int, default=3)
    ap.add_argument("--cpu-seconds", type=float, default=15.0, help="target CPU time of the oracle sample")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--kmv-only", action="store_true", help="time the kernel product only (profiling)")
    ap.add_argument("--kmv-fp64", default="",
                    help="with --kmv-only: also time the float64 product (the refinement residual) at these "
                         "comma-separated column counts")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="with --kmv-only: first run one plain 1 GiB device copy, whose HBM counter readings "
                         "scale the kernel's (rocprofv3 --pmc FETCH_SIZE / WRITE_SIZE)")
    ap.add_argument("--verbose", action="store_true")
    ap.add_argument("--prec", default="f16x3_d10", choices=["bf16x3", "bf16x3_d6", "bf16x3_d10", "f16x3_d10"],
                    help="kernel-product precision of the batched workload")
    ap.add_argument("--no-autotune", action="store_true",
                    help="skip the tile autotuner (heuristic chunk widths)")
    ap.add_argument("--tile-cache", default=os.path.expanduser("~/.cache/paper_2609_08136_amd/tiles.json"),
                    help="JSON cache of autotuned chunk widths")
    ap.add_argument("--workload", default="batched_lambda_grid",
                    choices=["batched_lambda_grid", "plain_fp64", "matrix_free_fp32", "precision_variant",
                             "differentiation"],
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
    Om = Om0.clone()
    def run():
        P = nys.build_preconditioner(X, Om, w.kind, w.sigma, sketch_prec)
        x, info, rc = nys.nyspcg_solve(X, B, w.lambdas, w.kind, w.sigma, P, tol=w.tol, prec=prec, **opts)
        return x, info, rc, P
    (x, info, rc, P), t = _timed(torch, run)
    return x, info, rc, P, t


def run_other(args):
    import numpy as np
    import torch

    import nys_inputs as ni
    import oracle as o
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
        K = o.kernel_matrix(w.X, w.X, w.kind, w.sigma)
        ref = o.direct_solve(K, w.B[:, 0], w.lambdas[0])
        xs = x.cpu().numpy().reshape(-1)
        t0 = time.perf_counter()
        o.nyspcg_dense(w.X, w.B, w.lambdas, w.kind, w.sigma, ni.gaussian_test_matrix(w.n, w.r, args.seed), tol=w.tol)
        t_cpu = time.perf_counter() - t0
        out.update(metric="NysPCG time-to-1e-8 rel. residual, n=2000 d=10, FP64", value=round(t, 5),
                   ms_per_step=round(t * 1e3, 3), dtype="f64",
                   config={"workload": "plain_fp64", "n": w.n, "d": w.d, "rank": w.r, "lambda": w.lambdas[0],
                           "sigma": w.sigma, "tol": w.tol},
                   solve={"status": rc, "iters": info[0]["iters"], "relres_true": info[0]["relres_true"],
                          "rel_error_vs_cholesky": float(np.linalg.norm(xs - ref) / np.linalg.norm(ref))},
                   cpu_baseline={"value": t_cpu, "unit": "s", "cores": os.cpu_count(), "kind": "oracle",
                                 "sample": "the whole workload: dense K, Nystrom, textbook PCG (float64 NumPy)"})
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
    else:  # differentiation
        from paper_2609_08136_amd import autograd as ag
        w = ni.differentiation(args.seed)
        X, y, Xv, yv = T(w.X), T(w.B[:, 0]), T(w.Xval), T(w.yval)
        g = torch.Generator(device=dev)
        g.manual_seed(args.seed + ni.OMEGA_SEED_OFFSET)
        Om0 = torch.randn((w.n, w.r), generator=g, device=dev, dtype=torch.float64)
        opts = dict(tol=1e-10, prec=nys.FP64)

        def loss_grad(theta):
            P = nys.build_preconditioner(X, Om0.clone(), w.kind, math.exp(theta[1]), nys.FP64)
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
KERNEL_SOURCES = ["kmv_common.h", "kmv_kernels.h", "kmv_host.hip", "kmv_bf16.hip", "kmv_f16.hip"]


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
    """Average duration of one kernel_matvec call (HIP events on the stream it runs on)."""
    g = torch.Generator(device=X.device)
    g.manual_seed(1234)
    dt = torch.float64 if prec == nys.FP64 else torch.float32
    V = torch.randn((X.shape[0], m), generator=g, device=X.device, dtype=dt)
    out = torch.empty_like(V)
    nys.kernel_matvec(X, X, V, nys.RBF, sigma, prec, out=out)     # untimed first call
    torch.cuda.synchronize()
    s = torch.cuda.Event(enable_timing=True)
    e = torch.cuda.Event(enable_timing=True)
    s.record()
    for _ in range(reps):
        nys.kernel_matvec(X, X, V, nys.RBF, sigma, prec, out=out)
    e.record()
    torch.cuda.synchronize()
    t = s.elapsed_time(e) / 1e3 / reps
    del V, out
    return t


def cpu_baseline(args, w, gpu_info):
    """The oracle's K V (float64 NumPy) on a bounded row sample of the same workload,
    scaled to a full time-to-solution estimate with the GPU run's product count."""
    import numpy as np
    import oracle as o

    n, m = w.n, 512
    rng = np.random.default_rng(7)
    V = rng.standard_normal((n, m))
    cores = os.cpu_count() or 1
    rows = 8
    t0 = time.perf_counter()
    o.kernel_matvec_rows(w.X[:rows], w.X, V, w.kind, w.sigma)
    t_small = time.perf_counter() - t0
    rows = max(rows, min(n, int(rows * args.cpu_seconds / max(t_small, 1e-3))))
    t0 = time.perf_counter()
    o.kernel_matvec_rows(w.X[:rows], w.X, V, w.kind, w.sigma)
    t_rows = time.perf_counter() - t0
    t_kv = t_rows * n / rows                       # one full 512-column K V, extrapolated
    kv_equiv = gpu_info["kv_equivalents"]
    est = t_kv * kv_equiv
    return {
        "value": est, "unit": "s", "cores": cores, "kind": "oracle",
        "sample": (f"oracle float64 K(X[0:{rows}], X) V with V n x 512 on the n={n} point set took "
                   f"{t_rows:.1f} s ({cores} host threads, {cpu_model()}); extrapolated x{n / rows:.0f} "
                   f"to one full 512-column product ({t_kv:.0f} s) and x{kv_equiv:.1f} to the GPU run's "
                   f"products (sum of column iterations and float64 refinements / 512)"),
        "kernel_matvec_tflops": n * n * (2 * w.d + 2 * m) / t_kv / 1e12,
    }


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU: this build has no multi-GPU path (asked for --gpus {args.gpus})",
              file=sys.stderr)
        sys.exit(2)
    if args.workload != "batched_lambda_grid":
        run_other(args)
        return

    import numpy as np
    import torch

    import nys_inputs as ni
    import paper_2609_08136_amd as nys

    nys.load()
    dev = torch.device("cuda:0")
    w = ni.batched_lambda_grid(args.seed, n=args.n)
    n, d, r = w.n, w.d, w.r
    nrhs, nlam = w.B.shape[1], len(w.lambdas)
    m = nrhs * nlam
    # the smallest lambda (1e-7 n) lies below the three-term distance error (the operator
    # would be indefinite); the ten-term split also removes the six-term split's structured
    # error, which limits what one float64 refinement cycle gains for the small lambdas
    prec = nys.PREC_BY_NAME[args.prec]
    X = torch.from_numpy(w.X).to(dev)
    B = torch.from_numpy(w.B).to(dev)
    g = torch.Generator(device=dev)
    g.manual_seed(args.seed + ni.OMEGA_SEED_OFFSET)
    Omega0 = torch.randn((n, r), generator=g, device=dev, dtype=torch.float64)
    Om = torch.empty_like(Omega0)
    log(args, f"inputs ready: n={n} d={d} r={r} columns={m}")

    t_tune = 0.0
    tiles = None
    if not args.no_autotune:
        t0 = time.perf_counter()
        tiles = nys.autotune(X, w.kind, w.sigma, prec, m, cache=args.tile_cache, n_rows=min(n, 262144))
        t_tune = time.perf_counter() - t0
        log(args, f"autotune ({t_tune:.1f} s): " + ", ".join(f"{k}: {v['tm']}" for k, v in tiles.items()))
    if args.kmv_only and args.copy_calibration:
        src = torch.ones(1 << 28, dtype=torch.float32, device=dev)      # 1 GiB
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        log(args, "copy calibration: 1 GiB device-to-device copy done")
        del src, dst
    # ---- dominant kernel: the 512-column BF16X3 product (the solve's first product width)
    t_kmv = time_kernel_matvec(nys, torch, X, w.sigma, m, prec, args.kmv_reps)
    flops = n * n * (2 * d + 2 * m)
    kmv_tflops = flops / t_kmv / 1e12
    log(args, f"kernel_matvec m={m}: {t_kmv * 1e3:.1f} ms, {kmv_tflops:.1f} TFLOP/s")
    t_kmv1 = time_kernel_matvec(nys, torch, X, w.sigma, 1, prec, args.kmv_reps)
    log(args, f"kernel_matvec m=1: {t_kmv1 * 1e3:.1f} ms")
    if args.kmv_only:
        res = {"kernel_matvec_ms": t_kmv * 1e3, "tflops": kmv_tflops, "m1_ms": t_kmv1 * 1e3}
        for mc in [int(c) for c in args.kmv_fp64.split(",") if c.strip()]:
            t64 = time_kernel_matvec(nys, torch, X, w.sigma, mc, nys.FP64, args.kmv_reps)
            log(args, f"float64 kernel_matvec m={mc}: {t64 * 1e3:.1f} ms")
            res[f"fp64_m{mc}_ms"] = t64 * 1e3
        print(json.dumps(res))
        return

    ws = torch.empty(nys.nys_workspace_bytes(nys.OP_SOLVE, n, 0, d, r, m, prec), dtype=torch.uint8, device=dev)

    def step(max_iters):
        Om.copy_(Omega0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        Y = nys.nys_sketch(X, Om, w.kind, w.sigma, prec)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        P = nys.nys_precond_build(Y, Om, prec, with_fp32=True)
        del Y
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        Xs, info, rc = nys.nyspcg_solve(X, B, w.lambdas, w.kind, w.sigma, P, tol=w.tol, max_iters=max_iters,
                                        prec=prec, refine_every=args.refine_every, refine_mode=args.refine_mode,
                                        refine_reduction=args.refine_reduction,
                                        workspace=ws)
        torch.cuda.synchronize()
        t3 = time.perf_counter()
        return Xs, info, rc, P, (t1 - t0, t2 - t1, t3 - t2, t3 - t0)

    for _ in range(args.warmup):
        step(10)
        log(args, "warmup done")
    times, phases, last = [], [], None
    for _ in range(args.steps):
        Xs, info, rc, P, ph = step(1000)
        times.append(ph[3])
        phases.append(ph)
        last = (Xs, info, rc, P)
        log(args, f"step: sketch {ph[0]:.2f}s build {ph[1]:.2f}s solve {ph[2]:.2f}s total {ph[3]:.2f}s rc={rc}")
    Xs, info, rc, P = last
    t_step = statistics.median(times)

    # ---- acceptance, after the timer: every column's float64 true relative residual
    rel_true = [c["relres_true"] for c in info]
    ok = all(0 <= v <= w.tol for v in rel_true) and rc == nys.OK
    iters = [c["iters"] for c in info]
    refs = [c["refinements"] for c in info]
    # independent check on 8192 sampled rows: r_i = b_i - (K x)_i - lambda x_i in float64
    # (|r_S| / |b_S| estimates each column's relative residual to a few per cent)
    rows = torch.from_numpy(np.sort(np.random.default_rng(3).choice(n, min(n, 8192), replace=False))).to(dev)
    KX = nys.kernel_matvec(X[rows].contiguous(), X, Xs, w.kind, w.sigma, nys.FP64)
    lam_col = torch.tensor([w.lambdas[c // nrhs] for c in range(m)], dtype=torch.float64, device=dev)
    Bcol = B[:, [c % nrhs for c in range(m)]]
    res = Bcol[rows] - KX - lam_col * Xs[rows]
    sampled = (res.norm(dim=0) / Bcol[rows].norm(dim=0)).max().item()
    per_lambda = {f"{w.lambdas[l]:.3g}": max(iters[l * nrhs:(l + 1) * nrhs]) for l in range(nlam)}
    kv_equiv = (sum(iters) + sum(refs) * 5) / m   # a float64 column product costs ~5 BF16X3 ones
    gpu_info = {"kv_equivalents": kv_equiv}

    cpu = None
    if not args.no_cpu:
        cpu = cpu_baseline(args, w, gpu_info)

    out = {
        "metric": METRIC,
        "value": round(t_step, 3),
        "unit": "s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
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
        },
        "tiles": {"autotune_s": round(t_tune, 1), "widths": {k: v["tm"] for k, v in (tiles or {}).items()}},
        "kernel_matvec_tflops": round(kmv_tflops, 1),
        "kernel_matvec": {"m": m, "ms": round(t_kmv * 1e3, 2), "tflops": round(kmv_tflops, 1),
                          "m1_ms": round(t_kmv1 * 1e3, 2),
                          "m1_gpairs_per_s": round(n * n / t_kmv1 / 1e9, 1)},
        "roofline": {
            "bound": "mfma",
            "achieved": round(kmv_tflops, 1),
            "peak": round(PEAK_BF16_TFLOPS / 3.0, 1),
            "unit": "TFLOP/s",
            "frac": round(kmv_tflops / (PEAK_BF16_TFLOPS / 3.0), 4),
            "traffic": counted_traffic(args.prec, n, m),
        },
        "phases_s": {"sketch": round(phases[-1][0], 3), "build": round(phases[-1][1], 3),
                     "solve": round(phases[-1][2], 3)},
        "solve": {"status": rc, "accepted_fp64": ok, "max_relres_true": max(rel_true),
                  "sampled_rows_max_relres": sampled, "max_iters_per_lambda": per_lambda,
                  "sum_column_iters": sum(iters), "sum_refinements": sum(refs), "rank": P.rank, "nu": P.nu},
        "cpu_baseline": cpu,
        "device": device_label(torch),
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
