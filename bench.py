#!/usr/bin/env python3
"""Throughput of the filtered Paterson-Stockmeyer hot path on one MI355X.

One step = one full evaluation F(Z) = sum_k c_k Z^k by filtered PS (all
powers, coefficient blocks and Horner steps) of the 2D 5-point Laplacian on a
200 x 200 grid (n = 40000, ||Z||_1 = 2), exp series m = 30, s = 6,
tau = 1e-12, with Z resident in HBM.  Prints one JSON line.

    python bench.py [--steps K] [--warmup W] [--gpus 1] [--workload lap2d|lap1d]
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, published
KERNEL_SRC = os.path.join(ROOT, "paper_2208_05683_amd", "csrc", "fps_kernels.hip")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def workload(name):
    from fps_inputs import generators as G

    if name == "lap2d":
        return G.config2()
    if name == "lap1d":
        return G.config1()
    raise SystemExit(f"unknown workload {name}")


def kernel_source_sha256() -> str:
    import hashlib

    with open(KERNEL_SRC, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()


def measured_traffic(workload_name: str):
    """HBM bytes per launch of the numeric kernel from the committed rocprofv3
    FETCH_SIZE / WRITE_SIZE summary, or None if there is none or the kernel
    source changed since it was taken."""
    p = os.path.join(ROOT, "profiles", f"traffic_k_numeric_lds_{workload_name}.json")
    if not os.path.exists(p):
        return None
    with open(p) as f:
        d = json.load(f)
    if d.get("source_sha256") != kernel_source_sha256():
        return None
    return d.get("hbm_bytes_per_launch")


def cpu_baseline(cfg, budget_s: float):
    """The CPU oracle timed on this host's cores on whole evaluations."""
    import oracle as O

    threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or min(16, os.cpu_count() or 1)
    Z, c, m, s, tau = cfg["Z"], cfg["coeffs"], cfg["m"], cfg["s"], cfg["tau"]
    O.filtered_ps(Z, c, m, s, tau, nthreads=threads)  # warm-up
    t0 = time.perf_counter()
    k = 0
    while True:
        O.filtered_ps(Z, c, m, s, tau, nthreads=threads)
        k += 1
        el = time.perf_counter() - t0
        if el >= budget_s or k >= 50:
            break
    return {"value": k / el, "unit": "evals/s", "cores": threads, "kind": "oracle",
            "sample": f"{k} full evaluations of the same workload after 1 warm-up ({el:.1f} s), "
                      f"{threads} OpenMP threads"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="lap2d")
    ap.add_argument("--cpu-budget", type=float, default=12.0, help="seconds of oracle timing (0 skips)")
    ap.add_argument("--filter", choices=["fixed", "adaptive", "series"], default="fixed",
                    help="fixed: the workload's tau; adaptive: Algorithm 1 with the eq. 28 thresholds and the "
                         "eq. 37 bounds; series: Algorithm 2 (N, q and the eq. 36 thresholds from --eps-tol)")
    ap.add_argument("--eps", type=float, default=1e-12, help="adaptive: filtering error budget")
    ap.add_argument("--eps-tol", type=float, default=1e-12, help="series: error tolerance of Algorithm 2")
    ap.add_argument("--e-r", type=float, default=0.1, help="adaptive: Algorithm 1 tolerance")
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="run one device-to-device copy of this many MiB first (calibrates HBM counters)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(how the evaluation would shard is described in DESIGN.md)", file=sys.stderr)
        sys.exit(2)
    if args.steps > 64:
        log("note: kernel timings average the last 64 evaluations")

    import torch
    from paper_2208_05683_amd import api, binding as B

    cfg = workload(args.workload)
    Z = cfg["Z"]
    log(f"workload {cfg['name']}: n={Z.n} nnz={Z.nnz}")
    Zd = api.to_device(Z.row_ptr, Z.col, Z.val)
    stream = torch.cuda.current_stream()
    if args.copy_mib > 0:
        src = torch.ones(args.copy_mib * (1 << 20) // 8, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"copied {args.copy_mib} MiB device to device")
        del src, dst
    series_info = None
    if args.filter == "adaptive":
        # norm bounds of eq. 37 computed by the library on the device
        plan = api.Plan(Zd, cfg["coeffs"], cfg["m"], cfg["s"], adaptive=True, eps=args.eps, e_r=args.e_r,
                        znorm=None, flags=B.FPS_FLAG_TIMING)
        cfg = dict(cfg, name=cfg["name"] + f"_adaptive_eps{args.eps:g}")
    elif args.filter == "series":
        from fps_inputs import generators as G

        plan = api.Plan.series(Zd, G.exp_coeffs(59), args.eps_tol, args.e_r, flags=B.FPS_FLAG_TIMING)
        series_info = plan.series_info()
        cfg = dict(cfg, name=cfg["name"].split("_m")[0] + f"_exp_series_tol{args.eps_tol:g}",
                   m=series_info["N"] - 1, s=series_info["q"])
        log(f"series mode: N = {series_info['N']}, q = {series_info['q']}, tail = {series_info['tail']:.3g}")
    else:
        plan = api.Plan(Zd, cfg["coeffs"], cfg["m"], cfg["s"], cfg["tau"], flags=B.FPS_FLAG_TIMING)

    for i in range(args.warmup):
        plan.eval(stream)
    torch.cuda.synchronize()
    log(f"warm-up done ({args.warmup} evals), F nnz = {plan.nnz()}")

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        plan.eval(stream)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    st = plan.stats()
    if st["resizes"]:
        log(f"warning: {st['resizes']} evaluations re-sized buffers")
    ms_per_step = 1e3 * el / args.steps
    evals_per_s = args.steps / el
    log(f"timed {args.steps} evals: {ms_per_step:.3f} ms/eval")

    # roofline of the dominant kernel, the shared-memory numeric kernel (every
    # stage launches it once; HIP events on the plan's stream around each launch)
    launches = st["numeric_launches"]
    kern_ms = st["numeric_ms"]
    bytes_eval = st["bytes_algorithmic"]
    achieved = (bytes_eval / (kern_ms * 1e-3)) / 1e9 if kern_ms > 0 else 0.0
    products = st["products"]
    prod_per_s = products / (ms_per_step * 1e-3)

    res = {
        "metric": "series evals/s + SpGEMM HBM GB/s vs plain filtered PS; p50/p99 latency at QPS",
        "value": evals_per_s,
        "unit": "evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": cfg["name"], "n": Z.n, "nnz_Z": Z.nnz, "m": cfg["m"], "s": cfg["s"],
                   "filter": args.filter,
                   **({"tau": cfg["tau"]} if args.filter == "fixed" else
                      {"eps": args.eps, "e_r": args.e_r} if args.filter == "adaptive" else
                      {"eps_tol": args.eps_tol, "e_r": args.e_r, "N": series_info["N"]}),
                   "series": "exp", "nnz_F": st["nnz_out"]},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": measured_traffic(cfg["name"]),
                     "traffic_unit": "HBM bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
                     "algorithmic_bytes_per_launch": bytes_eval / launches if launches else None,
                     "kernel": "k_numeric_lds",
                     "launches_per_step": launches,
                     "avg_launch_ms": kern_ms / launches if launches else None,
                     "algorithmic_bytes_per_step": bytes_eval},
        "products_per_s": prod_per_s,
        "products_per_step": products,
        "products_skipped_per_step": st["products_skipped"],
        "stage_ms": {f"{['power', 'block', 'gstep', 'horner'][k]}{i}": round(ms, 4)
                     for k, i, ms in zip(st["kind"], st["index"], st["stage_ms"])},
    }
    if args.filter != "fixed":
        res["alg1_iters_per_step"] = int(sum(st["stage_alg1_iters"]))
    if args.cpu_budget > 0 and args.filter == "fixed":
        log("timing the CPU oracle ...")
        res["cpu_baseline"] = cpu_baseline(cfg, args.cpu_budget)
    plan.close()
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
