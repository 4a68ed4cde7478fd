#!/usr/bin/env python3
"""Throughput of the filtered Paterson-Stockmeyer hot path on one MI355X.

One step = one full evaluation F(Z) = sum_k c_k Z^k by filtered PS (all
powers, coefficient blocks and Horner steps) of the 2D 5-point Laplacian on a
200 x 200 grid (n = 40000, ||Z||_1 = 2), exp series m = 30, s = 6,
tau = 1e-12, with Z resident in HBM.  Prints one JSON line.

    python bench.py [--steps K] [--warmup W] [--gpus 1] [--workload lap2d|lap1d]

Other lines (not the headline): --filter adaptive|series time Algorithm 1 and
Algorithm 2 on the same matrix; --sweep banded times the paper's second test
set (random banded 1000 x 1000, bandwidth 1..15, exp and cos, eps_tol 1e-14)
against the unfiltered scheme and a dense fp64 Horner.
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


def dense_ps(Zt, c, m, s):
    """Plain PS (eqs. 2-6) on a dense fp64 device matrix: powers, blocks and the
    Horner recurrence as GEMMs (the dense comparison of the banded sweep)."""
    import torch

    n = Zt.shape[0]
    N, q = m + 1, s
    b = -(-N // q)
    eye = torch.eye(n, dtype=torch.float64, device=Zt.device)
    J = q if b >= 2 else m
    P = [eye, Zt]
    for _ in range(2, J + 1):
        P.append(Zt @ P[-1])

    def block(i, jmax):
        acc = torch.zeros_like(Zt)
        for j in range(jmax + 1):
            k = i * q + j
            if k <= m and c[k] != 0.0:
                acc = acc + float(c[k]) * P[j]
        return acc

    if b == 1:
        return block(0, q - 1)
    g = 1 if N - q * (b - 1) == 1 else 0
    S = block(b - 2, q) if g else block(b - 1, q - 1)
    for i in range(1 + g, b):
        S = block(b - 1 - i, q - 1) + P[q] @ S
    return S


def banded_sweep(count: int, eps_tol: float, e_r: float, bands):
    """The paper's second test set on the GPU: for each bandwidth, `count`
    matrices; the series mode (Algorithm 2), the unfiltered scheme with the same
    N and q, and the dense Horner, timed per matrix; sparsity of F; relative
    Frobenius errors against the matrix exponential / cosine computed densely
    (torch.linalg.matrix_exp, cos through the complex exponential)."""
    import numpy as np
    import torch
    from fps_inputs import generators as G
    from paper_2208_05683_amd import api

    def dev_ms(fn):
        torch.cuda.synchronize()
        t = time.perf_counter()
        out = fn()
        torch.cuda.synchronize()
        return out, 1e3 * (time.perf_counter() - t)

    def dense(csr):
        rp, cl, vl = (x.cpu().numpy() for x in csr)
        rows = np.repeat(np.arange(len(rp) - 1), np.diff(rp))
        d = torch.zeros((len(rp) - 1, len(rp) - 1), dtype=torch.float64)
        d[rows, cl] = torch.from_numpy(vl)
        return d.cuda()

    out = []
    for fname, coeffs in (("exp", G.exp_coeffs(199)), ("cos", G.cos_coeffs(199))):
        rows = []
        for bw in bands:
            acc = {k: [] for k in ("psscf_setup_ms", "psscf_ms", "ps_ms", "dense_ms", "sparsity_psscf",
                                   "sparsity_ps", "err_psscf", "err_ps", "N", "q")}
            for k in range(count):
                Z = G.banded_sweep_matrix(bw, 1000, seed=1000 * bw + k)
                Zd = api.to_device(Z.row_ptr, Z.col, Z.val)
                plan, t_setup = dev_ms(lambda: api.Plan.series(Zd, coeffs, eps_tol, e_r))
                info = plan.series_info()
                plan.eval()  # sizing run
                _, t_eval = dev_ms(plan.eval)
                F = plan.result()
                plan.close()
                m, s = info["N"] - 1, info["q"]
                ps = api.Plan(Zd, coeffs, m, s, 0.0)
                ps.eval()
                _, t_ps = dev_ms(ps.eval)
                Fps = ps.result()
                ps.close()
                Zt = dense((Zd[0], Zd[1], Zd[2]))
                dense_ps(Zt, coeffs, m, s)  # warm-up
                _, t_dense = dev_ms(lambda: dense_ps(Zt, coeffs, m, s))
                if fname == "exp":
                    ref = torch.linalg.matrix_exp(Zt)
                else:
                    ref = torch.linalg.matrix_exp(1j * Zt.to(torch.complex128)).real
                nref = torch.linalg.norm(ref)
                acc["err_psscf"].append(float(torch.linalg.norm(dense(F) - ref) / nref))
                acc["err_ps"].append(float(torch.linalg.norm(dense(Fps) - ref) / nref))
                acc["sparsity_psscf"].append(F[1].numel() / Z.n ** 2)
                acc["sparsity_ps"].append(Fps[1].numel() / Z.n ** 2)
                for key, v in (("psscf_setup_ms", t_setup), ("psscf_ms", t_eval), ("ps_ms", t_ps),
                               ("dense_ms", t_dense), ("N", info["N"]), ("q", info["q"])):
                    acc[key].append(v)
            row = {"b": bw, **{k: float(np.mean(v)) for k, v in acc.items()}}
            log(f"{fname} b={bw}: " + ", ".join(f"{k}={v:.3g}" for k, v in row.items() if k != "b"))
            rows.append(row)
        out.append({"function": fname, "rows": rows})
    return out


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
    ap.add_argument("--sweep", choices=["banded"], default=None,
                    help="banded: the paper's second test set instead of the headline workload")
    ap.add_argument("--sweep-count", type=int, default=30, help="sweep: matrices per bandwidth")
    ap.add_argument("--sweep-bands", default="1-15", help="sweep: bandwidths, e.g. 1-15 or 1,5,11")
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="run one device-to-device copy of this many MiB first (calibrates HBM counters)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(the throughput reported is that of a single GPU)", file=sys.stderr)
        sys.exit(2)
    if args.steps > 8 * 64:
        log("note: kernel timings average the last 64 sampled evaluations (every 8th one)")

    import torch
    from paper_2208_05683_amd import api, binding as B

    if args.sweep == "banded":
        if "-" in args.sweep_bands:
            lo, hi = (int(x) for x in args.sweep_bands.split("-"))
            bands = list(range(lo, hi + 1))
        else:
            bands = [int(x) for x in args.sweep_bands.split(",")]
        tol = args.eps_tol if args.eps_tol != 1e-12 else 1e-14
        res = {"sweep": "banded", "n": 1000, "matrices_per_band": args.sweep_count, "eps_tol": tol,
               "e_r": args.e_r, "data": "synthetic: every in-band entry N(0, 1), seed 1000 b + k",
               "results": banded_sweep(args.sweep_count, tol, args.e_r, bands)}
        print(json.dumps(res), flush=True)
        return

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
    torch.cuda.synchronize()
    t_setup = time.perf_counter()
    if args.filter == "adaptive":
        # norm bounds of eq. 37 computed by the library on the device
        plan = api.Plan(Zd, cfg["coeffs"], cfg["m"], cfg["s"], adaptive=True, eps=args.eps, e_r=args.e_r,
                        znorm=None, flags=B.FPS_FLAG_TIMING)
        cfg = dict(cfg, name=cfg["name"] + f"_adaptive_eps{args.eps:g}")
    elif args.filter == "series":
        from fps_inputs import generators as G

        plan = api.Plan.series(Zd, G.exp_coeffs(59), args.eps_tol, args.e_r, flags=B.FPS_FLAG_TIMING)
        series_info = plan.series_info()
        cfg = dict(cfg, name=cfg["name"].split("_m")[0] + f"_series_tol{args.eps_tol:g}",
                   m=series_info["N"] - 1, s=series_info["q"])
        log(f"series mode: N = {series_info['N']}, q = {series_info['q']}, tail = {series_info['tail']:.3g}")
    else:
        plan = api.Plan(Zd, cfg["coeffs"], cfg["m"], cfg["s"], cfg["tau"], flags=B.FPS_FLAG_TIMING)
    torch.cuda.synchronize()
    setup_ms = 1e3 * (time.perf_counter() - t_setup)  # plan creation (with the norm estimates of eq. 37)

    for i in range(args.warmup):
        plan.eval(stream)
    torch.cuda.synchronize()
    log(f"warm-up done ({args.warmup} evals), F nnz = {plan.nnz()}")
    plan.stats()  # the kernel times reported below are those of the timed evaluations

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
    # stage launches it once; HIP events on the plan's stream around each launch
    # of the first timed evaluation and every 8th one after it)
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
        "plan_setup_ms": setup_ms,
        "rows_wide_per_step": st["rows_wide"],
        "rows_global_per_step": st["rows_global"],
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
