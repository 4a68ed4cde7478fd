#!/usr/bin/env python3
"""Throughput of the filtered Paterson-Stockmeyer hot path on one MI355X.

One step = one full evaluation F(Z) = sum_k c_k Z^k by filtered PS (all
powers, coefficient blocks and Horner steps) of the 2D 5-point Laplacian on a
200 x 200 grid (n = 40000, ||Z||_1 = 2), exp series m = 30, s = 6,
tau = 1e-12, with Z resident in HBM.  Prints one JSON line.

    python bench.py [--steps K] [--warmup W] [--gpus 1] [--workload lap2d|lap1d]

The headline line also carries the batched leg (512 seeded banded instances
in one graph-replayed batch against 512 plain evaluations; --batch-count 0
skips it), the serving leg (the server against plain sequential evaluations
on the mixed request stream, saturation and Poisson arrivals with p50/p99;
--serve-requests 0 skips it) and the CPU oracle baseline (--cpu-budget 0
skips it).

Other lines (not the headline): --filter adaptive|series time Algorithm 1 and
Algorithm 2 on the same matrix; --workload lap3d|banded (with --side) and
--dense|--dense-exact take other matrices and the dense paths; --sweep banded
times the paper's second test set (random banded 1000 x 1000, bandwidth
1..15, exp and cos, eps_tol 1e-14) against the unfiltered scheme and a dense
fp64 Horner.
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


def workload(name, side=None):
    from fps_inputs import generators as G

    if name == "lap2d":
        return G.config2()
    if name == "lap1d":
        return G.config1()
    if name == "lap3d":
        return G.config3(side=side or 20)
    if name == "banded":
        # one matrix of the paper's second test set (n = 1000, half-bandwidth
        # b = side, default 15, the sweep's first seed for that b)
        b = side or 15
        return dict(name=f"banded_n1000_b{b}_exp_m30_s6", Z=G.banded_sweep_matrix(b, 1000, seed=1000 * b),
                    coeffs=G.exp_coeffs(30), m=30, s=6, tau=1e-12)
    raise SystemExit(f"unknown workload {name}")


def kernel_source_sha256() -> str:
    import hashlib

    with open(KERNEL_SRC, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()


def measured_traffic(workload_name: str, kernel: str):
    """HBM bytes per launch of a numeric kernel from the committed rocprofv3
    FETCH_SIZE / WRITE_SIZE summary, or None if there is none or the kernel
    source changed since it was taken."""
    p = os.path.join(ROOT, "profiles", f"traffic_{kernel}_{workload_name}.json")
    if not os.path.exists(p):
        return None
    with open(p) as f:
        d = json.load(f)
    if d.get("source_sha256") != kernel_source_sha256():
        return None
    return d.get("hbm_bytes_per_launch")


def host_cpu():
    """nproc and the CPU model of this host."""
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return os.cpu_count() or 1, model


def cpu_baseline(cfg, reps: int = 5):
    """The CPU oracle on this host's cores, whole evaluations of the same
    workload: median of `reps` runs after one warm-up, with OpenMP on all the
    cores the run may use and on one core."""
    import statistics

    import oracle as O

    nproc, model = host_cpu()
    threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or nproc
    Z, c, m, s, tau = cfg["Z"], cfg["coeffs"], cfg["m"], cfg["s"], cfg["tau"]

    def med(nt):
        O.filtered_ps(Z, c, m, s, tau, nthreads=nt)  # warm-up
        ts = []
        for _ in range(reps):
            t0 = time.perf_counter()
            O.filtered_ps(Z, c, m, s, tau, nthreads=nt)
            ts.append(time.perf_counter() - t0)
        return statistics.median(ts)

    t_all = med(threads)
    t_one = med(1)
    return {"value": 1.0 / t_all, "unit": "evals/s", "cores": threads, "kind": "oracle",
            "sample": f"median of {reps} full evaluations of the same workload after 1 warm-up, "
                      f"{threads} OpenMP threads",
            "value_1core": 1.0 / t_one, "median_s": t_all, "median_s_1core": t_one,
            "nproc": nproc, "cpu_model": model}


def event_times(run, steps, stream):
    """Per-step milliseconds from HIP events on `stream` around each call."""
    import torch

    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for a, b in evs:
        a.record(stream)
        run()
        b.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return [a.elapsed_time(b) for a, b in evs], wall


def median(v):
    import statistics

    return statistics.median(v)


def bench_serve(args, stream):
    """The server on the serving mix (n log-uniform in [1000, 60000], half 2D
    Laplacians and half random banded matrices, exp / cos / random series,
    m in 12..30, tau = 1e-12; a pool of distinct requests kept on the device
    and submitted in turn).  Throughputs: plain sequential evaluations (plan,
    evaluation, result size, release, one request after the other, as the
    plain API does them) and, at saturation (the median of three runs), a
    one-slot server (the plain path behind a queue, buffers reused) and the
    multi-slot server.  Then
    Poisson arrivals at fractions of the plain rate and of the server's
    saturation rate, with p50/p99 of arrival-to-result-ready latency.  Both
    servers are long-lived and warmed on the request pool first."""
    import threading

    import numpy as np
    import torch
    from fps_inputs import generators as G
    from paper_2208_05683_amd import api

    pool = G.serving_requests(count=args.serve_pool, seed=5)
    dev = [api.to_device(r["Z"].row_ptr, r["Z"].col, r["Z"].val) for r in pool]
    q = [max(1, int(np.floor(np.sqrt(r["m"])))) for r in pool]
    torch.cuda.synchronize()

    def plain_one(k):
        r = pool[k % len(pool)]
        p = api.Plan(dev[k % len(pool)], r["coeffs"], r["m"], q[k % len(pool)], r["tau"])
        p.eval(stream)
        p.nnz()
        p.close()

    for k in range(min(8, len(pool))):  # warm-up
        plain_one(k)
    nplain = args.serve_requests
    t0 = time.perf_counter()
    for k in range(nplain):
        plain_one(k)
    x_plain = nplain / (time.perf_counter() - t0)

    budget = int(args.serve_budget_gib * (1 << 30))
    count = args.serve_requests

    def run(sv, rate, n, offset, seed):
        """n requests (rate None: all at once); returns throughput, latencies
        (ms) and the number that failed."""
        infos, tickets = [], []
        done_evt = threading.Event()

        def consumer():
            for i in range(n):
                while len(tickets) <= i:
                    time.sleep(0.0002)
                t = tickets[i]
                sv.wait(t, -1)
                infos.append(sv.info(t))
                sv.release(t)
            done_evt.set()

        th = threading.Thread(target=consumer)
        th.start()
        rng = np.random.default_rng(seed)
        arrivals = np.zeros(n) if rate is None else np.cumsum(rng.exponential(1.0 / rate, n))
        start = time.perf_counter()
        for i in range(n):
            k = (offset + i) % len(pool)
            wait = start + arrivals[i] - time.perf_counter()
            if wait > 0:
                time.sleep(wait)
            r = pool[k]
            tickets.append(sv.submit(dev[k], r["coeffs"], r["m"], r["tau"], s=q[k]))
        done_evt.wait()
        th.join()
        t_first = min(x["t_submit_ns"] for x in infos)
        t_last = max(x["t_done_ns"] for x in infos)
        lat = [(x["t_done_ns"] - x["t_submit_ns"]) * 1e-6 for x in infos]
        failed = sum(1 for x in infos if x["state"] != 2)
        return n / ((t_last - t_first) * 1e-9), lat, failed

    slots = args.serve_slots
    servers = {"one_slot": api.Server(slots=1, hbm_budget=budget, max_queue=count + 8),
               "server": api.Server(slots=slots, hbm_budget=budget, max_queue=count + 8)}
    try:
        for sv in servers.values():  # warm: threads, streams and the buffer pools
            run(sv, None, len(pool), 0, 1)
        # saturation: three runs of `count` requests submitted at once, the
        # run of median throughput reported (one run alone can be spoiled by
        # a single stall of the host or the device)
        sat = {}
        for name, sv in servers.items():
            runs = sorted((run(sv, None, count, 0, 2 + k) for k in range(3)), key=lambda t: t[0])
            x, lat, failed = runs[1]
            sat[name] = {"evals_per_s": x, "p50_ms": float(np.percentile(lat, 50)),
                         "p99_ms": float(np.percentile(lat, 99)), "failed": failed,
                         "runs_evals_per_s": [t[0] for t in runs]}
        x_srv = sat["server"]["evals_per_s"]
        levels = []
        for base_name, base in (("plain", x_plain), ("server", x_srv)):
            for frac in (0.25, 0.5, 0.75, 0.9):
                rate = frac * base
                row = {"fraction_of": f"{base_name} saturation", "fraction": frac, "qps": rate}
                for name, sv in servers.items():
                    if base_name == "server" and name == "one_slot" and rate > sat["one_slot"]["evals_per_s"]:
                        row[name] = "overloaded: offered rate above its saturation throughput"
                        continue
                    x, lat, failed = run(sv, rate, count, 17, int(1000 * frac) + len(base_name))
                    row[name] = {"evals_per_s": x, "p50_ms": float(np.percentile(lat, 50)),
                                 "p99_ms": float(np.percentile(lat, 99)), "failed": failed}
                log(f"serve {frac:.2f} x {base_name} ({rate:.0f} qps): " + "; ".join(
                    f"{k} p50 {v['p50_ms']:.2f} p99 {v['p99_ms']:.2f} ms" for k, v in row.items()
                    if isinstance(v, dict)))
                levels.append(row)
        stats = {name: sv.stats() for name, sv in servers.items()}
    finally:
        for sv in servers.values():
            sv.close()
    return {
        "workload": "serving_mix_n1000-60000_lap2d-banded_exp-cos-rand_m12-30",
        "distinct_requests": len(pool), "requests_per_run": count, "slots": slots,
        "budget_GiB": args.serve_budget_gib,
        "plain_sequential_evals_per_s": x_plain,
        "saturation": sat,
        "server_saturation_evals_per_s": x_srv,
        "speedup_vs_plain": x_srv / x_plain,
        "speedup_vs_one_slot": x_srv / sat["one_slot"]["evals_per_s"],
        "poisson": levels,
        "server_stats": {k: {kk: v[kk] for kk in ("completed", "failed", "retries", "grows", "peak_running",
                                                   "peak_reserved")} for k, v in stats.items()},
    }


def bench_batch(args, stream):
    """The batched layer against the plain path on 512 seeded banded instances
    (n log-uniform in [500, 20000], half-bandwidth 1..5, in-band density 0.6,
    ||Z||_1 ~ U(0.5, 2), exp m = 20, tau = 1e-12 ||Z||_1, s in {4, 5} from the
    autotuner): one batch evaluation (a graph replay) against 512 fps_eval
    calls of plans with the same s, both after their sizing evaluations."""
    import numpy as np
    import torch
    from fps_inputs import generators as G
    from paper_2208_05683_amd import api

    inst = G.batch_instances(count=args.batch_count)
    dev = [api.to_device(x["Z"].row_ptr, x["Z"].col, x["Z"].val) for x in inst]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    b = api.Batch([dict(Zd=d, coeffs=x["coeffs"], m=x["m"], s=0, tau=x["tau"]) for d, x in zip(dev, inst)],
                  s_lo=4, s_hi=5)
    torch.cuda.synchronize()
    create_ms = 1e3 * (time.perf_counter() - t0)
    chosen = [b.item_info(i)["s"] for i in range(len(inst))]
    for _ in range(3):  # sizing, the eager one, then the graph capture
        b.eval(stream)
    torch.cuda.synchronize()
    bt, bwall = event_times(lambda: b.eval(stream), args.batch_steps, stream)
    bst = b.stats()
    plans = [api.Plan(d, x["coeffs"], x["m"], s, x["tau"]) for d, x, s in zip(dev, inst, chosen)]
    for p in plans:
        p.eval(stream)
        p.eval(stream)
    torch.cuda.synchronize()

    def seq():
        for p in plans:
            p.eval(stream)

    pt, pwall = event_times(seq, args.batch_steps, stream)
    # spot check: the batch gives each instance's own result
    same = 0
    for i in range(0, len(inst), max(1, len(inst) // 16)):
        g = [x.cpu().numpy() for x in b.result(i)]
        h = [x.cpu().numpy() for x in plans[i].result()]
        same += int(all(np.array_equal(u.view(np.uint8), v.view(np.uint8)) for u, v in zip(g, h)))
    checked = len(range(0, len(inst), max(1, len(inst) // 16)))
    products = bst["products"]
    for p in plans:
        p.close()
    b.close()
    bms, pms = median(bt), median(pt)
    return {
        "workload": f"batch{len(inst)}_banded_exp_m20",
        "instances": len(inst), "rows": bst["rows"], "groups": bst["groups"],
        "s_chosen": {"4": chosen.count(4), "5": chosen.count(5)},
        "batch_ms": bms, "batch_evals_per_s": len(inst) / (bms * 1e-3),
        "plain_ms": pms, "plain_evals_per_s": len(inst) / (pms * 1e-3),
        "speedup_vs_plain": pms / bms,
        "graph": bst["graph"], "steps": args.batch_steps,
        "batch_wall_ms_per_step": 1e3 * bwall / args.batch_steps,
        "plain_wall_ms_per_step": 1e3 * pwall / args.batch_steps,
        "create_ms": create_ms, "products_per_step": products,
        "bytes_algorithmic_per_step": bst["bytes_algorithmic"],
        "hbm_frac_algorithmic": bst["bytes_algorithmic"] / (bms * 1e-3) / 1e9 / HBM_PEAK_GBS,
        "nnz_out": bst["nnz_out"], "results_checked_bitwise": f"{same}/{checked}",
    }


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
            acc = {k: [] for k in ("psscf_setup_ms", "psscf_ms", "psscf_mfma_ms", "psscf_exact_ms", "ps_ms",
                                   "dense_ms", "sparsity_psscf", "sparsity_ps", "err_psscf", "err_psscf_mfma",
                                   "err_ps", "exact_bitwise", "N", "q")}
            for k in range(count):
                Z = G.banded_sweep_matrix(bw, 1000, seed=1000 * bw + k)
                Zd = api.to_device(Z.row_ptr, Z.col, Z.val)
                plan, t_setup = dev_ms(lambda: api.Plan.series(Zd, coeffs, eps_tol, e_r))
                info = plan.series_info()
                plan.eval()  # sizing run
                _, t_eval = dev_ms(plan.eval)
                F = plan.result()
                plan.close()
                # the same with the dense products on the matrix cores
                from paper_2208_05683_amd import binding as B

                pm = api.Plan.series(Zd, coeffs, eps_tol, e_r, flags=B.FPS_FLAG_DENSE)
                pm.eval()
                _, t_mfma = dev_ms(pm.eval)
                Fm = pm.result()
                pm.close()
                # the exact dense paths: the sparse result bit for bit
                px = api.Plan.series(Zd, coeffs, eps_tol, e_r, flags=B.FPS_FLAG_DENSE_EXACT)
                px.eval()
                _, t_exact = dev_ms(px.eval)
                Fx = px.result()
                px.close()
                same = all(a.shape == b.shape and torch.equal(a.view(torch.int64) if a.dtype == torch.float64 else a,
                                                             b.view(torch.int64) if b.dtype == torch.float64 else b)
                           for a, b in zip(F, Fx))
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
                acc["err_psscf_mfma"].append(float(torch.linalg.norm(dense(Fm) - ref) / nref))
                acc["sparsity_psscf"].append(F[1].numel() / Z.n ** 2)
                acc["sparsity_ps"].append(Fps[1].numel() / Z.n ** 2)
                for key, v in (("psscf_setup_ms", t_setup), ("psscf_ms", t_eval), ("psscf_mfma_ms", t_mfma),
                               ("psscf_exact_ms", t_exact), ("exact_bitwise", 1.0 if same else 0.0),
                               ("ps_ms", t_ps),
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
    ap.add_argument("--workload", default="lap2d",
                    help="lap2d (headline), lap1d, lap3d (with --side), banded (n = 1000, half-bandwidth --side)")
    ap.add_argument("--side", type=int, default=None, help="lap3d: grid side (default 20); banded: half-bandwidth (default 15)")
    ap.add_argument("--dense", action="store_true", help="FPS_FLAG_DENSE: dense products on the FP64 matrix cores")
    ap.add_argument("--dense-exact", action="store_true",
                    help="FPS_FLAG_DENSE_EXACT: filled-in products on the exact dense paths (bitwise)")
    ap.add_argument("--no-small", action="store_true",
                    help="FPS_FLAG_NO_SMALL: every row on a 64-lane wavefront (no small-row tier)")
    ap.add_argument("--cpu-budget", type=float, default=1.0, help="0 skips the CPU oracle timing")
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
    ap.add_argument("--batch-count", type=int, default=512, help="instances of the batch leg (0 skips it)")
    ap.add_argument("--batch-steps", type=int, default=10, help="timed batch evaluations")
    ap.add_argument("--serve-requests", type=int, default=200, help="requests per serving run (0 skips the leg)")
    ap.add_argument("--serve-pool", type=int, default=96, help="distinct serving requests kept on the device")
    ap.add_argument("--serve-slots", type=int, default=8, help="server slots")
    ap.add_argument("--serve-budget-gib", type=float, default=96.0, help="server device-memory budget")
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

    cfg = workload(args.workload, args.side)
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

        plan = api.Plan.series(Zd, G.exp_coeffs(59), args.eps_tol, args.e_r,
                               flags=B.FPS_FLAG_TIMING | (B.FPS_FLAG_DENSE if args.dense else 0)
                               | (B.FPS_FLAG_DENSE_EXACT if args.dense_exact else 0))
        series_info = plan.series_info()
        dense_tag = "_dense" if args.dense else "_dense_exact" if args.dense_exact else ""
        cfg = dict(cfg, name=cfg["name"].split("_m")[0] + f"_series_tol{args.eps_tol:g}" + dense_tag,
                   m=series_info["N"] - 1, s=series_info["q"])
        log(f"series mode: N = {series_info['N']}, q = {series_info['q']}, tail = {series_info['tail']:.3g}")
    else:
        plan = api.Plan(Zd, cfg["coeffs"], cfg["m"], cfg["s"], cfg["tau"],
                        flags=B.FPS_FLAG_TIMING | (B.FPS_FLAG_DENSE if args.dense else 0)
                        | (B.FPS_FLAG_DENSE_EXACT if args.dense_exact else 0)
                        | (B.FPS_FLAG_NO_SMALL if args.no_small else 0))
        if args.dense:
            cfg = dict(cfg, name=cfg["name"] + "_dense")
        elif args.dense_exact:
            cfg = dict(cfg, name=cfg["name"] + "_dense_exact")
    torch.cuda.synchronize()
    setup_ms = 1e3 * (time.perf_counter() - t_setup)  # plan creation (with the norm estimates of eq. 37)

    try:
        for i in range(max(1, args.warmup)):
            plan.eval(stream)
        nnz_first = plan.nnz()
    except B.FpsError as e:
        if e.status != B.FPS_ERR_CAPACITY:
            raise
        # the fill outgrew the device: report the library's footprint message
        print(json.dumps({"metric": "series evals/s + SpGEMM HBM GB/s vs plain filtered PS; p50/p99 latency at QPS",
                          "value": None, "unit": "evals/s", "n_gpus": 1, "status": e.status,
                          "message": str(e), "config": {"workload": cfg["name"], "n": Z.n, "nnz_Z": Z.nnz}}),
              flush=True)
        return
    torch.cuda.synchronize()
    log(f"warm-up done ({args.warmup} evals), F nnz = {nnz_first}")
    plan.stats()  # the kernel times reported below are those of the timed evaluations

    # each evaluation timed by HIP events on the stream it runs on; the value
    # is the median (the bracketed wall time is reported beside it)
    times, el = event_times(lambda: plan.eval(stream), args.steps, stream)
    st = plan.stats()
    if st["resizes"]:
        log(f"warning: {st['resizes']} evaluations re-sized buffers")
    ms_per_step = median(times)
    evals_per_s = 1e3 / ms_per_step
    log(f"timed {args.steps} evals: median {ms_per_step:.3f} ms/eval (wall {1e3 * el / args.steps:.3f})")

    # roofline of the dominant kernel, the shared-memory numeric kernel (every
    # stage launches it once; the library records HIP events on the plan's
    # stream around each launch of the first timed evaluation and every 8th
    # one after it).  Algorithmic bytes count the rows each stage computes
    # (a stage whose rows were all proven empty counts its analysis reads).
    launches = st["numeric_launches"]
    kern_ms = st["numeric_ms"]
    bytes_eval = st["bytes_algorithmic"]
    # the numeric kernel's own bytes: a stage whose rows were all proven empty
    # by the analysis only writes each row's (empty) end in it, 8 bytes a row
    n1 = Z.n + 1
    kern_bytes = [8.0 * n1 if sk >= Z.n else by for by, sk in zip(st["stage_bytes"], st["stage_rows_skipped"])]
    bytes_kernel = sum(kern_bytes)
    achieved = (bytes_kernel / (kern_ms * 1e-3)) / 1e9 if kern_ms > 0 else 0.0
    products = st["products"]
    prod_per_s = products / (ms_per_step * 1e-3)
    names = [f"{['power', 'block', 'gstep', 'horner'][k]}{i}" for k, i in zip(st["kind"], st["index"])]
    stages = {}
    for nm, ms, by, pr, sk, mn, mw in zip(names, st["stage_ms"], kern_bytes, st["stage_products"],
                                          st["stage_rows_skipped"], st["stage_max_ns"], st["stage_max_words"]):
        gbs = by / (ms * 1e-3) / 1e9 if ms > 0 else 0.0
        stages[nm] = {"us": round(1e3 * ms, 2), "bytes": by, "GBps": round(gbs, 1),
                      "frac": round(gbs / HBM_PEAK_GBS, 4), "products": pr, "rows_skipped": sk,
                      "max_row": mn, "max_window_words": mw}
    dom = max(stages, key=lambda k: stages[k]["us"]) if stages else None
    dense_ld = st.get("dense_ld", 0)
    dense_stages = [nm for nm, d in zip(names, st["stage_dense"]) if d == 1]  # on the matrix cores
    # the stages by the kernel that ran them: the small-row tier, the dense
    # path, or the 64-lane shared-memory kernel (with its fallback tiers)
    kernels = {}
    for i, nm in enumerate(names):
        k = {1: "k_dgemm_mfma", 2: "k_spmm_rows", 3: "k_dgemm_ordered"}.get(
            st["stage_dense"][i], "k_numeric_small" if st["stage_small"][i] else "k_numeric_lds")
        stages[nm]["kernel"] = k
        d = kernels.setdefault(k, {"launches": 0, "us": 0.0, "bytes": 0.0, "stages": []})
        d["launches"] += 1
        d["us"] += stages[nm]["us"]
        d["bytes"] += kern_bytes[i]
        d["stages"].append(nm)
    for d in kernels.values():
        d["us"] = round(d["us"], 2)
        d["avg_launch_us"] = round(d["us"] / d["launches"], 2)
        d["GBps"] = round(d["bytes"] / (d["us"] * 1e-6) / 1e9, 1) if d["us"] > 0 else 0.0
        d["frac"] = round(d["GBps"] / HBM_PEAK_GBS, 4)
    sparse_k = {k: d for k, d in kernels.items() if k not in ("k_dgemm_mfma", "k_spmm_rows", "k_dgemm_ordered")}
    dom_k = max(sparse_k, key=lambda k: sparse_k[k]["us"]) if sparse_k else "k_numeric_lds"
    dk = kernels.get(dom_k, {"launches": 0, "us": 0.0, "bytes": 0.0})
    k_launches, k_ms, k_bytes = dk["launches"], dk["us"] / 1e3, dk["bytes"]
    k_achieved = (k_bytes / (k_ms * 1e-3)) / 1e9 if k_ms > 0 else 0.0
    traffic = measured_traffic(cfg["name"], dom_k)
    for nm in dense_stages:
        fl = 2.0 * dense_ld ** 3
        us = stages[nm]["us"]
        stages[nm]["dense"] = True
        stages[nm]["dense_flops"] = fl
        stages[nm]["TFLOPs"] = round(fl / (us * 1e-6) / 1e12, 2) if us > 0 else None

    res = {
        "metric": "series evals/s + SpGEMM HBM GB/s vs plain filtered PS; p50/p99 latency at QPS",
        "value": evals_per_s,
        "unit": "evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "wall_ms_per_step": 1e3 * el / args.steps,
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
                   "series": "cos" if "_cos_" in cfg["name"] else "exp", "nnz_F": st["nnz_out"]},
        "roofline": {"bound": "hbm", "achieved": k_achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": k_achieved / HBM_PEAK_GBS,
                     "traffic": traffic,
                     "traffic_unit": "HBM bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
                     "traffic_frac": (traffic / ((k_ms / k_launches) * 1e-3) / 1e9 / HBM_PEAK_GBS
                                      if traffic and k_launches and k_ms > 0 else None),
                     "algorithmic_bytes_per_launch": k_bytes / k_launches if k_launches else None,
                     "kernel": dom_k,
                     "launches_per_step": k_launches,
                     "avg_launch_ms": k_ms / k_launches if k_launches else None,
                     "algorithmic_bytes_per_step": k_bytes,
                     "numeric_bytes_per_step": bytes_kernel,
                     "numeric_GBps": achieved,
                     "numeric_frac": achieved / HBM_PEAK_GBS,
                     "evaluation_bytes_per_step": bytes_eval,
                     "evaluation_GBps": bytes_eval / (ms_per_step * 1e-3) / 1e9,
                     "dominant_launch": dom,
                     "dominant_launch_frac": stages[dom]["frac"] if dom else None},
        "kernels": kernels,
        "stages": stages,
        **({"dense": {"ld": dense_ld, "stages": dense_stages,
                      "flops_per_step": 2.0 * dense_ld ** 3 * len(dense_stages),
                      "stage_us": sum(stages[nm]["us"] for nm in dense_stages),
                      "TFLOPs": (2.0 * dense_ld ** 3 * len(dense_stages)
                                 / (sum(stages[nm]["us"] for nm in dense_stages) * 1e-6) / 1e12)
                      if dense_stages else None,
                      "peak_TFLOPs": 78.6,
                      "note": "stage time includes densifying the operands and the write-out"}}
           if args.dense else {}),
        "products_per_s": prod_per_s,
        "products_per_step": products,
        "products_skipped_per_step": st["products_skipped"],
        "plan_setup_ms": setup_ms,
        "rows_wide_per_step": st["rows_wide"],
        "rows_global_per_step": st["rows_global"],
    }
    if dense_stages:
        # the dominant kernel is the matrix-core product: its roofline is the
        # FP64 matrix peak (stage time, densifying and write-out included)
        d = res["dense"]
        res["roofline_sparse"] = res["roofline"]
        res["roofline"] = {"bound": "mfma", "achieved": d["TFLOPs"], "peak": 78.6, "unit": "TFLOP/s",
                           "frac": d["TFLOPs"] / 78.6, "traffic": None, "kernel": "k_dgemm_mfma",
                           "flops_per_launch": 2.0 * dense_ld ** 3, "launches_per_step": len(dense_stages),
                           "avg_stage_ms": d["stage_us"] / len(dense_stages) / 1e3,
                           "note": "per dense stage: densify, block sum, product, write-out"}
    if args.filter != "fixed":
        res["alg1_iters_per_step"] = int(sum(st["stage_alg1_iters"]))
    plan.close()
    if args.batch_count > 0 and args.filter == "fixed" and args.workload == "lap2d":
        log(f"batch leg: {args.batch_count} banded instances ...")
        res["batch"] = bench_batch(args, stream)
        log(f"batch: {res['batch']['batch_ms']:.2f} ms vs plain {res['batch']['plain_ms']:.2f} ms "
            f"({res['batch']['speedup_vs_plain']:.2f}x)")
    if args.serve_requests > 0 and args.filter == "fixed" and args.workload == "lap2d":
        log(f"serving leg: {args.serve_requests} requests per run ...")
        res["serve"] = bench_serve(args, stream)
        log(f"serve: plain {res['serve']['plain_sequential_evals_per_s']:.0f}/s, server saturation "
            f"{res['serve']['server_saturation_evals_per_s']:.0f}/s ({res['serve']['speedup_vs_plain']:.2f}x)")
    if args.cpu_budget > 0 and args.filter == "fixed" and args.workload != "lap3d":
        log("timing the CPU oracle ...")
        res["cpu_baseline"] = cpu_baseline(cfg)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
