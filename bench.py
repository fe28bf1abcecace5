"""Benchmark of the lattice MVM inside CG on one MI355X.

One step = the whole hot path on one batch of synthetic input: build the
lattice of X (elevation, simplex, hash insert, numbering, neighbours), then
20 iterations of batched CG on 16 right-hand-side columns (1 target + 15
Rademacher probes), each iteration one fused multi-column splat/blur/slice
plus the CG vector updates. Inputs are resident in HBM before timing.

value = n * C * (MVMs per step) / step time   [points*channels/s]

Printed as one JSON line, with a roofline entry for the dominant kernel
(algorithmic bytes per launch over its HIP-event-measured mean duration) and
the CPU oracle timed on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E


def kernel_bytes(kind: str, n: int, d: int, m: int, C: int, r: int, sym: bool, cg: bool) -> float:
    """Algorithmic HBM bytes of ONE launch of a kernel kind: int32 indices,
    fp32 weights, every array touched once per launch. Inside CG (cg=True)
    the values and lattice accumulators are fp64, in lattice_mvm fp32."""
    D, T = d + 1, 2 * r
    chains = 2 if sym else 1
    vb = ub = 8 if cg else 4
    if kind == "splat":      # idx + w, V in, U out
        return n * D * 8 + n * C * vb + m * C * ub
    if kind == "slice":      # idx + w, U (both chains) in, out (+ p in CG)
        return n * D * 8 + chains * m * C * ub + n * C * vb + (n * C * vb if cg else 0)
    if kind == "blur":       # average per launch: per chain U in, U out, neighbour lists
        return blur_bytes_per_mvm(d, m, C, r, sym, cg) / blur_launches(d, r)
    if kind == "cg_update":  # q, r in; r out (fp64)
        return 3 * n * C * 8
    if kind == "cg_dir":     # p, r in (fp64), x in (fp32); p out (fp64), x out (fp32)
        return 3 * n * C * 8 + 2 * n * C * 4
    if kind == "cg_init":    # b in (fp32); r, p out (fp64), x out (fp32)
        return n * C * 4 + 2 * n * C * 8 + n * C * 4
    if kind == "cg_out":     # x in, x out (fp32)
        return n * C * 8
    if kind == "fill":
        return m * C * ub
    return 0.0


def blur_launches(d, r):
    """Launches per blur: with a three-tap stencil two direction steps share
    a launch (the intermediate lattice values stay in registers)."""
    return (d + 2) // 2 if r == 1 else d + 1


def blur_bytes_per_mvm(d, m, C, r, sym, cg):
    ub = 8 if cg else 4
    T = 2 * r
    chains = 2 if sym else 1
    if r == 1:
        pairs, single = (d + 1) // 2, (d + 1) % 2
        return (pairs * chains * (2 * m * C * ub + 2 * T * m * 4)
                + single * chains * (2 * m * C * ub + T * m * 4))
    return (d + 1) * chains * (2 * m * C * ub + T * m * 4)


def mvm_bytes(n, d, m, C, r, sym, cg=False):
    return (kernel_bytes("splat", n, d, m, C, r, sym, cg) + blur_bytes_per_mvm(d, m, C, r, sym, cg)
            + kernel_bytes("slice", n, d, m, C, r, sym, cg))


# Kernel sources whose code the stored HBM traffic was measured on; the
# traffic is reported only while they are unchanged.
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "ws3_traffic.json")
TRAFFIC_SOURCES = ["paper_2106_06695_amd/csrc/lattice_mvm.hip", "paper_2106_06695_amd/csrc/sgp_internal.h",
                   "paper_2106_06695_amd/csrc/cg.hip", "paper_2106_06695_amd/csrc/cg_step.h"]


def sources_digest() -> dict:
    import hashlib
    return {f: hashlib.sha256(open(os.path.join(ROOT, f), "rb").read()).hexdigest() for f in TRAFFIC_SOURCES}


def stored_traffic(stage: str):
    """HBM bytes per launch of a stage from the committed FETCH_SIZE /
    WRITE_SIZE measurement (copy-calibrated), or None if the kernel sources
    changed since."""
    try:
        t = json.load(open(TRAFFIC_FILE))
    except (OSError, ValueError):
        return None
    if t.get("source_sha256") != sources_digest():
        return None
    k = t.get("stages", {}).get(stage)
    return None if k is None else k["fetch_bytes"] + k["write_bytes"]


def probe():
    """A few CG iterations of the ws3 step (every MVM and CG kernel), then a
    plain 512 MiB device copy whose FETCH_SIZE / WRITE_SIZE calibrate the
    counters."""
    import torch
    import paper_2106_06695_amd as sgp
    import workloads
    torch.cuda.set_device(0)
    w = workloads.ws3()
    X = torch.from_numpy(w.X).cuda()
    V = torch.from_numpy(w.values).cuda()
    lat = sgp.lattice_build(X, w.lengthscales)
    x = torch.empty_like(V)
    sgp.cg_solve(lat, V, w.noise, 0.0, max_iter=3, x=x)
    a = torch.ones(64 * 1024 * 1024, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    lat.free()
    print(json.dumps({"probe": "ws3 build + 3 CG iterations, then a 512 MiB device copy", "m": lat.m}),
          flush=True)
    return 0


def cpu_baseline(w, n_sample: int, iters: int):
    """The oracle as it stands: build + per-column CG on the first n_sample
    points, single-threaded."""
    import oracle
    Xs, Vs = w.X[:n_sample], w.values[:n_sample].astype(np.float64)
    t0 = time.perf_counter()
    olat = oracle.Lattice(Xs, w.lengthscales)
    olat.cg(Vs, w.noise, 0.0, max_iter=iters)
    dt = time.perf_counter() - t0
    C = w.values.shape[1]
    return {"value": n_sample * C * iters / dt, "unit": "points*ch/s", "cores": 1, "kind": "oracle",
            "sample": f"first {n_sample} of {w.n} points, all {C} columns: oracle build + {iters} "
                      f"CG iterations per column (fp64, single thread), {dt:.2f} s"}


def _host_cpu():
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return model, len(os.sched_getaffinity(0))


def cpu_baseline_all_cores(w, n_sample: int, iters: int):
    """The same oracle work spread over the host: one single-threaded oracle
    process per column (python -m oracle cg: build + iters CG iterations on
    that column), as many at once as there are cores (at most 16)."""
    import subprocess
    import tempfile

    model, ncpu = _host_cpu()
    C = w.values.shape[1]
    procs = max(1, min(C, ncpu, 16))
    with tempfile.TemporaryDirectory() as td:
        np.save(os.path.join(td, "X.npy"), w.X[:n_sample])
        np.save(os.path.join(td, "ell.npy"), np.asarray(w.lengthscales, dtype=np.float64))
        for c in range(C):
            np.save(os.path.join(td, f"v{c}.npy"), w.values[:n_sample, c:c + 1].astype(np.float64))

        def launch(c):
            return subprocess.Popen(
                [sys.executable, "-m", "oracle", "cg", "--X", os.path.join(td, "X.npy"),
                 "--ell", os.path.join(td, "ell.npy"), "--values", os.path.join(td, f"v{c}.npy"),
                 "--noise", repr(float(w.noise)), "--tol", "0", "--max-iter", str(iters),
                 "--out", os.path.join(td, f"x{c}.npy")],
                cwd=ROOT, stdout=subprocess.DEVNULL, stderr=subprocess.PIPE)

        t0 = time.perf_counter()
        pending, running = list(range(C)), []
        while pending or running:
            while pending and len(running) < procs:
                running.append(launch(pending.pop(0)))
            done = running.pop(0)
            _, err = done.communicate()
            if done.returncode != 0:
                raise RuntimeError(f"oracle process failed: {err.decode()[-400:]}")
        dt = time.perf_counter() - t0
    return {"value": n_sample * C * iters / dt, "unit": "points*ch/s", "cores": procs,
            "kind": "oracle, one single-threaded process per column",
            "host": f"{model}, {ncpu} cores available",
            "sample": f"first {n_sample} of {w.n} points, {C} columns: per column an oracle build + "
                      f"{iters} CG iterations (fp64), {dt:.2f} s wall"}


def serving_bench(workers: int, count: int, rhos=(0.5, 0.9, 1.5), seed: int = 1005):
    """Served solves (predictive means) at Poisson arrival rates rho / T, with
    T the mean one-at-a-time service time measured first: p50/p99 latency
    (completion - arrival) and throughput of the continuous-batching server
    against the same stream served one request at a time."""
    import workloads
    from paper_2106_06695_amd import serve

    warm = workloads.ws5_requests(seed=seed + 1, count=8, mean_gap_s=0.0)
    serve.Server(workers=workers).run(warm, realtime=False)
    reqs = workloads.ws5_requests(seed=seed, count=count, mean_gap_s=0.0)
    solo = serve.Server(workers=1).run(reqs, realtime=False)
    service = np.array([r.done_s - r.admitted_s for r in solo])
    T = float(service.mean())
    print(f"serving: one-at-a-time service {T * 1e3:.2f} ms mean over {count} requests",
          file=sys.stderr, flush=True)
    iters = np.array([r.iters.max() for r in solo])
    out = {"requests": count, "workers": workers, "mean_service_ms": T * 1e3,
           "median_cg_iterations": float(np.median(iters)),
           "nonconverged": int(sum(int(np.any(r.rel > q.tol)) for r, q in zip(solo, reqs))),
           "rates": []}
    for rho in rhos:
        reqs = workloads.ws5_requests(seed=seed, count=count, mean_gap_s=T / rho)
        entry = {"rho": rho, "lambda_per_s": rho / T}
        for name, wk in (("batched", workers), ("one_at_a_time", 1)):
            srv = serve.Server(workers=wk)
            res = srv.run(reqs, realtime=True)
            summ = serve.latency_summary(res)
            summ["max_reserved_GB"] = srv.max_reserved / 1e9
            entry[name] = summ
            print(f"serving rho={rho} {name}: {summ}", file=sys.stderr, flush=True)
        out["rates"].append(entry)
    return out


def paper_sparsity_bench(sgp, X, V, w, x, args):
    """The same step on ws3's points with lengthscales scaled to the paper's
    lattice sparsity (ws3p, m / (n (d+1)) ~ 0.04): one warm-up step, then
    args.paper_steps timed ones, and standalone fp32 MVMs."""
    import torch
    import workloads
    scale = workloads.ws3p_scale()
    ell = w.lengthscales * scale
    iters = w.max_iter

    def step():
        lat = sgp.lattice_build(X, ell, blur=args.blur)
        sgp.cg_solve(lat, V, w.noise, 0.0, max_iter=iters, x=x)
        m = lat.m
        lat.free()
        return m

    m = step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.paper_steps):
        step()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / args.paper_steps
    lat = sgp.lattice_build(X, ell, blur=args.blur)
    out = torch.empty_like(V)
    sgp.lattice_mvm(lat, V, out)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    reps = 5
    for _ in range(reps):
        sgp.lattice_mvm(lat, V, out)
    torch.cuda.synchronize()
    mvm_s = (time.perf_counter() - t0) / reps
    lat.free()
    n, d, C = w.n, w.d, w.C
    B = mvm_bytes(n, d, m, C, 1, args.blur == "symmetric")
    return {"workload": "ws3p: ws3 with lengthscales x %.4f (the paper's Houseelectric sparsity)" % scale,
            "m": m, "m_over_L": m / (n * (d + 1)), "steps": args.paper_steps, "ms_per_step": ms,
            "value": n * C * iters / (ms / 1e3), "unit": "points*ch/s",
            "mvm_only": {"ms": mvm_s * 1e3, "points_ch_per_s": n * C / mvm_s, "algo_bytes": B,
                         "algo_GBps": B / mvm_s / 1e9, "frac_of_hbm_peak": B / mvm_s / 1e9 / HBM_PEAK_GBS}}


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--blur", default="symmetric", choices=["symmetric", "forward"])
    ap.add_argument("--cpu-sample", type=int, default=200_000,
                    help="points in the oracle's CPU-baseline sample (0 = skip)")
    ap.add_argument("--mvm-reps", type=int, default=20, help="extra timed lattice_mvm calls")
    ap.add_argument("--serve", type=int, default=0,
                    help="also run the serving benchmark with this many requests (0 = skip)")
    ap.add_argument("--serve-workers", type=int, default=8)
    ap.add_argument("--autotune", type=int, default=1,
                    help="1: autotune the MVM launch shapes on the first lattice before timing")
    ap.add_argument("--paper-steps", type=int, default=3,
                    help="timed steps of the ws3p secondary measurement (0 = skip)")
    ap.add_argument("--probe", action="store_true",
                    help="only run the short counter-collection workload")
    args = ap.parse_args(argv)
    if args.gpus != 1:
        print("bench.py measures one GPU; --gpus must be 1", file=sys.stderr)
        return 2
    if args.probe:
        return probe()

    import torch
    import paper_2106_06695_amd as sgp
    import workloads

    torch.cuda.set_device(0)
    w = workloads.ws3()
    n, d, C = w.n, w.d, w.C
    X = torch.from_numpy(w.X).cuda()
    V = torch.from_numpy(w.values).cuda()
    x = torch.empty_like(V)
    iters = w.max_iter
    sym = args.blur == "symmetric"

    def step():
        lat = sgp.lattice_build(X, w.lengthscales, blur=args.blur)
        sgp.cg_solve(lat, V, w.noise, 0.0, max_iter=iters, x=x)
        m = lat.m
        lat.free()
        return m

    # launch shapes for this lattice class, chosen once before any timing
    tuned = None
    if args.autotune:
        lat = sgp.lattice_build(X, w.lengthscales, blur=args.blur)
        tuned = sgp.autotune(lat, C, fp64=True, reps=3)
        lat.free()
    for _ in range(args.warmup):
        m = step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        m = step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_per_step = (t1 - t0) * 1e3 / args.steps
    value = n * C * iters / (ms_per_step / 1e3)

    # per-kernel event timings, from separate steps (the events would
    # otherwise add to the timed ones)
    prof_steps = 2
    with sgp.profile() as prof:
        for _ in range(prof_steps):
            step()
        torch.cuda.synchronize()
    kernels = {}
    for kind, (launches, ms) in prof.results.items():
        if launches:
            b = kernel_bytes(kind, n, d, m, C, 1, sym, cg=True)
            avg = ms / launches
            kernels[kind] = {"launches": launches, "total_ms": round(ms, 3), "avg_us": round(avg * 1e3, 2),
                             "algo_GBps": round(b / (avg / 1e3) / 1e9, 1) if b else None}
    # the splat runs as two passes (per-tile reduction, then per-lattice-point
    # gather of the tile partials, whose small fix-up kernel for lattice
    # points spanning several gather ranges is timed with it); its
    # algorithmic bytes cover all three kernels
    stage_ms = {k: kernels[k]["total_ms"] for k in ("blur", "slice") if k in kernels}
    stage_ms["splat"] = kernels["splat"]["total_ms"] + kernels.get("splat_gather", {"total_ms": 0.0})["total_ms"]
    dom = max(stage_ms, key=stage_ms.get)
    dom_bytes = kernel_bytes(dom, n, d, m, C, 1, sym, cg=True)
    dom_avg_s = stage_ms[dom] / kernels[dom]["launches"] / 1e3
    achieved = dom_bytes / dom_avg_s / 1e9

    # standalone MVMs on a resident lattice (outside the timed steps)
    lat = sgp.lattice_build(X, w.lengthscales, blur=args.blur)
    out = torch.empty_like(V)
    for _ in range(3):
        sgp.lattice_mvm(lat, V, out)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.mvm_reps):
        sgp.lattice_mvm(lat, V, out)
    torch.cuda.synchronize()
    mvm_s = (time.perf_counter() - t0) / args.mvm_reps
    B = mvm_bytes(n, d, lat.m, C, 1, sym)

    # the same 20 iterations as C separate single-column solves
    sep_x = torch.empty((n, 1), dtype=torch.float32, device=V.device)
    cols = [V[:, c:c + 1].contiguous() for c in range(C)]
    sgp.cg_solve(lat, cols[0], w.noise, 0.0, max_iter=iters, x=sep_x)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sgp.cg_solve(lat, V, w.noise, 0.0, max_iter=iters, x=x)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for c in range(C):
        sgp.cg_solve(lat, cols[c], w.noise, 0.0, max_iter=iters, x=sep_x)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    lat.free()

    paper = paper_sparsity_bench(sgp, X, V, w, x, args) if args.paper_steps > 0 else None

    line = {
        "metric": "lattice MVM points*ch/s at n=2M d=11 (build + 20 batched CG iterations per step)",
        "value": value,
        "unit": "points*ch/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64 CG vectors and lattice accumulation, f32 weights",
        "data": "synthetic",
        "config": {"workload": "ws3: n=2,000,000 d=11 X from a 50-component Gaussian mixture "
                               "(standardised), lengthscales logU[0.5,2], C=16 (1 target + 15 "
                               "Rademacher probes), noise 0.05, RBF r=1, " + args.blur + " blur, 20 CG iterations",
                   "n": n, "d": d, "C": C, "m": m, "m_over_L": m / (n * (d + 1)),
                   "cg_iterations": iters, "blur": args.blur},
        "roofline": {"bound": "hbm", "kernel": dom + (" (splat_tile + splat_gather + gather_fix)" if dom == "splat" else ""),
                     "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": stored_traffic(dom),
                     "algo_bytes_per_launch": dom_bytes},
        "mvm_only": {"ms": mvm_s * 1e3, "points_ch_per_s": n * C / mvm_s,
                     "algo_bytes": B, "algo_GBps": B / mvm_s / 1e9,
                     "frac_of_hbm_peak": B / mvm_s / 1e9 / HBM_PEAK_GBS},
        "batched_vs_separate": {"cg_iterations": iters, "batched_C16_ms": (t1 - t0) * 1e3,
                                "separate_16x_C1_ms": (t2 - t1) * 1e3,
                                "speedup": (t2 - t1) / (t1 - t0)},
        "kernels": kernels,
        "profiled_steps": prof_steps,
        "autotune": tuned,
    }
    if paper is not None:
        line["paper_sparsity"] = paper
    if args.serve > 0:
        line["serving"] = serving_bench(args.serve_workers, args.serve)
    if args.cpu_sample > 0:
        line["cpu_baseline"] = cpu_baseline(w, min(args.cpu_sample, n), iters)
        line["cpu_baseline_all_cores"] = cpu_baseline_all_cores(w, min(args.cpu_sample, n), iters)
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
