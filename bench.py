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


def kernel_bytes(kind: str, n: int, d: int, m: int, C: int, r: int, sym: bool, cg: bool,
                 dir_frac: float = 0.0) -> float:
    """Algorithmic HBM bytes of ONE launch of a kernel kind: int32 indices,
    fp32 weights, every array touched once per launch. Inside CG (cg=True)
    the values and lattice accumulators are fp64, in lattice_mvm fp32.
    dir_frac: the share of the splat launches that also apply the CG
    direction update (r and x in, p and x out: 24 bytes per element)."""
    D, T = d + 1, 2 * r
    chains = 2 if sym else 1
    vb = ub = 8 if cg else 4
    if kind == "splat":      # idx + w, V in, U out (+ the fused direction update)
        return n * D * 8 + n * C * vb + m * C * ub + dir_frac * 24 * n * C
    if kind == "slice":      # idx + w, U (both chains) in, out (+ p and r in inside CG, out being r)
        return n * D * 8 + chains * m * C * ub + n * C * vb + (2 * n * C * vb if cg else 0)
    if kind == "blur":       # average per launch: per chain U in, U out, neighbour lists
        return blur_bytes_per_mvm(d, m, C, r, sym, cg) / blur_launches(d, r)
    if kind == "cg_alpha":   # u and B u in (fp64)
        return 2 * m * C * 8
    if kind == "cg_dir":     # p, r in (fp64), x in (fp32); p out (fp64), x out (fp32)
        return 3 * n * C * 8 + 2 * n * C * 4
    if kind == "cg_init":    # b in (fp32); r, p out (fp64), x out (fp32)
        return n * C * 4 + 2 * n * C * 8 + n * C * 4
    if kind == "cg_out":     # x in, p in (the last x update), x out
        return n * C * 16
    if kind == "fill":
        return m * C * ub
    return 0.0


def survey_bytes(kind: str, n: int, d: int, m: int, C: int, r: int, sym: bool,
                 dir_frac: float = 0.0) -> float:
    """Algorithmic HBM bytes of ONE launch under the survey's byte model:
    fp32 values, int32 indices and fp32 weights whatever precision a kernel
    computes in, neighbour lists counted once per sweep. The splat stage is
    k_splat_tile + k_splat_gather + k_gather_fix; inside CG the slice also
    reads the direction p and moves the residual r (in and out), and every
    vector pass counts n*C*4 bytes (the splat's fused direction update: r and
    x in, p and x out)."""
    D = d + 1
    chains = 2 if sym else 1
    if kind == "splat_stage":
        return n * D * 8 + n * C * 4 + m * C * 4 + dir_frac * 16 * n * C
    if kind == "splat":      # k_splat_tile alone: W and V in (U is the gather's)
        return n * D * 8 + n * C * 4 + dir_frac * 16 * n * C
    if kind == "blur":
        return blur_bytes_per_mvm(d, m, C, r, sym, False) / blur_launches(d, r)
    if kind == "slice":      # CG variant: idx + w, U, p and r in, r out
        return n * D * 8 + chains * m * C * 4 + 3 * n * C * 4
    if kind == "cg_alpha":   # u and B u in
        return 2 * m * C * 4
    if kind == "cg_dir":     # p, r, x in; p, x out
        return 5 * n * C * 4
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


TRAFFIC_KERNELS = {"splat": ["k_splat_tile"], "splat_stage": ["k_splat_tile", "k_splat_gather", "k_gather_fix"],
                   "blur": ["k_blur"], "slice": ["k_slice_tile"], "cg_alpha": ["k_cg_alpha"],
                   "cg_dir": ["k_cg_dir"]}


def stored_traffic(stage: str):
    """HBM bytes per launch of a kernel (or the splat stage) from the
    committed FETCH_SIZE / WRITE_SIZE measurement (copy-calibrated), or None
    if the kernel sources changed since."""
    try:
        t = json.load(open(TRAFFIC_FILE))
    except (OSError, ValueError):
        return None
    if t.get("source_sha256") != sources_digest():
        return None
    ks = t.get("kernels", {})
    names = TRAFFIC_KERNELS.get(stage, [])
    if not names or any(k not in ks for k in names):
        return None
    return sum(ks[k]["fetch_bytes"] + ks[k]["write_bytes"] for k in names)


def hbm_probe():
    """HBM rates a plain stream reaches on this GPU, as a reference for the
    kernels' measured traffic: a 2 GiB fp64 device copy (read + write) and a
    read-only sum of the same array, each the mean of 20 after 3 untimed."""
    import torch
    torch.cuda.set_device(0)
    n = 256 * 1024 * 1024
    a = torch.ones(n, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)

    def timed(fn, reps=20):
        for _ in range(3):
            fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / reps

    copy_s = timed(lambda: b.copy_(a))
    sum_s = timed(lambda: a.sum())
    nbytes = n * 8
    print(json.dumps({"hbm_probe": "2 GiB fp64: device copy (read + write) and read-only sum",
                      "copy_GBps": 2 * nbytes / copy_s / 1e9, "read_GBps": nbytes / sum_s / 1e9,
                      "copy_ms": copy_s * 1e3, "sum_ms": sum_s * 1e3}), flush=True)
    return 0


def probe():
    """A few CG iterations of the ws3 step (every MVM and CG kernel; the last
    one in its steady state), then a plain 512 MiB device copy whose
    FETCH_SIZE / WRITE_SIZE calibrate the counters."""
    import torch
    import paper_2106_06695_amd as sgp
    import workloads
    torch.cuda.set_device(0)
    w = workloads.ws3()
    X = torch.from_numpy(w.X).cuda()
    V = torch.from_numpy(w.values).cuda()
    lat = sgp.lattice_build(X, w.lengthscales)
    x = torch.empty_like(V)
    sgp.cg_solve(lat, V, w.noise, 0.0, max_iter=4, x=x)
    a = torch.ones(64 * 1024 * 1024, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    lat.free()
    print(json.dumps({"probe": "ws3 build + 4 CG iterations, then a 512 MiB device copy", "m": lat.m}),
          flush=True)
    return 0


def cpu_baseline(w, n_sample: int, iters: int):
    """The oracle as it stands: build + per-column CG on the first n_sample
    points, single-threaded and pinned to one core of the host."""
    import oracle
    model, _ = _host_cpu()
    before = os.sched_getaffinity(0)
    core = min(before)
    Xs, Vs = w.X[:n_sample], w.values[:n_sample].astype(np.float64)
    os.sched_setaffinity(0, {core})
    try:
        t0 = time.perf_counter()
        olat = oracle.Lattice(Xs, w.lengthscales)
        olat.cg(Vs, w.noise, 0.0, max_iter=iters)
        dt = time.perf_counter() - t0
    finally:
        os.sched_setaffinity(0, before)
    C = w.values.shape[1]
    return {"value": n_sample * C * iters / dt, "unit": "points*ch/s", "cores": 1, "kind": "oracle",
            "pinned_core": core, "host": model,
            "sample": f"first {n_sample} of {w.n} points, all {C} columns: oracle build + {iters} "
                      f"CG iterations per column (fp64, single thread pinned to core {core}), "
                      f"{dt:.2f} s"}


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


def _median_ms(fn, reps: int):
    import torch
    ts = []
    for _ in range(reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        fn()
        torch.cuda.synchronize()
        ts.append((time.perf_counter() - t0) * 1e3)
    return float(np.median(ts))


def configs_bench(sgp):
    """The other workloads of the benchmark set, each timed on its own
    (median of warm repetitions, host clock around synchronised calls):
      ws1  n=2,000 d=3 C=1: latency of build, one MVM and CG to 1e-4;
      ws2  n=500,000 d=8 C=1: 100 repeated fp32 MVMs and CG to 1e-2;
      ws4  n=1,000,000 d=16 C=8: forward fp32 MVM and the adjoint with
           respect to X and the log-lengthscales (Section 4.2)."""
    import torch
    import workloads
    out = {}

    # ws1: small-problem latency
    w = workloads.ws1()
    X = torch.from_numpy(w.X).cuda()
    V = torch.from_numpy(w.values).cuda()
    lat = sgp.lattice_build(X, w.lengthscales)
    y = torch.empty_like(V)
    sgp.lattice_mvm(lat, V, y)
    x, its, rel = sgp.cg_solve(lat, V, w.noise, w.tol, max_iter=w.max_iter)
    build_ms = _median_ms(lambda: sgp.lattice_build(X, w.lengthscales).free(), 20)
    mvm_ms = _median_ms(lambda: sgp.lattice_mvm(lat, V, y), 50)
    cg_ms = _median_ms(lambda: sgp.cg_solve(lat, V, w.noise, w.tol, max_iter=w.max_iter, x=x), 20)

    def whole():
        L = sgp.lattice_build(X, w.lengthscales)
        sgp.lattice_mvm(L, V, y)
        sgp.cg_solve(L, V, w.noise, w.tol, max_iter=w.max_iter, x=x)
        L.free()
    out["ws1"] = {"workload": "n=2,000 d=3 X~N(0,I) l=1 C=1, CG on K+0.1I to 1e-4", "m": lat.m,
                  "build_ms": build_ms, "mvm_ms": mvm_ms, "cg_ms": cg_ms, "cg_iterations": int(its[0]),
                  "cg_rel_residual": float(rel[0]), "build_mvm_cg_ms": _median_ms(whole, 20)}
    lat.free()

    # ws2: single-column throughput
    w = workloads.ws2()
    X = torch.from_numpy(w.X).cuda()
    V = torch.from_numpy(w.values).cuda()
    build_ms = _median_ms(lambda: sgp.lattice_build(X, w.lengthscales).free(), 5)
    lat = sgp.lattice_build(X, w.lengthscales)
    y = torch.empty_like(V)
    sgp.lattice_mvm(lat, V, y)
    reps = 100
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        sgp.lattice_mvm(lat, V, y)
    torch.cuda.synchronize()
    mvm_s = (time.perf_counter() - t0) / reps
    B = mvm_bytes(w.n, w.d, lat.m, 1, 1, True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    x, its, rel = sgp.cg_solve(lat, V, w.noise, w.tol, max_iter=w.max_iter)
    cg_s = time.perf_counter() - t0
    out["ws2"] = {"workload": "n=500,000 d=8 20-component mixture, l~logU[0.5,2], C=1; "
                              "100 repeated MVMs; CG on K+0.05I to 1e-2",
                  "m": lat.m, "build_ms": build_ms, "mvm_ms": mvm_s * 1e3,
                  "mvm_points_ch_per_s": w.n / mvm_s, "mvm_algo_bytes": B,
                  "mvm_algo_GBps": B / mvm_s / 1e9, "mvm_frac_of_hbm_peak": B / mvm_s / 1e9 / HBM_PEAK_GBS,
                  "cg_ms": cg_s * 1e3, "cg_iterations": int(its[0]), "cg_rel_residual": float(rel[0]),
                  "cg_ms_per_iteration": cg_s * 1e3 / max(1, int(its[0]))}
    lat.free()

    # ws4: forward MVM and adjoint
    w = workloads.ws4()
    X = torch.from_numpy(w.X).cuda()
    V = torch.from_numpy(w.values).cuda()
    G = torch.from_numpy(np.random.default_rng(4).standard_normal(w.values.shape).astype(np.float32)).cuda()
    build_ms = _median_ms(lambda: sgp.lattice_build(X, w.lengthscales).free(), 3)
    lat = sgp.lattice_build(X, w.lengthscales)
    y = torch.empty_like(V)
    sgp.lattice_mvm(lat, V, y)
    mvm_ms = _median_ms(lambda: sgp.lattice_mvm(lat, V, y), 10)
    sgp.lattice_mvm_grad(lat, X, V, G)
    adj_ms = _median_ms(lambda: sgp.lattice_mvm_grad(lat, X, V, G), 3)
    B = mvm_bytes(w.n, w.d, lat.m, w.C, 1, True)
    out["ws4"] = {"workload": "n=1,000,000 d=16 X~U[-1,1]^16, l~logU[0.3,3], C=8; forward MVM "
                              "and adjoint (dX, dlog l) of sum(G * K V)",
                  "m": lat.m, "build_ms": build_ms, "mvm_ms": mvm_ms,
                  "mvm_points_ch_per_s": w.n * w.C / (mvm_ms / 1e3), "mvm_algo_bytes": B,
                  "mvm_algo_GBps": B / (mvm_ms / 1e3) / 1e9,
                  "mvm_frac_of_hbm_peak": B / (mvm_ms / 1e3) / 1e9 / HBM_PEAK_GBS,
                  "adjoint_ms": adj_ms, "adjoint_points_ch_per_s": w.n * w.C / (adj_ms / 1e3)}
    lat.free()
    return out


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
    ap.add_argument("--serve", type=int, default=256,
                    help="requests of the serving benchmark (0 = skip)")
    ap.add_argument("--configs", type=int, default=1,
                    help="1: also time the n=2,000, n=500,000 and n=1,000,000 (d=16) workloads")
    ap.add_argument("--serve-workers", type=int, default=8)
    ap.add_argument("--autotune", type=int, default=1,
                    help="1: autotune the MVM launch shapes on the first lattice before timing")
    ap.add_argument("--paper-steps", type=int, default=3,
                    help="timed steps of the ws3p secondary measurement (0 = skip)")
    ap.add_argument("--probe", action="store_true",
                    help="only run the short counter-collection workload")
    ap.add_argument("--hbm-probe", action="store_true",
                    help="only measure a plain device copy and a read-only sum (HBM reference rates)")
    args = ap.parse_args(argv)
    if args.gpus != 1:
        print("bench.py measures one GPU; --gpus must be 1", file=sys.stderr)
        return 2
    if args.probe:
        return probe()
    if args.hbm_probe:
        return hbm_probe()

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

    # build table shape and MVM launch shapes for this lattice class, chosen
    # once before any timing
    tuned = None
    if args.autotune:
        tuned = {"build": sgp.autotune_build(X, w.lengthscales, reps=2, blur=args.blur)}
        lat = sgp.lattice_build(X, w.lengthscales, blur=args.blur)
        tuned["mvm"] = sgp.autotune(lat, C, fp64=True, reps=3)
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
    # every splat but a solve's first applies the previous direction update
    dir_frac = (iters - 1) / iters
    kernels = {}
    for kind, (launches, ms) in prof.results.items():
        if launches:
            b = kernel_bytes(kind, n, d, m, C, 1, sym, cg=True, dir_frac=dir_frac)
            avg = ms / launches
            kernels[kind] = {"launches": launches, "total_ms": round(ms, 3), "avg_us": round(avg * 1e3, 2),
                             "algo_GBps": round(b / (avg / 1e3) / 1e9, 1) if b else None}
    # Roofline of the kernel with the largest time per step, and of the
    # splat stage (k_splat_tile, then k_splat_gather + k_gather_fix, which
    # the "splat_gather" kind times together). "achieved" uses the survey's
    # byte model (fp32 values whatever precision the kernel computes in);
    # "achieved_operand_bytes" the kernel's own operand widths (fp64 values
    # and lattice rows inside CG).
    def roof(kind_label, kinds, survey_b, native_b, traffic_key):
        tot = sum(kernels[k]["total_ms"] for k in kinds if k in kernels)
        avg_s = tot / kernels[kinds[0]]["launches"] / 1e3
        a_s = survey_b / avg_s / 1e9
        a_n = native_b / avg_s / 1e9
        return {"bound": "hbm", "kernel": kind_label, "avg_us": avg_s * 1e6,
                "achieved": a_s, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": a_s / HBM_PEAK_GBS,
                "traffic": stored_traffic(traffic_key), "algo_bytes_per_launch": survey_b,
                "byte_model": "survey (fp32 values, int32 indices, fp32 weights)",
                "achieved_operand_bytes": a_n, "frac_operand_bytes": a_n / HBM_PEAK_GBS,
                "operand_bytes_per_launch": native_b}

    names = {"splat": "k_splat_tile<double, G, true> (with the fused CG direction update)",
             "blur": "k_blur2_split / k_blur2",
             "slice": "k_slice_tile<double, G, true> (with the fused CG residual update)",
             "cg_alpha": "k_cg_alpha", "cg_dir": "k_cg_dir"}
    single = {k: kernels[k]["total_ms"] for k in names if k in kernels}
    dom = max(single, key=single.get)
    splat_native = kernel_bytes("splat", n, d, m, C, 1, sym, cg=True, dir_frac=dir_frac)
    dom_survey = survey_bytes(dom, n, d, m, C, 1, sym, dir_frac=dir_frac)
    dom_native = kernel_bytes(dom, n, d, m, C, 1, sym, cg=True, dir_frac=dir_frac)
    if dom == "splat":  # the tile kernel alone reads W and V; U is written by the gather
        dom_native -= m * C * 8
    roofline = roof(names[dom], [dom], dom_survey, dom_native, dom)
    splat_stage = roof("k_splat_tile + k_splat_gather + k_gather_fix", ["splat", "splat_gather"],
                       survey_bytes("splat_stage", n, d, m, C, 1, sym, dir_frac=dir_frac), splat_native,
                       "splat_stage")

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
        "roofline": roofline,
        "splat_stage": splat_stage,
        "mvm_only": {"ms": mvm_s * 1e3, "points_ch_per_s": n * C / mvm_s,
                     "algo_bytes": B, "algo_GBps": B / mvm_s / 1e9,
                     "frac_of_hbm_peak": B / mvm_s / 1e9 / HBM_PEAK_GBS,
                     "byte_model": "survey B_mvm (fp32 lattice_mvm, C=16)"},
        "batched_vs_separate": {"cg_iterations": iters, "batched_C16_ms": (t1 - t0) * 1e3,
                                "separate_16x_C1_ms": (t2 - t1) * 1e3,
                                "speedup": (t2 - t1) / (t1 - t0)},
        "kernels": kernels,
        "profiled_steps": prof_steps,
        "autotune": tuned,
    }
    if paper is not None:
        line["paper_sparsity"] = paper
    if args.configs:
        line["configs"] = configs_bench(sgp)
    if args.serve > 0:
        line["serving"] = serving_bench(args.serve_workers, args.serve)
    if args.cpu_sample > 0:
        line["cpu_baseline"] = cpu_baseline(w, min(args.cpu_sample, n), iters)
        line["cpu_baseline_all_cores"] = cpu_baseline_all_cores(w, min(args.cpu_sample, n), iters)
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
