"""Continuous-batching GP solve server on one GPU.

Each request carries training inputs X (n x d), test inputs X* (n* x d),
lengthscales, and right-hand sides `values` (n x C: the target, then probe
vectors).
Serving one request means:
  1. build one lattice on [X; X*], with CG restricted to the first n points;
  2. solve (outputscale*K + noise*I) A = values to the request's tolerance
     (Section 2, Krylov methods);
  3. compute the predictive mean at X* as one MVM of [a; 0] (Section 2,
     eq. gp_pred_mean, zero prior mean).

Scheduling: requests queue in arrival order. Workers each own a HIP stream,
so the requests in flight overlap on the device. The head of the queue is
admitted when a worker is free and its worst-case device footprint fits
the remaining HBM budget. That worst case assumes every vertex of every
simplex is distinct (m = N(d+1) for N = n + n* points). A request whose worst
case exceeds the whole budget runs alone. After the build, the reservation shrinks to
the lattice's actual footprint plus its solver buffers, so later requests can
start while earlier ones are still solving. Admission never lets the sum of
reservations exceed the budget.

All device work runs in the library's kernels; the host only copies inputs
in and results out.
"""
from __future__ import annotations

import collections
import dataclasses
import threading
import time
from typing import List, Optional

import numpy as np

from . import cg_solve, lattice_build, lattice_info, lattice_mvm


@dataclasses.dataclass
class SolveRequest:
    rid: int
    arrival_s: float
    X: np.ndarray          # (n, d) fp32
    X_test: np.ndarray     # (n*, d) fp32
    lengthscales: np.ndarray
    values: np.ndarray     # (n, C) fp32, column 0 the target
    noise: float
    tol: float = 1e-4
    max_iter: int = 1000
    outputscale: float = 1.0


@dataclasses.dataclass
class SolveResult:
    rid: int
    mean: np.ndarray       # (n*,) predictive mean from column 0
    alpha: np.ndarray      # (n,) solution column 0
    iters: np.ndarray
    rel: np.ndarray
    arrival_s: float
    admitted_s: float
    done_s: float
    reserved_bytes: int
    actual_bytes: int

    @property
    def latency_s(self) -> float:
        return self.done_s - self.arrival_s


def build_peak_bytes(N: int, d: int, order: int = 1) -> int:
    """Upper bound on the device bytes a lattice build of N points touches,
    transient hash tables (load factor 1/2) and sort buffers included, with
    every vertex distinct. Per splat entry (N(d+1) of them): 48 bytes of hash
    table, 12 of slots and unsorted entries, about 40 of sort and order
    buffers, 27 of the kept structure, 4 d of keys and 8 order (d+1) of
    neighbour table."""
    D = d + 1
    L = N * D
    return int((128 + 4 * d + 8 * order * D) * L + 8 * N * d + (64 << 20))


def solve_bytes(N: int, C: int, d: int, m: int) -> int:
    """Solver and MVM work buffers: fp64 lattice values (5 m rows plus at
    most N(d+1) tile-run rows), two fp64 CG vectors and an fp32 one, and
    the request's own fp32 inputs and outputs."""
    runs = N * (d + 1)
    return int(8 * C * (5 * m + runs) + 20 * N * C + 4 * N * (d + 2 * C + 2) + (16 << 20))


def footprint_worst(req) -> int:
    N = req.X.shape[0] + req.X_test.shape[0]
    d = req.X.shape[1]
    return build_peak_bytes(N, d) + solve_bytes(N, req.values.shape[1], d, N * (d + 1))


class Server:
    """Serve a stream of SolveRequests with `workers` concurrent slots within
    `hbm_budget` bytes of device memory."""

    def __init__(self, workers: int = 4, hbm_budget: Optional[int] = None, device: int = 0):
        import torch
        self.workers = workers
        self.device = device
        if hbm_budget is None:
            free, _total = torch.cuda.mem_get_info(device)
            hbm_budget = int(0.8 * free)
        self.budget = int(hbm_budget)
        self._cv = threading.Condition()
        self._queue: collections.deque = collections.deque()
        self._reserved = 0
        self.max_reserved = 0
        self._results: List[SolveResult] = []
        self._errors: List[BaseException] = []
        self._closed = False
        self._t0 = 0.0

    # -- admission -----------------------------------------------------------
    def _admit(self):
        """Block until the queue head fits; return (request, reservation)."""
        with self._cv:
            while True:
                if self._queue:
                    req = self._queue[0]
                    need = min(footprint_worst(req), self.budget)
                    if self._reserved + need <= self.budget:
                        self._queue.popleft()
                        self._reserved += need
                        self.max_reserved = max(self.max_reserved, self._reserved)
                        return req, need
                elif self._closed:
                    return None, 0
                self._cv.wait()

    def _adjust(self, old: int, new: int):
        with self._cv:
            self._reserved += new - old
            self.max_reserved = max(self.max_reserved, self._reserved)
            self._cv.notify_all()

    # -- one request -----------------------------------------------------------
    def _serve_one(self, req, slot: dict, stream):
        """Serve one request; slot["reserved"] always holds the bytes this
        request has reserved, so the worker releases exactly that amount
        whether the request finishes or fails."""
        import torch
        admitted = time.perf_counter() - self._t0
        n, d = req.X.shape
        n_test = req.X_test.shape[0]
        N = n + n_test
        C = req.values.shape[1]
        outputscale = float(getattr(req, "outputscale", 1.0))
        max_iter = int(getattr(req, "max_iter", 1000))
        dev = torch.device("cuda", self.device)
        with torch.cuda.stream(stream):
            X_all = torch.from_numpy(np.concatenate([req.X, req.X_test]).astype(np.float32)).to(dev)
            B = torch.zeros((N, C), dtype=torch.float32, device=dev)
            B[:n] = torch.from_numpy(np.ascontiguousarray(req.values, dtype=np.float32)).to(dev)
            lat = lattice_build(X_all, req.lengthscales, outputscale=outputscale, solve_rows=n)
            try:
                actual = int(lattice_info(lat)["device_bytes"]) + solve_bytes(N, C, d, lat.m)
                if actual < slot["reserved"]:
                    self._adjust(slot["reserved"], actual)
                    slot["reserved"] = actual
                A, iters, rel = cg_solve(lat, B, req.noise, req.tol, max_iter=max_iter)
                a = torch.zeros((N, 1), dtype=torch.float32, device=dev)
                a[:n] = A[:n, :1]
                mu = lattice_mvm(lat, a)[n:, 0].cpu().numpy()
                alpha = a[:n, 0].cpu().numpy()
            finally:
                lat.free()
        done = time.perf_counter() - self._t0
        return SolveResult(req.rid, mu, alpha, np.asarray(iters), np.asarray(rel), req.arrival_s,
                           admitted, done, slot["reserved"], actual)

    def _worker(self):
        import torch
        torch.cuda.set_device(self.device)
        stream = torch.cuda.Stream(device=self.device)  # default priority
        while True:
            req, reserved = self._admit()
            if req is None:
                return
            slot = {"reserved": reserved}
            try:
                res = self._serve_one(req, slot, stream)
                with self._cv:
                    self._results.append(res)
            except BaseException as e:  # surface in run()
                with self._cv:
                    self._errors.append(e)
            finally:
                self._adjust(slot["reserved"], 0)

    # -- driver ------------------------------------------------------------------
    def run(self, requests, realtime: bool = True) -> List[SolveResult]:
        """Submit requests at their arrival times (relative to now) and return
        the results in request order."""
        self._results, self._errors = [], []
        self._closed = False
        self._reserved = 0
        self.max_reserved = 0
        threads = [threading.Thread(target=self._worker, daemon=True) for _ in range(self.workers)]
        self._t0 = time.perf_counter()
        for t in threads:
            t.start()
        for req in sorted(requests, key=lambda r: r.arrival_s):
            if realtime:
                wait = req.arrival_s - (time.perf_counter() - self._t0)
                if wait > 0:
                    time.sleep(wait)
            with self._cv:
                self._queue.append(req)
                self._cv.notify_all()
        with self._cv:
            self._closed = True
            self._cv.notify_all()
        for t in threads:
            t.join()
        if self._errors:
            raise self._errors[0]
        return sorted(self._results, key=lambda r: r.rid)


def latency_summary(results: List[SolveResult]) -> dict:
    lat = np.array([r.latency_s for r in results]) * 1e3
    span = max(r.done_s for r in results) - min(r.arrival_s for r in results)
    return {"requests": len(results), "p50_ms": float(np.percentile(lat, 50)),
            "p99_ms": float(np.percentile(lat, 99)), "mean_ms": float(lat.mean()),
            "throughput_rps": len(results) / span if span > 0 else float("nan")}
