"""Serving loop: pseudospectrum requests (matrix, region, grid, epsilon
levels) arriving over time, run with continuous batching on one GPU.

A request is admitted as soon as it has arrived, a slot is free
(``max_active``) and its device-memory footprint fits what the running
requests leave of ``hbm_budget``; requests are admitted in arrival order (a
request that does not fit blocks the ones behind it, so none starves).  Each
admitted request gets its own library handle on its own HIP stream and runs
on a worker thread: the ctypes calls release the interpreter lock, so the
kernels of all running requests overlap on the device.  When a request
finishes, its handle (and with it every device buffer: operator, recycled
stores, preconditioner sites) is released and the next requests are
admitted.  Latency is completion time minus arrival time.

Argument marshalling and scheduling only: the numerical work is the C ABI's
``ps_create`` / ``ps_eval``.
"""
from __future__ import annotations

import dataclasses
import heapq
import threading
import time
from typing import Callable, List, Optional

import numpy as np


@dataclasses.dataclass
class Request:
    rid: int
    workload: object                 # workloads.Workload
    arrival: float = 0.0             # seconds after the start of the run
    params: dict = dataclasses.field(default_factory=dict)


@dataclasses.dataclass
class Result:
    rid: int
    sigma: np.ndarray
    member: np.ndarray
    flags: np.ndarray
    stats: dict
    arrival: float
    start: float
    done: float
    footprint: int

    @property
    def latency(self) -> float:
        return self.done - self.arrival


# per-request memory caps handed to the library (they bound the footprint)
SERVE_TILE_MEM_GB = 2
SERVE_SITE_MEM_GB = 2


def footprint_bytes(wl, tile_mem_gb: int = SERVE_TILE_MEM_GB, site_mem_gb: int = SERVE_SITE_MEM_GB,
                    k_max: int = 32, r: int = 8) -> int:
    """Upper estimate of a handle's device memory: the operator (C and C^*,
    dense or CSR, plus C^* C for the dense preconditioner), the per-tile
    state within tile_mem_gb (at least one tile), the preconditioner sites
    within site_mem_gb, and the work arrays of the dense apply."""
    m, n = wl.m, wl.n
    if wl.kind == "dense":
        op = 16 * (2 * m * n + n * n)
        ws = 16 * max(m, n) * 64 * 4
    else:
        nnz = len(wl.vals)
        op = 2 * (20 * nnz + 8 * (m + 1)) + 40 * (nnz + n)
        ws = 0
    per_tile = 16 * (8 * max(m, n) * k_max + 20 * max(m, n) * r)
    tiles = max(per_tile, min(tile_mem_gb * 10 ** 9, per_tile * max(1, wl.nx * wl.ny // 80)))
    if wl.kind != "dense":
        ws += 16 * n * k_max * 9 * 4       # projection stores of the sparse sites (within site_mem_gb)
    return int(op + tiles + site_mem_gb * (1 << 30) + ws + (512 << 20))


class LibraryBackend:
    """Runs a request through the C ABI on its own HIP stream."""

    def __init__(self):
        import torch
        import paper_2606_26785_amd as P
        self.P = P
        self.torch = torch

    def run(self, req: Request):
        P, torch = self.P, self.torch
        wl = req.workload
        stream = torch.cuda.Stream()
        kw = dict(tile_mem_gb=SERVE_TILE_MEM_GB, site_mem_gb=SERVE_SITE_MEM_GB)
        kw.update(req.params)
        mat = P.create_from_workload(wl, params=P.default_params(**kw), stream=stream.cuda_stream)
        try:
            g = P.ps_grid(*wl.region, wl.nx, wl.ny)
            res = P.ps_eval(mat, g, wl.eps)
            g.close()
        finally:
            mat.close()
        return res.sigma, res.member, res.flags, res.stats


class Server:
    def __init__(self, backend, hbm_budget: int, max_active: int = 8,
                 footprint: Callable = footprint_bytes, clock: Callable = time.perf_counter):
        self.backend = backend
        self.hbm_budget = int(hbm_budget)
        self.max_active = int(max_active)
        self.footprint = footprint
        self.clock = clock
        self.peak_bytes = 0
        self.peak_active = 0

    def run(self, requests: List[Request], time_limit: Optional[float] = None) -> List[Result]:
        """Serve the requests (their arrival times are relative to the start)
        and return one Result per request, in request order."""
        reqs = sorted(requests, key=lambda q: (q.arrival, q.rid))
        for q in reqs:
            if self.footprint(q.workload) > self.hbm_budget:
                raise ValueError("request %d alone exceeds the memory budget" % q.rid)
        lock = threading.Condition()
        results = {}
        errors = []
        state = {"used": 0, "active": 0}
        t0 = self.clock()

        def worker(q: Request, fp: int, t_start: float):
            try:
                sig, mem, fl, st = self.backend.run(q)
                t_done = self.clock() - t0
                results[q.rid] = Result(q.rid, sig, mem, fl, st, q.arrival, t_start, t_done, fp)
            except Exception as e:      # reported after the run
                errors.append((q.rid, e))
            finally:
                with lock:
                    state["used"] -= fp
                    state["active"] -= 1
                    lock.notify_all()

        threads = []
        i = 0
        with lock:
            while i < len(reqs) or state["active"] > 0:
                now = self.clock() - t0
                if time_limit is not None and now > time_limit:
                    raise TimeoutError("serving run exceeded %.0f s" % time_limit)
                admitted = False
                while i < len(reqs) and reqs[i].arrival <= now and state["active"] < self.max_active:
                    fp = self.footprint(reqs[i].workload)
                    if state["used"] + fp > self.hbm_budget:
                        break
                    q = reqs[i]
                    i += 1
                    state["used"] += fp
                    state["active"] += 1
                    self.peak_bytes = max(self.peak_bytes, state["used"])
                    self.peak_active = max(self.peak_active, state["active"])
                    th = threading.Thread(target=worker, args=(q, fp, now), daemon=True)
                    threads.append(th)
                    th.start()
                    admitted = True
                if admitted:
                    continue
                # wait for a completion or the next arrival
                wait = None
                if i < len(reqs) and state["active"] < self.max_active:
                    wait = max(0.0, reqs[i].arrival - now)
                lock.wait(timeout=wait if wait is not None else 1.0)
        for th in threads:
            th.join()
        if errors:
            raise RuntimeError("requests failed: %s" % errors)
        return [results[q.rid] for q in requests]


def poisson_arrivals(n: int, rate: float, seed: int) -> np.ndarray:
    """n arrival times of a Poisson process of the given rate (per second)."""
    rng = np.random.default_rng(seed)
    return np.cumsum(rng.exponential(1.0 / rate, size=n))


def latency_percentiles(results: List[Result]):
    lat = np.array([r.latency for r in results])
    return float(np.percentile(lat, 50)), float(np.percentile(lat, 99))
