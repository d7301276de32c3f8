"""Host logic of the serving loop (CPU): admission by memory footprint in
arrival order, the concurrency cap, no admission before arrival, results in
request order, error propagation, and the Poisson arrival generator.  The
backend is a stand-in that sleeps; the GPU alone-vs-mix test is in
test_gpu_serving.py."""
import threading
import time

import numpy as np
import pytest

from paper_2606_26785_amd import serving


class FakeWorkload:
    def __init__(self, size, dur):
        self.size = size
        self.dur = dur


class SleepBackend:
    """Records the memory in use and the number of running requests."""

    def __init__(self, server_ref):
        self.lock = threading.Lock()
        self.used = 0
        self.active = 0
        self.max_used = 0
        self.max_active = 0
        self.starts = {}
        self.server_ref = server_ref

    def run(self, req):
        wl = req.workload
        with self.lock:
            self.used += wl.size
            self.active += 1
            self.max_used = max(self.max_used, self.used)
            self.max_active = max(self.max_active, self.active)
            self.starts[req.rid] = time.perf_counter()
        time.sleep(wl.dur)
        with self.lock:
            self.used -= wl.size
            self.active -= 1
        if wl.size < 0:
            raise RuntimeError("bad request")
        return np.full(4, req.rid, dtype=float), np.zeros((1, 4), np.uint8), np.zeros(4, np.uint8), {"rid": req.rid}


def _serve(sizes, durs, arrivals, budget, max_active, time_limit=30.0):
    reqs = [serving.Request(i, FakeWorkload(s, d), a) for i, (s, d, a) in enumerate(zip(sizes, durs, arrivals))]
    be = SleepBackend(None)
    srv = serving.Server(be, hbm_budget=budget, max_active=max_active, footprint=lambda wl: abs(wl.size))
    t0 = time.perf_counter()
    res = srv.run(reqs, time_limit=time_limit)
    return reqs, res, be, srv, t0


def test_admission_respects_budget_and_cap():
    rng = np.random.default_rng(5)
    sizes = rng.integers(1, 6, size=24)
    durs = rng.uniform(0.01, 0.05, size=24)
    arrivals = np.zeros(24)
    reqs, res, be, srv, _ = _serve(sizes, durs, arrivals, budget=10, max_active=3)
    assert be.max_used <= 10
    assert be.max_active <= 3
    assert srv.peak_bytes <= 10 and srv.peak_active <= 3
    # more than one request ran at a time (continuous batching)
    assert be.max_active >= 2
    assert [r.rid for r in res] == list(range(24))
    for r in res:
        assert np.all(r.sigma == r.rid)
        assert r.start >= r.arrival and r.done >= r.start


def test_admission_in_arrival_order():
    # a large request blocks the small ones behind it (no overtaking)
    sizes = [6, 8, 1, 1]
    durs = [0.15, 0.05, 0.01, 0.01]
    arrivals = [0.0, 0.01, 0.02, 0.03]
    reqs, res, be, srv, _ = _serve(sizes, durs, arrivals, budget=10, max_active=4)
    start = {r.rid: r.start for r in res}
    assert start[1] >= start[0]
    assert start[2] >= start[1] and start[3] >= start[2]
    # request 1 (8) could only start once request 0 (6) had finished
    assert start[1] >= res[0].done - 1e-3


def test_no_admission_before_arrival():
    arrivals = [0.0, 0.2, 0.25]
    reqs, res, be, srv, _ = _serve([1, 1, 1], [0.01, 0.01, 0.01], arrivals, budget=10, max_active=4)
    for r in res:
        assert r.start >= r.arrival - 1e-6
        assert r.latency >= 0.0


def test_oversized_request_rejected():
    with pytest.raises(ValueError):
        _serve([11], [0.01], [0.0], budget=10, max_active=2)


def test_errors_propagate():
    with pytest.raises(RuntimeError):
        _serve([1, -1, 1], [0.01, 0.01, 0.01], [0.0, 0.0, 0.0], budget=10, max_active=2)


def test_poisson_arrivals_and_percentiles():
    t = serving.poisson_arrivals(20000, rate=4.0, seed=7)
    assert np.all(np.diff(t) > 0)
    gaps = np.diff(np.concatenate([[0.0], t]))
    assert abs(gaps.mean() - 0.25) < 0.01
    # exponential gaps: std equals the mean
    assert abs(gaps.std() - 0.25) < 0.01

    class R:
        def __init__(self, lat):
            self.latency = lat
    p50, p99 = serving.latency_percentiles([R(x) for x in range(1, 101)])
    assert p50 == pytest.approx(50.5) and p99 == pytest.approx(99.01)


def test_footprint_grows_with_size():
    import workloads
    a = workloads.triangular_disk(seed=1, n=64, grid=8)
    b = workloads.triangular_disk(seed=1, n=256, grid=8)
    c = workloads.convection_diffusion(N=30, grid=8)
    fa, fb, fc = (serving.footprint_bytes(w) for w in (a, b, c))
    assert 0 < fa < fb
    assert fc > 0
    # the per-request caps bound it
    assert fb < (serving.SERVE_TILE_MEM_GB + serving.SERVE_SITE_MEM_GB + 2) * (1 << 30)
