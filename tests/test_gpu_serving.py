"""Serving on the GPU (marked gpu): a small seeded stream of mixed requests
(dense triangular and CSR convection-diffusion, uneven sizes and grids)
served concurrently, each on its own handle and stream, must give the
results of each request run alone within 1e-8 ||C||_2 (tolerance-equal; the
test does not ask for bit equality), and a sample of each request's points
must match the dense Jacobi oracle."""
import numpy as np
import pytest

import oracle
import workloads

P = pytest.importorskip("paper_2606_26785_amd")
from paper_2606_26785_amd import serving  # noqa: E402

pytestmark = pytest.mark.gpu

TOL = 1e-8


def _norm2(wl):
    if wl.kind == "dense":
        return float(np.linalg.norm(wl.dense, 2))
    return oracle.norm2_sparse(wl.n, wl.n, wl.rowptr, wl.colind, wl.vals)


def test_alone_vs_mix():
    wls = workloads.serving_requests(seed=1005, n_req=6, dense_range=(96, 192), sparse_N_range=(16, 24),
                                     grid_range=(6, 9))
    assert {w.kind for w in wls} == {"dense", "csr"}
    reqs = [serving.Request(i, wl, 0.02 * i) for i, wl in enumerate(wls)]
    be = serving.LibraryBackend()
    alone = []
    for q in reqs:
        print("alone: request %d %s n=%d grid %d" % (q.rid, q.workload.name, q.workload.n, q.workload.nx), flush=True)
        alone.append(be.run(q))
    budget = sum(serving.footprint_bytes(w) for w in wls)
    srv = serving.Server(be, hbm_budget=budget, max_active=4)
    print("mix: %d requests, budget %.1f GB" % (len(reqs), budget / 1e9), flush=True)
    mix = srv.run(reqs, time_limit=240)
    assert srv.peak_active >= 2
    for q, a, r in zip(reqs, alone, mix):
        wl = q.workload
        nC = _norm2(wl)
        err = np.max(np.abs(r.sigma - a[0]))
        print("request %d (%s, n=%d): max|mix - alone|/|C| = %.2e, latency %.2f s" % (
            q.rid, wl.name, wl.n, err / nC, r.latency), flush=True)
        assert err <= TOL * nC
        # membership equal away from the levels
        far = np.abs(a[0][None, :] - np.asarray(wl.eps)[:, None]) > TOL * nC
        assert np.array_equal(r.member[far], a[1][far])
        # a sample against the oracle
        zs = oracle.grid_points(*wl.region, wl.nx, wl.ny)
        idx = workloads.sample_indices(zs.size, 4, 77 + q.rid)
        ref, sw = oracle.sigma_min_dense(wl.to_dense(), zs[idx])
        assert (sw > 0).all()
        assert np.max(np.abs(r.sigma[idx] - ref)) <= TOL * nC
