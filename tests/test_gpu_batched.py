"""A batch of uneven matrices on the GPU (marked gpu): dense triangular
matrices of different sizes and rectangular CSR foldings, all submitted at
once and run with continuous batching (one handle and stream each, several
at a time), every point against the oracle (O1 for dense, the banded O2 for
the foldings) at 1e-8 ||C||_2."""
import numpy as np
import pytest

import oracle
import workloads

P = pytest.importorskip("paper_2606_26785_amd")
from paper_2606_26785_amd import serving  # noqa: E402

pytestmark = pytest.mark.gpu

TOL = 1e-8


def test_uneven_batch_parity():
    wls = workloads.batched_uneven(seed=1004, n_dense=3, n_fold=2, grid=5, dense_range=(64, 160),
                                   fold_range=(150, 300))
    reqs = [serving.Request(i, wl, 0.0) for i, wl in enumerate(wls)]
    be = serving.LibraryBackend()
    budget = sum(serving.footprint_bytes(w) for w in wls)
    srv = serving.Server(be, hbm_budget=budget, max_active=len(wls))
    res = srv.run(reqs, time_limit=240)
    assert srv.peak_active >= 2
    for wl, r in zip(wls, res):
        zs = oracle.grid_points(*wl.region, wl.nx, wl.ny)
        if wl.kind == "dense":
            ref, sw = oracle.sigma_min_dense(wl.dense, zs)
            assert (sw > 0).all()
            nC = float(np.linalg.norm(wl.dense, 2))
        else:
            band, kl, ku = oracle.band_from_csr(wl.m, wl.n, wl.rowptr, wl.colind, wl.vals)
            ref = oracle.sigma_min_banded(band, wl.m, wl.n, kl, ku, zs)
            nC = float(oracle.banded_smallest(band, wl.m, wl.n, kl, ku, 0.0, k=wl.n)[-1])
        err = np.abs(r.sigma - ref)
        print("%s (m=%d n=%d): max|err|/|C| = %.2e, latency %.2f s" % (wl.name, wl.m, wl.n, err.max() / nC,
                                                                      r.latency), flush=True)
        assert err.max() <= TOL * nC
        assert (r.sigma >= ref - 1e-11 * nC).all()
