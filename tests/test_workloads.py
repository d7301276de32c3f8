"""The seeded inputs: shapes, structure and regions follow their recipes, and
the stored oracle values belong to the workload that regenerates today."""
import json
import os

import numpy as np
import pytest

import workloads

GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def test_toeplitz_structure_and_numerical_range_box():
    wl = workloads.toeplitz_band(n=300, grid=7)
    C = wl.dense
    t = wl.info["toeplitz"]
    i, j = np.indices(C.shape)
    d = j - i
    assert np.all(C[(d < -1) | (d > 3)] == 0)                  # one sub-, three superdiagonals
    for k in range(-1, 4):
        assert np.all(C[d == k] == t[k + 1])
    # bounding box of the numerical range from dense Hermitian / skew parts, padded 10%
    H = (C + C.conj().T) / 2
    K = (C - C.conj().T) / 2j
    hx, kx = np.linalg.eigvalsh(H), np.linalg.eigvalsh(K)
    wx, wy = hx[-1] - hx[0], kx[-1] - kx[0]
    want = (hx[0] - 0.1 * wx, hx[-1] + 0.1 * wx, kx[0] - 0.1 * wy, kx[-1] + 0.1 * wy)
    assert np.allclose(wl.region, want, atol=1e-10)


def test_seeded_draws_repeat():
    a = workloads.triangular_disk(seed=1001, n=50, grid=4)
    b = workloads.triangular_disk(seed=1001, n=50, grid=4)
    assert np.array_equal(a.dense, b.dense)
    lam = np.diag(a.dense)
    assert np.all(np.abs(lam) <= 1.0)                            # eigenvalues in the unit disk
    assert np.allclose(np.tril(a.dense, -1), 0)                  # upper triangular


def test_golden_reference_matches_generator():
    path = os.path.join(GOLD, "toeplitz_n4000_grid200_sigma.json")
    if not os.path.exists(path):
        pytest.skip("stored oracle values not generated")
    meta = json.load(open(path))
    wl = workloads.toeplitz_band()
    assert (meta["n"], meta["nx"], meta["ny"]) == (wl.n, wl.nx, wl.ny)
    assert np.allclose(meta["region"], wl.region, rtol=0, atol=1e-12)
    assert meta["c00"] == [float(wl.dense[0, 0].real), float(wl.dense[0, 0].imag)]
    sig = np.load(os.path.join(GOLD, "toeplitz_n4000_grid200_sigma.npy"))
    assert sig.shape == (wl.nx * wl.ny,) and np.all(np.isfinite(sig)) and np.all(sig >= 0)


def _dense_from_csr(wl):
    C = np.zeros((wl.m, wl.n), dtype=np.complex128)
    for r in range(wl.m):
        for p in range(wl.rowptr[r], wl.rowptr[r + 1]):
            C[r, wl.colind[p]] += wl.vals[p]
    return C


def test_convection_diffusion_stencil_by_loops():
    """The CSR stencil against the stencil written out point by point: centre
    4, west/south -1 - beta, east/north -1 + beta, beta = Pe h / (2 sqrt 2),
    Dirichlet boundary, index i + N j, each row times its own phase."""
    import math
    N, Pe = 6, 50.0
    wl = workloads.convection_diffusion(seed=7, N=N, grid=4, region_override=(0, 1, 0, 1), peclet=Pe)
    n = N * N
    h = 1.0 / (N + 1)
    beta = Pe * h / (2 * math.sqrt(2))
    A = np.zeros((n, n), dtype=np.complex128)
    for j in range(N):
        for i in range(N):
            p = i + N * j
            A[p, p] = 4.0
            if i > 0:
                A[p, p - 1] = -1 - beta
            if j > 0:
                A[p, p - N] = -1 - beta
            if i < N - 1:
                A[p, p + 1] = -1 + beta
            if j < N - 1:
                A[p, p + N] = -1 + beta
    C = _dense_from_csr(wl)
    assert wl.rowptr[-1] == 5 * N * N - 4 * N                 # nnz = 5N^2 - 4N
    ph = C[np.arange(n), np.arange(n)] / 4.0                 # the row phases
    assert np.allclose(np.abs(ph), 1.0)
    assert np.allclose(C, ph[:, None] * A)
    for r in range(n):                                       # sorted column indices per row
        cols = wl.colind[wl.rowptr[r]:wl.rowptr[r + 1]]
        assert np.all(np.diff(cols) > 0)


def test_folding_is_a_banded_toeplitz_truncation():
    """m = n + 4 rows, entry (j, k) = a_{j-k} for |j - k| <= 4 (all nine
    entries in every column from the fifth on), and a region that contains
    the symbol curve."""
    wl = workloads.folding(seed=11, n=30, grid=8)
    a = wl.info["toeplitz"]
    C = _dense_from_csr(wl)
    assert (wl.m, wl.n) == (34, 30)
    for j in range(wl.m):
        for k in range(wl.n):
            d = j - k
            assert C[j, k] == (a[d + 4] if abs(d) <= 4 else 0)
    assert np.all(np.count_nonzero(C, axis=0) == np.minimum(np.arange(wl.n) + 5, 9))
    th = np.linspace(0, 2 * np.pi, 512)
    sym = sum(a[d + 4] * np.exp(1j * d * th) for d in range(-4, 5))
    re_lo, re_hi, im_lo, im_hi = wl.region
    assert re_lo < sym.real.min() and sym.real.max() < re_hi
    assert im_lo < sym.imag.min() and sym.imag.max() < im_hi


def test_triangular_disk_draw_order():
    """u, v, then an n x n CN(0,1) block whose strict upper triangle / sqrt(n)
    is N: the matrix regenerates from the stated draw order."""
    import math
    n = 9
    wl = workloads.triangular_disk(seed=1234, n=n, grid=3)
    rng = np.random.default_rng(1234)
    u = rng.random(n)
    v = rng.random(n)
    G = (rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))) / math.sqrt(2)
    C = np.diag(np.sqrt(u) * np.exp(2j * np.pi * v)) + np.triu(G, 1) / math.sqrt(n)
    assert np.allclose(wl.dense, C, rtol=0, atol=1e-15)
    assert wl.region == (-2.0, 2.0, -2.0, 2.0)


def test_batched_and_serving_streams_follow_their_ranges():
    ws = workloads.batched_uneven(seed=1004, n_dense=6, n_fold=3, grid=4, dense_range=(64, 80),
                                  fold_range=(100, 120))
    assert len(ws) == 9
    assert all(w.kind == "dense" and 64 <= w.n <= 80 and w.m == w.n for w in ws[:6])
    assert all(w.kind == "csr" and 100 <= w.n <= 120 and w.m == w.n + 4 for w in ws[6:])
    reqs = workloads.serving_requests(seed=1005, n_req=8, dense_range=(64, 80), sparse_N_range=(10, 12),
                                      grid_range=(4, 6))
    assert len(reqs) == 8
    for r in reqs:
        assert 4 <= r.nx <= 6 and r.nx == r.ny
        if r.kind == "dense":
            assert 64 <= r.n <= 80
        else:
            assert int(round(r.n ** 0.5)) ** 2 == r.n and 10 <= int(round(r.n ** 0.5)) <= 12
