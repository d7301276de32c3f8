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
