"""The sparse path on the GPU (marked gpu): a CSR convection-diffusion C with
the two-level preconditioner over an incomplete-Cholesky base (paper Sec. 3),
against the oracle.

* reduced instances (N = 30 and N = 50, n = 900 and 2,500) on whole grids,
  against the dense Jacobi oracle O1 (N = 30) and the sparse scale oracle O2
  (N = 50), which is itself pinned to O1 on the CPU;
* the full size (N = 500, n = 250,000) on the 20 x 20 sub-grid (every 5th
  line of the 100 x 100 grid) that holds the 64 points stored by
  tests/golden/make_convdiff_ref.py from O2.
"""
import json
import os

import numpy as np
import pytest

import oracle
import workloads

P = pytest.importorskip("paper_2606_26785_amd")

pytestmark = pytest.mark.gpu

TOL = 1e-8
LOW = 1e-11
GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "convdiff_n250000_grid100_sigma.json")


def _check(res, ref, normC, eps, label):
    sig = res.sigma
    err = np.abs(sig - ref)
    print("%s: max|err|/|C| = %.3e, points %d, stats %s" % (
        label, err.max() / normC, sig.size, {k: res.stats[k] for k in (
            "accepted", "refined", "uncertified", "lobpcg_iters", "rebuilds", "proj_accepted", "proj_refined",
            "proj_iters", "t_total_ms")}), flush=True)
    assert err.max() <= TOL * normC, "%s: worst %g at %d" % (label, err.max(), int(np.argmax(err)))
    assert (sig >= ref - LOW * normC).all(), label
    if len(eps):
        far = np.abs(ref[None, :] - np.asarray(eps)[:, None]) > TOL * normC
        assert np.array_equal(res.member[far], oracle.membership(ref, eps)[far])


def _eval(wl, region, nx, ny, **pk):
    mat = P.create_from_workload(wl, params=P.default_params(**pk))
    g = P.ps_grid(*region, nx, ny)
    res = P.ps_eval(mat, g, wl.eps)
    mat.close()
    return res


@pytest.mark.parametrize("N,grid,ref_kind", [(30, 10, "O1"), (50, 12, "O2")])
def test_convdiff_reduced_parity(N, grid, ref_kind):
    wl = workloads.convection_diffusion(N=N, grid=grid)
    zs = oracle.grid_points(*wl.region, wl.nx, wl.ny)
    normC = oracle.norm2_sparse(wl.n, wl.n, wl.rowptr, wl.colind, wl.vals)
    if ref_kind == "O1":
        ref, sw = oracle.sigma_min_dense(wl.to_dense(), zs)
        assert (sw > 0).all()
    else:
        ref, steps = oracle.sigma_min_sparse_lu(wl.n, wl.n, wl.rowptr, wl.colind, wl.vals, zs, normC=normC)
        assert (steps >= 0).all()
    res = _eval(wl, wl.region, wl.nx, wl.ny)
    _check(res, ref, normC, wl.eps, "convdiff N=%d %dx%d" % (N, grid, grid))
    assert res.stats["rebuilds"] >= 1


@pytest.mark.parametrize("N,which", [(12, "centre"), (17, "corner")])
def test_incomplete_cholesky_site(N, which):
    """The sparse base site: K = F^* F from the GPU factor agrees with
    N(z) + alpha I on the pattern of C^* C (incomplete Cholesky without fill
    is exact there), K is Hermitian positive definite, and F^{-*} is the
    conjugate transpose of F^{-1}."""
    wl = workloads.convection_diffusion(N=N, grid=4)
    n = wl.n
    z = wl.z_center if which == "centre" else complex(wl.region[0], wl.region[2])
    mat = P.create_from_workload(wl, params=P.default_params(precond=1))
    try:
        I = np.eye(n, dtype=np.complex128)
        Fi = np.hstack([P.debug_sparse_site(mat, z, I[:, c:c + 64], 0)[0] for c in range(0, n, 64)])
        Fh = np.hstack([P.debug_sparse_site(mat, z, I[:, c:c + 64], 1)[0] for c in range(0, n, 64)])
        alpha = P.debug_sparse_site(mat, z, I[:, :1], 0)[1]
    finally:
        mat.close()
    assert alpha > 0
    assert np.max(np.abs(Fh - Fi.conj().T)) <= 1e-12 * np.max(np.abs(Fi))
    F = np.linalg.inv(Fi)
    K = F.conj().T @ F
    A = wl.to_dense() - z * np.eye(n)
    Nz = A.conj().T @ A + alpha * np.eye(n)
    pat = (np.abs(wl.to_dense().conj().T) @ np.abs(wl.to_dense()) + np.eye(n)) > 0
    scale = np.max(np.abs(Nz))
    assert np.max(np.abs((K - Nz)[pat])) <= 1e-10 * scale
    assert np.max(np.abs(K - K.conj().T)) <= 1e-10 * scale
    assert np.linalg.eigvalsh(0.5 * (K + K.conj().T)).min() > 0


def test_convdiff_base_only_parity():
    wl = workloads.convection_diffusion(N=30, grid=8)
    zs = oracle.grid_points(*wl.region, wl.nx, wl.ny)
    ref, sw = oracle.sigma_min_dense(wl.to_dense(), zs)
    normC = oracle.norm2_sparse(wl.n, wl.n, wl.rowptr, wl.colind, wl.vals)
    res = _eval(wl, wl.region, wl.nx, wl.ny, precond=1)
    _check(res, ref, normC, wl.eps, "convdiff N=30 8x8 base preconditioner only")


def test_convdiff_full_size_sample():
    if not os.path.exists(GOLD):
        pytest.skip("stored oracle values not generated")
    meta = json.load(open(GOLD))
    wl = workloads.convection_diffusion()
    assert np.allclose(meta["region"], wl.region, rtol=0, atol=1e-12)
    stride = 5
    nxs = (wl.nx - 1) // stride + 1
    nys = (wl.ny - 1) // stride + 1
    re_lo, re_hi, im_lo, im_hi = wl.region
    hx = (re_hi - re_lo) / (wl.nx - 1)
    hy = (im_hi - im_lo) / (wl.ny - 1)
    region = (re_lo, re_lo + (nxs - 1) * stride * hx, im_lo, im_lo + (nys - 1) * stride * hy)
    res = _eval(wl, region, nxs, nys)
    idx = np.asarray(meta["indices"])
    i, j = idx % wl.nx, idx // wl.nx
    assert (i % stride == 0).all() and (j % stride == 0).all()
    sub = (j // stride) * nxs + (i // stride)
    ref = np.asarray(meta["sigma"])

    class R:
        pass
    r = R()
    r.sigma = res.sigma[sub]
    r.member = res.member[:, sub]
    r.stats = res.stats
    _check(r, ref, float(meta["normC"]), wl.eps, "convdiff N=500 sample of %d points" % ref.size)
