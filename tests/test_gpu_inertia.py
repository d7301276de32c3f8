"""The inertia test behind the certificates (marked gpu): N(z) - mu I is
reported positive definite exactly when mu < sigma_min(C - z I)^2, checked
with mu 1% below and above sigma_min^2 from LAPACK (Sylvester's law of
inertia: every Cholesky pivot is positive iff the Hermitian matrix is
positive definite).  Dense handles factor N(z) - mu I densely; a CSR
folding (N = C^* C of bandwidth 8) by the band Cholesky."""
import numpy as np
import pytest

import workloads

P = pytest.importorskip("paper_2606_26785_amd")

pytestmark = pytest.mark.gpu


def _smin(A, z):
    m, n = A.shape
    return np.linalg.svd(A - z * np.eye(m, n), compute_uv=False)[-1]


@pytest.mark.parametrize("kind", ["dense", "csr-folding"])
def test_inertia_brackets_sigma_min(kind):
    if kind == "dense":
        wl = workloads.triangular_disk(seed=5, n=150, grid=4)
    else:
        wl = workloads.folding(seed=77, n=300, grid=4)
    A = wl.to_dense()
    mat = P.create_from_workload(wl, params=P.default_params(precond=1))
    try:
        for z in (wl.z_center, complex(wl.region[0], wl.region[2]), 0.3 + 0.1j):
            s = _smin(A, z)
            assert P.debug_inertia(mat, z, 0.99 * s * s), (kind, z, s)
            assert not P.debug_inertia(mat, z, 1.01 * s * s), (kind, z, s)
    finally:
        mat.close()


def test_folding_parity_with_certificates():
    """A rectangular folding on the GPU with the incomplete Cholesky base and
    the band-Cholesky certificates, against the banded oracle."""
    import oracle
    wl = workloads.folding(seed=77, n=400, grid=10)
    zs = oracle.grid_points(*wl.region, wl.nx, wl.ny)
    band, kl, ku = oracle.band_from_csr(wl.m, wl.n, wl.rowptr, wl.colind, wl.vals)
    ref = oracle.sigma_min_banded(band, wl.m, wl.n, kl, ku, zs)
    nC = float(oracle.banded_smallest(band, wl.m, wl.n, kl, ku, 0.0, k=wl.n)[-1])
    mat = P.create_from_workload(wl)
    g = P.ps_grid(*wl.region, wl.nx, wl.ny)
    res = P.ps_eval(mat, g, wl.eps)
    mat.close()
    err = np.abs(res.sigma - ref)
    print("folding n=400 m=404 10x10: max|err|/|C| = %.2e, stats %s" % (err.max() / nC, {
        k: res.stats[k] for k in ("refined", "certified", "cert_tests", "uncertified", "lobpcg_iters")}), flush=True)
    assert err.max() <= 1e-8 * nC
    assert (res.sigma >= ref - 1e-11 * nC).all()
