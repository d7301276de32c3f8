"""The two-level preconditioner on the GPU (marked gpu), against dense numpy
linear algebra of the same definitions (paper Sec. 3):

* the base preconditioner K = F^* F = N(z_dag) + d I built at a site z_dag,
  with N(z) = (C - z I)^* (C - z I);
* the projection vectors Ebar = F^{-1} Xbar from the projection LOBPCG-SVD on
  Mbar(z) = C(z) F^{-1} at a nearby point z: K-orthonormal (eq. (genM)) and
  close to the smallest eigenvectors of the pencil (N(z), K);
* the apply K_Ebar^{-1} W = K^{-1} W + Ebar Lambda_bar^{-1} Ebar^* W
  (eq. (twolevel) with Z = Ebar, Z^* N(z) Z = Lambda_bar);
* Lemma 3.1: the eigenvalues of K_Ebar^{-1} N(z) are those of the pencil
  with the rbar smallest raised by one.
"""
import numpy as np
import pytest
import scipy.linalg as sla

import workloads

P = pytest.importorskip("paper_2606_26785_amd")

pytestmark = pytest.mark.gpu


def _cplx(rng, *shape):
    return (rng.standard_normal(shape) + 1j * rng.standard_normal(shape)) / np.sqrt(2)


@pytest.mark.parametrize("n,offset", [(120, 1e-3), (200, 3e-2)])
def test_two_level_preconditioner_lemma(n, offset):
    wl = workloads.triangular_disk(seed=1001, n=n, grid=4)
    C = wl.dense
    lam_c = np.diag(C)
    z = lam_c[0] + offset          # near an eigenvalue: C(z) has small singular values
    zdag = z + 0.05
    mat = P.ps_create(dense=C, params=P.default_params(precond=2, eta_proj=1e-10))
    rng = np.random.default_rng(n)
    W = _cplx(rng, n, 8)
    Y, E, lam, it, d, gamma = P.debug_twolevel(mat, zdag, z, W)
    mat.close()
    I = np.eye(n)
    Ad = C - zdag * I
    K = Ad.conj().T @ Ad + d * I
    Az = C - z * I
    Nz = Az.conj().T @ Az
    print("n=%d iters=%d d=%.3e gamma=%.3e lam=%s" % (n, it, d, gamma, np.array2string(lam, precision=3)))
    # gamma = ||F^{-1}||_2 = lambda_min(K)^{-1/2}, estimated by twelve power
    # steps (from below)
    g_ref = 1.0 / np.sqrt(np.linalg.eigvalsh(K)[0])
    assert 0.99 * g_ref <= gamma <= g_ref * (1 + 1e-9)
    # Ebar is K-orthonormal
    assert np.max(np.abs(E.conj().T @ K @ E - np.eye(8))) <= 1e-9
    # the apply follows eq. (twolevel)
    Yref = np.linalg.solve(K, W) + E @ ((E.conj().T @ W) / lam[:, None])
    assert np.max(np.abs(Y - Yref)) <= 1e-9 * np.max(np.abs(Yref))
    # Ebar spans the eigenvectors of the 8 smallest pencil eigenvalues
    pen = sla.eigh(Nz, K, eigvals_only=True)
    assert np.max(np.abs(np.sort(lam) - pen[:8])) <= 1e-8 * pen[-1]
    # Lemma 3.1
    KE = np.linalg.inv(K) + E @ np.diag(1.0 / lam) @ E.conj().T
    got = np.sort(np.linalg.eigvals(KE @ Nz).real)
    want = np.sort(np.concatenate([pen[:8] + 1.0, pen[8:]]))
    assert np.max(np.abs(got - want)) <= 1e-6 * want[-1]
