"""CPU checks (numpy) of the identities the GPU path is built on, each a
restatement of the paper's algebra or of a textbook fact, independent of the
HIP code:

* cached R factors: with W1 = C V, W2 = S V and [W1 W2] = Q_A R_A, the Ritz
  singular values of C(z) = C - z S on span V (Sec. 2.2, Alg. 1) are the
  singular values of B(z) = R_A[:, :k] - z R_A[:, k:], and B^* B equals the
  projected matrix H(z) = H1 - z H2 - conj(z) H2^* + |z|^2 H3 of eq. (H);
* the residual norm of a Ritz pair from R_res, the R factor of
  [C^*C V, C^*S V, S^*C V, V] (eq. (fastresidual), S^* S = I_n);
* the neighbour bound: for a unit x, ||C(z) x||^2 = ||C(z') x||^2 -
  2 Re(conj(z - z') gamma) + |z - z'|^2 ||S x||^2 with gamma = (S x)^* C(z') x;
* the inertia test: N(z) - mu I has a Cholesky factor iff mu < sigma_min^2.
"""
import numpy as np
import pytest


def _cn(rng, *shape):
    return (rng.standard_normal(shape) + 1j * rng.standard_normal(shape)) / np.sqrt(2)


def _setup(m=40, n=30, k=8, seed=3):
    rng = np.random.default_rng(seed)
    C = _cn(rng, m, n)
    S = np.zeros((m, n), complex)
    S[np.arange(n), np.arange(n)] = 1.0
    V, _ = np.linalg.qr(_cn(rng, n, k))
    return C, S, V


@pytest.mark.parametrize("z", [0.3 - 0.2j, -1.1 + 0.7j, 0.0])
def test_cached_r_factor_ritz_values(z):
    C, S, V = _setup()
    k = V.shape[1]
    W1, W2 = C @ V, S @ V
    RA = np.linalg.qr(np.hstack([W1, W2]), mode="r")
    B = RA[:, :k] - z * RA[:, k:]
    direct = np.linalg.svd((C - z * S) @ V, compute_uv=False)
    assert np.allclose(np.linalg.svd(B, compute_uv=False), direct, rtol=0, atol=1e-12)
    H1, H2, H3 = W1.conj().T @ W1, W1.conj().T @ W2, W2.conj().T @ W2
    Hz = H1 - z * H2 - np.conj(z) * H2.conj().T + abs(z) ** 2 * H3
    assert np.allclose(B.conj().T @ B, Hz, atol=1e-12)
    assert np.allclose(np.sqrt(np.sort(np.linalg.eigvalsh(Hz))), np.sort(direct), atol=1e-7)


@pytest.mark.parametrize("z", [0.3 - 0.2j, 1.5j])
def test_residual_from_cached_r_factor(z):
    C, S, V = _setup()
    k = V.shape[1]
    W3, W4, W5 = C.conj().T @ C @ V, C.conj().T @ S @ V, S.conj().T @ C @ V
    Rres = np.linalg.qr(np.hstack([W3, W4, W5, V]), mode="r")
    _, s, Gh = np.linalg.svd((C - z * S) @ V)
    g, xi = Gh.conj().T[:, -1], s[-1]            # smallest Ritz pair
    x = V @ g
    T = (C - z * S).conj().T @ (C - z * S)
    direct = np.linalg.norm(T @ x - xi ** 2 * x)
    u = np.concatenate([g, -z * g, -np.conj(z) * g, (abs(z) ** 2 - xi ** 2) * g])
    assert abs(np.linalg.norm(Rres @ u) - direct) <= 1e-10 * max(1.0, direct)
    assert k == V.shape[1]


def test_neighbour_bound_expansion():
    C, S, _ = _setup(m=34, n=30)
    rng = np.random.default_rng(9)
    x = _cn(rng, 30)
    x /= np.linalg.norm(x)
    zq, z = 0.4 + 0.1j, 0.43 + 0.08j
    sq = np.linalg.norm((C - zq * S) @ x)
    gamma = np.vdot(S @ x, (C - zq * S) @ x)
    d = z - zq
    bound2 = sq ** 2 - 2 * (np.conj(d) * gamma).real + abs(d) ** 2 * np.linalg.norm(S @ x) ** 2
    assert abs(np.sqrt(bound2) - np.linalg.norm((C - z * S) @ x)) <= 1e-12
    # and it bounds sigma_min(C(z)) from above, below the 1-Lipschitz bound
    smin = np.linalg.svd(C - z * S, compute_uv=False)[-1]
    assert smin <= np.sqrt(bound2) + 1e-12 <= sq + abs(d) + 1e-12


def test_inertia_test_brackets_sigma_min():
    C, S, _ = _setup(m=30, n=30, seed=5)
    z = 0.2 + 0.3j
    A = C - z * S
    N = A.conj().T @ A
    smin = np.linalg.svd(A, compute_uv=False)[-1]
    for f, expect in ((0.999, True), (0.9, True), (1.001, False), (1.2, False)):
        mu = (f * smin) ** 2
        try:
            np.linalg.cholesky(N - mu * np.eye(30))
            ok = True
        except np.linalg.LinAlgError:
            ok = False
        assert ok == expect, (f, ok)


def test_two_level_preconditioner_lifts_smallest_pencil_eigenvalues():
    """Lemma 3.1 (Sec. 3.1): with E the K-orthonormal eigenvectors of the
    rbar smallest eigenvalues of the pencil (N, K), K_E^{-1} = K^{-1} +
    E Lambda^{-1} E^* (eq. (twolevel) with Z = E, since Z^* N Z = Lambda)
    maps them to lambda_j + 1 and leaves the others.  The coarse part of the
    preconditioner is not built in this version; this pins the reading of
    Z^* N(z) Z it relies on."""
    rng = np.random.default_rng(11)
    n, rbar = 24, 4
    A = _cn(rng, n, n)
    N = A.conj().T @ A + 1e-3 * np.eye(n)
    B = _cn(rng, n, n)
    K = B.conj().T @ B + n * np.eye(n)
    Fc = np.linalg.cholesky(K).conj().T                 # K = F^* F
    Fi = np.linalg.inv(Fc)
    lam, Xb = np.linalg.eigh(Fi.conj().T @ N @ Fi)      # F^{-*} N F^{-1} Xbar = Xbar Lambda
    E = Fi @ Xb[:, :rbar]                               # E = F^{-1} Xbar, K-orthonormal
    assert np.allclose(E.conj().T @ K @ E, np.eye(rbar), atol=1e-10)
    assert np.allclose(E.conj().T @ N @ E, np.diag(lam[:rbar]), atol=1e-8)
    KEinv = np.linalg.inv(K) + E @ np.diag(1.0 / lam[:rbar]) @ E.conj().T
    got = np.sort(np.linalg.eigvals(KEinv @ N).real)
    want = np.sort(np.concatenate([lam[:rbar] + 1.0, lam[rbar:]]))
    assert np.allclose(got, want, rtol=1e-8, atol=1e-8)
