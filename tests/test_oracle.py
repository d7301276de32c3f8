"""Pins of the oracle to facts outside itself (CPU only).

The oracle computes sigma_min(C - z I_{m x n}) (paper, Sec. 1, eq.
(defSquareSVD)).  Each test below fixes it by something it does not
compute itself: LAPACK's SVD, closed forms for normal matrices, invariance
under unitary similarity, the 1-Lipschitz bound in z, brute force on tiny
matrices, eigenvalue bounds, folding monotonicity and Weyl's perturbation
bound.  A dropped term, a sign error, a transposed operand or a wrong index
in either oracle method makes at least one of them fail.
"""
import numpy as np
import pytest

import oracle
import workloads


def _cplx(rng, *shape):
    return (rng.standard_normal(shape) + 1j * rng.standard_normal(shape)) / np.sqrt(2)


def _haar_unitary(rng, n):
    Z = _cplx(rng, n, n)
    Q, R = np.linalg.qr(Z)
    d = np.diag(R)
    return Q * (d / np.abs(d))[None, :]


@pytest.mark.parametrize("m,n", [(1, 1), (4, 4), (17, 17), (40, 40), (23, 11), (9, 1)])
def test_o1_all_singular_values_match_lapack(m, n):
    rng = np.random.default_rng(m * 100 + n)
    A = _cplx(rng, m, n) * rng.uniform(0.1, 10.0)
    s = oracle.singular_values_dense(A)
    ref = np.linalg.svd(A, compute_uv=False)
    assert np.max(np.abs(s - ref)) <= 1e-12 * ref[0]


def test_o1_graded_columns_small_singular_value():
    # A matrix with a singular value 1e-12 below the largest: absolute
    # accuracy ~ eps ||A|| is what the definition needs.
    rng = np.random.default_rng(3)
    U = _haar_unitary(rng, 30)
    V = _haar_unitary(rng, 30)
    s = np.logspace(0, -12, 30)
    A = (U * s[None, :]) @ V.conj().T
    got = oracle.singular_values_dense(A)
    assert np.max(np.abs(got - s)) <= 1e-14 * 30


def test_o1_normal_closed_form_square():
    rng = np.random.default_rng(11)
    n = 32
    lam = _cplx(rng, n) * 1.5
    U = _haar_unitary(rng, n)
    C = (U * lam[None, :]) @ U.conj().T
    zs = _cplx(rng, 40) * 2.0
    sig, sw = oracle.sigma_min_dense(C, zs)
    ref = np.min(np.abs(lam[None, :] - zs[:, None]), axis=1)
    normC = np.max(np.abs(lam))
    assert (sw > 0).all()
    assert np.max(np.abs(sig - ref)) <= 1e-12 * normC


def test_o1_normal_closed_form_rectangular():
    # C = P [diag(lam); 0] Q^* with P = diag(Q, Q2): P I_{m x n} Q^* = I_{m x n},
    # so sigma_min(C - z I) = min |lam_i - z|.
    rng = np.random.default_rng(12)
    n, extra = 20, 7
    m = n + extra
    lam = _cplx(rng, n)
    Q = _haar_unitary(rng, n)
    Q2 = _haar_unitary(rng, extra)
    P = np.zeros((m, m), dtype=complex)
    P[:n, :n] = Q
    P[n:, n:] = Q2
    D = np.zeros((m, n), dtype=complex)
    D[np.arange(n), np.arange(n)] = lam
    C = P @ D @ Q.conj().T
    zs = _cplx(rng, 30)
    sig, _ = oracle.sigma_min_dense(C, zs)
    ref = np.min(np.abs(lam[None, :] - zs[:, None]), axis=1)
    assert np.max(np.abs(sig - ref)) <= 1e-12 * np.max(np.abs(lam))


def test_o1_unitary_similarity_invariance():
    wl = workloads.triangular_disk(seed=5, n=40, grid=6)
    C = wl.dense
    rng = np.random.default_rng(5)
    Q = _haar_unitary(rng, 40)
    C2 = Q @ C @ Q.conj().T
    zs = oracle.grid_points(*wl.region, wl.nx, wl.ny)
    s1, _ = oracle.sigma_min_dense(C, zs)
    s2, _ = oracle.sigma_min_dense(C2, zs)
    normC = np.linalg.norm(C, 2)
    assert np.max(np.abs(s1 - s2)) <= 1e-12 * normC


def test_o1_one_lipschitz_over_grid():
    wl = workloads.triangular_disk(seed=6, n=30, grid=14)
    zs = oracle.grid_points(*wl.region, wl.nx, wl.ny)
    s, _ = oracle.sigma_min_dense(wl.dense, zs)
    S = s.reshape(wl.ny, wl.nx)
    Z = zs.reshape(wl.ny, wl.nx)
    normC = np.linalg.norm(wl.dense, 2)
    dx = np.abs(S[:, 1:] - S[:, :-1]) - np.abs(Z[:, 1:] - Z[:, :-1])
    dy = np.abs(S[1:, :] - S[:-1, :]) - np.abs(Z[1:, :] - Z[:-1, :])
    assert dx.max() <= 1e-12 * normC and dy.max() <= 1e-12 * normC
    # and the bound is not vacuous: some neighbours do differ
    assert np.abs(S[:, 1:] - S[:, :-1]).max() > 1e-3


def test_o1_brute_force_1x1_and_mx1():
    rng = np.random.default_rng(7)
    c = complex(_cplx(rng, 1)[0])
    zs = _cplx(rng, 10)
    s, _ = oracle.sigma_min_dense(np.array([[c]]), zs)
    assert np.allclose(s, np.abs(c - zs), rtol=0, atol=1e-15)
    col = _cplx(rng, 6).reshape(6, 1)
    s, _ = oracle.sigma_min_dense(col, zs)
    ref = [np.sqrt(abs(col[0, 0] - z) ** 2 + np.sum(np.abs(col[1:, 0]) ** 2)) for z in zs]
    assert np.allclose(s, ref, rtol=0, atol=1e-14)


def test_o1_brute_force_2x2_closed_form():
    rng = np.random.default_rng(8)
    for _ in range(20):
        C = _cplx(rng, 2, 2)
        z = complex(_cplx(rng, 1)[0])
        A = C - z * np.eye(2)
        det = abs(A[0, 0] * A[1, 1] - A[0, 1] * A[1, 0])
        F = np.sum(np.abs(A) ** 2)
        smax = np.sqrt((F + np.sqrt(max(F * F - 4 * det * det, 0.0))) / 2)
        ref = det / smax
        s, _ = oracle.sigma_min_dense(C, [z])
        assert abs(s[0] - ref) <= 1e-14 * smax


def test_o1_brute_force_3x3_sphere_search():
    rng = np.random.default_rng(9)
    C = _cplx(rng, 3, 3)
    z = 0.3 - 0.2j
    A = C - z * np.eye(3)
    # dense random sample of the unit sphere in C^3, then shrinking local search
    X = _cplx(rng, 3, 200000)
    X /= np.linalg.norm(X, axis=0, keepdims=True)
    vals = np.linalg.norm(A @ X, axis=0)
    x = X[:, np.argmin(vals)]
    best = vals.min()
    step = 0.1
    for _ in range(400):
        Y = x[:, None] + step * _cplx(rng, 3, 64)
        Y /= np.linalg.norm(Y, axis=0, keepdims=True)
        v = np.linalg.norm(A @ Y, axis=0)
        if v.min() < best:
            best = v.min(); x = Y[:, np.argmin(v)]
        else:
            step *= 0.8
    s, _ = oracle.sigma_min_dense(C, [z])
    assert s[0] <= best + 1e-14
    assert best - s[0] <= 1e-7 * np.linalg.norm(A, 2)


def test_o1_eigenvalue_bound_triangular():
    wl = workloads.triangular_disk(seed=10, n=40, grid=4)
    lam = wl.info["eigenvalues"]
    normC = np.linalg.norm(wl.dense, 2)
    s, _ = oracle.sigma_min_dense(wl.dense, lam[:8])
    assert np.all(s <= 1e-13 * normC)           # singular at an eigenvalue
    rng = np.random.default_rng(10)
    zs = _cplx(rng, 20) * 1.5
    s, _ = oracle.sigma_min_dense(wl.dense, zs)
    bound = np.min(np.abs(lam[None, :] - zs[:, None]), axis=1)
    assert np.all(s <= bound + 1e-13 * normC)


def test_o1_weyl_perturbation():
    wl = workloads.triangular_disk(seed=13, n=30, grid=3)
    rng = np.random.default_rng(13)
    E = _cplx(rng, 30, 30) * 1e-3
    nE = np.linalg.norm(E, 2)
    zs = oracle.grid_points(*wl.region, 5, 5)
    s1, _ = oracle.sigma_min_dense(wl.dense, zs)
    s2, _ = oracle.sigma_min_dense(wl.dense + E, zs)
    assert np.all(np.abs(s1 - s2) <= nE * (1 + 1e-12))


def test_jacobi_single_rotation_identities():
    rng = np.random.default_rng(14)
    ap = _cplx(rng, 12)
    aq = _cplx(rng, 12)
    a, b, c, t = oracle.jacobi_rotate(ap, aq)
    a2 = np.vdot(ap, ap).real
    b2 = np.vdot(aq, aq).real
    c2 = abs(np.vdot(ap, aq))
    assert abs(a2 - (a - t * c)) <= 1e-13 * (a + b)
    assert abs(b2 - (b + t * c)) <= 1e-13 * (a + b)
    assert c2 <= 1e-14 * np.sqrt(a * b) * 12


def test_membership_is_strict():
    s = np.array([0.1, 0.05, 0.2])
    mem = oracle.membership(s, [0.1])
    assert mem.tolist() == [[0, 1, 0]]


# ------------------------------------------------------------------ O2 ----

def _toeplitz_dense(t, lo, n, m=None):
    m = n if m is None else m
    C = np.zeros((m, n), dtype=complex)
    for d, val in enumerate(t):
        off = d - lo                     # column - row
        for i in range(m):
            j = i + off
            if 0 <= j < n:
                C[i, j] = val
    return C


def test_o2_matches_o1_square_banded():
    rng = np.random.default_rng(21)
    t = _cplx(rng, 5)
    C = _toeplitz_dense(t, 1, 60)
    band, kl, ku = oracle.band_from_dense(C)
    assert (kl, ku) == (1, 3)
    zs = _cplx(rng, 12) * 2
    s1, _ = oracle.sigma_min_dense(C, zs)
    s2 = oracle.sigma_min_banded(band, 60, 60, kl, ku, zs)
    assert np.max(np.abs(s1 - s2)) <= 1e-12 * np.linalg.norm(C, 2)


def test_o2_matches_o1_rectangular_folding_full_spectrum():
    wl = workloads.folding(seed=22, n=50, grid=4)
    C = wl.to_dense()
    band, kl, ku = oracle.band_from_csr(wl.m, wl.n, wl.rowptr, wl.colind, wl.vals)
    assert (kl, ku) == (4, 4)
    z = 0.25 + 0.4j
    A = C.copy()
    A[np.arange(wl.n), np.arange(wl.n)] -= z
    full = oracle.singular_values_dense(A)[::-1]
    got = oracle.banded_smallest(band, wl.m, wl.n, kl, ku, z, k=wl.n)
    assert np.max(np.abs(full - got)) <= 1e-12 * full[-1]


def test_o2_hermitian_tridiagonal_closed_form_large():
    # T = tridiag(conj(b), a, b) Hermitian Toeplitz: eigenvalues
    # a + 2|b| cos(k pi/(n+1)); T - zI is normal, so sigma_min = min_k |lam_k - z|.
    n = 3000
    a, b = 0.4, 0.7 - 0.3j
    band = np.zeros((n, 3), dtype=complex)
    band[:, 0] = np.conj(b)
    band[:, 1] = a
    band[:, 2] = b
    band[0, 0] = 0
    band[-1, 2] = 0
    lam = a + 2 * abs(b) * np.cos(np.arange(1, n + 1) * np.pi / (n + 1))
    zs = np.array([0.1 + 0.05j, 1.3 - 0.2j, 2.5 + 0j, -1.9 + 1e-3j])
    s = oracle.sigma_min_banded(band, n, n, 1, 1, zs)
    ref = np.min(np.abs(lam[None, :] - zs[:, None]), axis=1)
    assert np.max(np.abs(s - ref)) <= 1e-12 * (abs(a) + 2 * abs(b))


def test_o2_matches_lapack_on_config2_like_toeplitz():
    wl = workloads.toeplitz_band(seed=1002, n=700, grid=5)
    band, kl, ku = oracle.band_from_dense(wl.dense)
    zs = oracle.grid_points(*wl.region, 3, 3)
    s2 = oracle.sigma_min_banded(band, wl.n, wl.n, kl, ku, zs)
    ref = np.array([np.linalg.svd(wl.dense - z * np.eye(wl.n), compute_uv=False)[-1] for z in zs])
    assert np.max(np.abs(s2 - ref)) <= 1e-12 * np.linalg.norm(wl.dense, 2)


def test_o2_folding_monotone_in_n():
    # Nested foldings: the first n columns of C_{n'} are [C_n; 0], so
    # sigma_min(C_{n'} - z I) <= sigma_min(C_n - z I).
    zs = np.array([0.2 + 0.1j, -0.7 + 0.3j, 1.1 - 0.4j])
    prev = None
    for n in (40, 80, 160, 320):
        wl = workloads.folding(seed=23, n=n, grid=2)
        band, kl, ku = oracle.band_from_csr(wl.m, wl.n, wl.rowptr, wl.colind, wl.vals)
        s = oracle.sigma_min_banded(band, wl.m, wl.n, kl, ku, zs)
        if prev is not None:
            assert np.all(s <= prev + 1e-13)
        prev = s


def test_o2_diagonal_matrix():
    d = np.array([1.0, 2.0 + 1j, -0.5j, 3.0])
    band = d.reshape(4, 1).astype(complex)
    zs = np.array([0.9, 0.1j, 2.1 + 0.9j])
    s = oracle.sigma_min_banded(band, 4, 4, 0, 0, zs)
    ref = np.min(np.abs(d[None, :] - zs[:, None]), axis=1)
    assert np.allclose(s, ref, rtol=0, atol=1e-15)


def test_grid_points_inclusive_endpoints_and_order():
    # Reading of the paper's "equispaced Cartesian grid" (Sec. 4): both ends
    # of each side are grid points, and point (i, j) sits at index j * nx + i.
    # Pinned with hand-computed coordinates, not with the library's grid.
    zs = oracle.grid_points(-1.0, 3.0, 2.0, 5.0, 5, 4)
    assert zs.shape == (20,)
    want_x = [-1.0, 0.0, 1.0, 2.0, 3.0]
    want_y = [2.0, 3.0, 4.0, 5.0]
    for j in range(4):
        for i in range(5):
            assert zs[j * 5 + i] == complex(want_x[i], want_y[j])
    # a single point per side sits at the low end
    assert oracle.grid_points(0.5, 9.0, -2.0, 7.0, 1, 1)[0] == complex(0.5, -2.0)
    one_row = oracle.grid_points(0.0, 1.0, 3.0, 4.0, 3, 1)
    assert list(one_row) == [3j, 0.5 + 3j, 1.0 + 3j]


@pytest.mark.parametrize("N", [12, 20])
def test_sparse_lu_oracle_matches_o1(N):
    # O2 for square sparse C (banded LU + inverse subspace iteration) against
    # the dense Jacobi oracle on reduced convection-diffusion instances
    wl = workloads.convection_diffusion(N=N, grid=5)
    zs = oracle.grid_points(*wl.region, 5, 5)
    s2, steps = oracle.sigma_min_sparse_lu(wl.n, wl.n, wl.rowptr, wl.colind, wl.vals, zs)
    s1, sw = oracle.sigma_min_dense(wl.to_dense(), zs)
    nC = oracle.norm2_sparse(wl.n, wl.n, wl.rowptr, wl.colind, wl.vals)
    assert (sw > 0).all() and (steps >= 0).all()
    assert np.max(np.abs(s1 - s2)) <= 1e-12 * nC


def test_sparse_lu_oracle_normal_closed_form():
    # a sparse normal matrix: diagonal D (any bandwidth-0 C), sigma = min |d_i - z|
    rng = np.random.default_rng(5)
    n = 300
    d = _cplx(rng, n) * 2.0
    rowptr = np.arange(n + 1, dtype=np.int64)
    colind = np.arange(n, dtype=np.int32)
    zs = _cplx(rng, 12)
    s, steps = oracle.sigma_min_sparse_lu(n, n, rowptr, colind, d, zs)
    ref = np.min(np.abs(d[None, :] - zs[:, None]), axis=1)
    assert np.max(np.abs(s - ref)) <= 1e-12 * np.max(np.abs(d))


def test_norm2_sparse_matches_lapack():
    wl = workloads.convection_diffusion(N=15, grid=3)
    nC = oracle.norm2_sparse(wl.n, wl.n, wl.rowptr, wl.colind, wl.vals)
    assert abs(nC - np.linalg.norm(wl.to_dense(), 2)) <= 1e-8 * nC
