"""Oracle for sigma_min(C - zI) over a grid of points.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and
the CPU-baseline leg of ``bench.py`` may import this package.  The product
library neither imports nor links it; the two share no code.  The only module
both sides read is ``workloads`` (seeded input generators, which hold none of
the method's arithmetic).

The oracle is the plain definition of the epsilon-pseudospectrum (paper,
Sec. 1, eqs. (defSquare) and (defSquareSVD)): sigma(z) is the smallest
singular value of A = C - z I, with I the m x n matrix [I_n; 0] when C is
rectangular (m >= n), and z belongs to the epsilon-pseudospectrum exactly
when sigma(z) < epsilon (strict).

Two independent plain methods, both in ``ps_oracle.c``:

* O1 ``sigma_min_dense``: dense one-sided Jacobi SVD of A at every point
  (Hestenes 1958; Demmel & Veselic 1992), one point per OpenMP thread.
* O2 ``sigma_min_banded``: for banded C, Givens QR to an upper band, Givens
  bulge chasing to bidiagonal form, and Sturm bisection on the Golub-Kahan
  tridiagonal.  Used where O1's O(m n^2) per point is out of reach
  (n = 4000 and above); checked against O1 where both run.

Grid convention (the paper only says "equispaced Cartesian grid", Sec. 4):
both ends included, like ``linspace``; point (i, j) has index j * nx + i.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ps_oracle.c")
_LIB = os.path.join(_HERE, "_libpsoracle.so")
_lock = threading.Lock()
_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle's C source with gcc and OpenMP; returns the path."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-fopenmp", "-fPIC", "-shared",
                               _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
                build(force=True)
            lib = ctypes.CDLL(_LIB)
            P = ctypes.c_void_p
            I64 = ctypes.c_int64
            lib.oracle_sigma_min_dense.argtypes = [P, I64, I64, I64, P, P, I64, ctypes.c_int, P, P]
            lib.oracle_sigma_min_dense.restype = ctypes.c_int
            lib.oracle_singular_values_dense.argtypes = [P, I64, I64, I64, P, ctypes.c_int]
            lib.oracle_singular_values_dense.restype = ctypes.c_int
            lib.oracle_banded_smallest.argtypes = [P, I64, I64, ctypes.c_int, ctypes.c_int,
                                                   ctypes.c_double, ctypes.c_double, I64, P]
            lib.oracle_banded_smallest.restype = ctypes.c_int
            lib.oracle_sigma_min_banded.argtypes = [P, I64, I64, ctypes.c_int, ctypes.c_int,
                                                    P, P, I64, P]
            lib.oracle_sigma_min_banded.restype = ctypes.c_int
            lib.oracle_jacobi_rotate.argtypes = [P, P, I64, ctypes.c_double, ctypes.c_double,
                                                 ctypes.c_double, ctypes.c_double, P]
            lib.oracle_jacobi_rotate.restype = None
            lib.oracle_num_threads.restype = ctypes.c_int
            _lib = lib
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def num_threads() -> int:
    """OpenMP threads the oracle uses (OMP_NUM_THREADS, else all cores)."""
    return int(_load().oracle_num_threads())


def grid_points(re_lo, re_hi, im_lo, im_hi, nx, ny) -> np.ndarray:
    """Grid points z[j * nx + i] = x_i + 1j * y_j with both ends included."""
    xs = np.linspace(re_lo, re_hi, nx) if nx > 1 else np.array([float(re_lo)])
    ys = np.linspace(im_lo, im_hi, ny) if ny > 1 else np.array([float(im_lo)])
    return (xs[None, :] + 1j * ys[:, None]).reshape(-1)


def singular_values_dense(A: np.ndarray, max_sweeps: int = 60) -> np.ndarray:
    """All singular values, descending, of a dense complex matrix by O1."""
    A = np.asfortranarray(np.asarray(A, dtype=np.complex128))
    m, n = A.shape
    sv = np.empty(n, dtype=np.float64)
    rc = _load().oracle_singular_values_dense(_ptr(A), m, n, m, _ptr(sv), max_sweeps)
    if rc == -2:
        raise MemoryError("oracle: out of memory")
    if rc < 0:
        raise RuntimeError("oracle O1: Jacobi did not converge in %d sweeps" % max_sweeps)
    return sv


def sigma_min_dense(C: np.ndarray, zs, max_sweeps: int = 40):
    """O1: sigma_min(C - z I_{m x n}) at each z; returns (sigma, sweeps).

    sweeps[k] == -1 flags a point whose Jacobi hit the sweep cap."""
    C = np.asfortranarray(np.asarray(C, dtype=np.complex128))
    m, n = C.shape
    if m < n:
        raise ValueError("oracle: need m >= n")
    zs = np.ascontiguousarray(np.asarray(zs, dtype=np.complex128).reshape(-1))
    zr = np.ascontiguousarray(zs.real)
    zi = np.ascontiguousarray(zs.imag)
    sigma = np.empty(zs.size, dtype=np.float64)
    sweeps = np.empty(zs.size, dtype=np.int32)
    rc = _load().oracle_sigma_min_dense(_ptr(C), m, n, m, _ptr(zr), _ptr(zi), zs.size,
                                        max_sweeps, _ptr(sigma), _ptr(sweeps))
    if rc != 0:
        raise MemoryError("oracle: out of memory")
    return sigma, sweeps


def band_from_dense(C: np.ndarray):
    """Band storage (m x (kl+ku+1), row-major) of a dense matrix, with its
    lower and upper bandwidths found from the nonzero pattern."""
    C = np.asarray(C, dtype=np.complex128)
    m, n = C.shape
    rows, cols = np.nonzero(C)
    if rows.size == 0:
        kl = ku = 0
    else:
        off = cols - rows
        kl = int(max(0, -off.min()))
        ku = int(max(0, off.max()))
    w = kl + ku + 1
    band = np.zeros((m, w), dtype=np.complex128)
    band[rows, cols - rows + kl] = C[rows, cols]
    return band, kl, ku


def band_from_csr(m: int, n: int, rowptr, colind, vals):
    """Band storage of a CSR matrix (same convention as band_from_dense)."""
    rowptr = np.asarray(rowptr, dtype=np.int64)
    colind = np.asarray(colind, dtype=np.int64)
    vals = np.asarray(vals, dtype=np.complex128)
    rows = np.repeat(np.arange(m, dtype=np.int64), np.diff(rowptr))
    off = colind - rows
    kl = int(max(0, -off.min())) if off.size else 0
    ku = int(max(0, off.max())) if off.size else 0
    band = np.zeros((m, kl + ku + 1), dtype=np.complex128)
    np.add.at(band, (rows, off + kl), vals)
    return band, kl, ku


def banded_smallest(band: np.ndarray, m: int, n: int, kl: int, ku: int, z: complex, k: int = 1):
    """O2: the k smallest singular values (ascending) of C - z I_{m x n}."""
    band = np.ascontiguousarray(band, dtype=np.complex128)
    assert band.shape == (m, kl + ku + 1)
    out = np.empty(k, dtype=np.float64)
    rc = _load().oracle_banded_smallest(_ptr(band), m, n, kl, ku, float(np.real(z)),
                                        float(np.imag(z)), k, _ptr(out))
    if rc != 0:
        raise RuntimeError("oracle O2: rc=%d" % rc)
    return out


def sigma_min_banded(band: np.ndarray, m: int, n: int, kl: int, ku: int, zs) -> np.ndarray:
    """O2 over many points: sigma_min(C - z I_{m x n}) for banded C."""
    band = np.ascontiguousarray(band, dtype=np.complex128)
    assert band.shape == (m, kl + ku + 1)
    zs = np.asarray(zs, dtype=np.complex128).reshape(-1)
    zr = np.ascontiguousarray(zs.real)
    zi = np.ascontiguousarray(zs.imag)
    sigma = np.empty(zs.size, dtype=np.float64)
    rc = _load().oracle_sigma_min_banded(_ptr(band), m, n, kl, ku, _ptr(zr), _ptr(zi),
                                         zs.size, _ptr(sigma))
    if rc != 0:
        raise RuntimeError("oracle O2: rc=%d" % rc)
    return sigma


def jacobi_rotate(ap: np.ndarray, aq: np.ndarray):
    """One O1 rotation of a column pair in place; returns (a, b, |c|, t) of
    the pair before the rotation.  Exposed so that a test can check the
    2x2 update a' = a - t|c|, b' = b + t|c| and the annihilated Gram entry."""
    assert ap.dtype == np.complex128 and aq.dtype == np.complex128
    a = float(np.vdot(ap, ap).real)
    b = float(np.vdot(aq, aq).real)
    c = complex(np.vdot(ap, aq))
    t = np.zeros(1)
    _load().oracle_jacobi_rotate(_ptr(ap), _ptr(aq), ap.size, a, b, c.real, c.imag, _ptr(t))
    return a, b, abs(c), float(t[0])


def membership(sigma: np.ndarray, eps_levels) -> np.ndarray:
    """member[e, k] = sigma[k] < eps_e (strict, eq. (defSquareSVD))."""
    eps = np.asarray(eps_levels, dtype=np.float64).reshape(-1, 1)
    return (np.asarray(sigma)[None, :] < eps).astype(np.uint8)


def norm2_sparse(m: int, n: int, rowptr, colind, vals, rel: float = 1e-12, seed: int = 7) -> float:
    """||C||_2 = sigma_max(C) of a CSR matrix: the largest eigenvalue of the
    Hermitian C^* C by ARPACK's implicitly restarted Lanczos (scipy eigsh,
    relative tolerance rel, seeded start vector), square-rooted."""
    import scipy.sparse as sp
    import scipy.sparse.linalg as spla
    A = sp.csr_matrix((np.asarray(vals, dtype=np.complex128), np.asarray(colind), np.asarray(rowptr)),
                      shape=(m, n))
    AH = A.conj().T.tocsr()
    op = spla.LinearOperator((n, n), matvec=lambda x: AH @ (A @ x), dtype=np.complex128)
    rng = np.random.default_rng(seed)
    v0 = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    lam = spla.eigsh(op, k=1, which="LA", v0=v0, tol=rel, return_eigenvectors=False, ncv=min(n, 40))
    return float(np.sqrt(lam[0]))


def sigma_min_sparse_lu(m: int, n: int, rowptr, colind, vals, zs, block: int = 8, tol_rel: float = 1e-14,
                        max_iter: int = 200, seed: int = 11, normC: float | None = None):
    """O2 for square sparse C of bandwidth b: sigma_min(C - z I) by block
    inverse subspace iteration on (A^* A)^{-1}, A = C - z I, with A factored
    once per point by LAPACK's banded LU with partial pivoting (zgbtrf).
    Each step: Y = A^{-1} (A^{-*} X), Q = qr(Y), Rayleigh-Ritz by the SVD of
    the n x block product A Q (its smallest singular value is a Ritz value,
    an upper bound of sigma_min), X = Q V.  Stops when the smallest Ritz value
    changes by at most tol_rel ||C|| between steps.  Returns (sigma, steps);
    steps = -1 marks a point that hit max_iter."""
    import scipy.sparse as sp
    from scipy.linalg import lapack
    if m != n:
        raise ValueError("sigma_min_sparse_lu: square C only")
    A0 = sp.csr_matrix((np.asarray(vals, dtype=np.complex128), np.asarray(colind), np.asarray(rowptr)),
                       shape=(m, n)).tocoo()
    off = A0.col.astype(np.int64) - A0.row.astype(np.int64)
    kl = int(max(0, -off.min())) if off.size else 0
    ku = int(max(0, off.max())) if off.size else 0
    if normC is None:
        normC = norm2_sparse(m, n, rowptr, colind, vals)
    zs = np.asarray(zs, dtype=np.complex128).reshape(-1)
    out = np.empty(zs.size)
    steps = np.empty(zs.size, dtype=np.int64)
    rng = np.random.default_rng(seed)
    X0 = rng.standard_normal((n, block)) + 1j * rng.standard_normal((n, block))
    X0, _ = np.linalg.qr(X0)
    Acsr = sp.csr_matrix((np.asarray(vals, dtype=np.complex128), np.asarray(colind), np.asarray(rowptr)),
                         shape=(m, n))
    eye = sp.identity(n, dtype=np.complex128, format="csr")
    for q, z in enumerate(zs):
        Az = (Acsr - z * eye).tocoo()
        ab = np.zeros((2 * kl + ku + 1, n), dtype=np.complex128, order="F")
        ab[kl + ku + Az.row - Az.col, Az.col] = Az.data
        lu, piv, info = lapack.zgbtrf(ab, kl, ku)
        if info != 0:
            raise RuntimeError("oracle O2: zgbtrf info=%d" % info)
        Azcsr = Az.tocsr()
        X = X0.copy()
        prev = np.inf
        sig = np.inf
        for it in range(max_iter):
            W, info1 = lapack.zgbtrs(lu, kl, ku, X, piv, trans=2)
            Y, info2 = lapack.zgbtrs(lu, kl, ku, W, piv, trans=0)
            if info1 or info2:
                raise RuntimeError("oracle O2: zgbtrs failed")
            Q, _ = np.linalg.qr(Y)
            B = Azcsr @ Q
            _, s, Vh = np.linalg.svd(B, full_matrices=False)
            X = Q @ Vh.conj().T[:, ::-1]
            sig = float(s[-1])
            if abs(prev - sig) <= tol_rel * normC:
                break
            prev = sig
        else:
            it = -1
        out[q] = sig
        steps[q] = it if it >= 0 else -1
    return out, steps
