"""Seeded synthetic inputs for the pseudospectra workloads.

This module is the only one that both the oracle and the product path read.
It draws random matrices and lays out regions and grids; it holds none of
the method's arithmetic.  Every draw uses ``numpy.random.default_rng(seed)``
(PCG64) in the order written below, and CN(0,1) is the circular complex
Gaussian (N(0,1) + i N(0,1)) / sqrt(2), i.e. E|z|^2 = 1.

The paper's own test matrices (Sec. 4, Table 1) are not available here; the
workloads below stand in for them with the shapes, structure and
conditioning the paper describes (dense nonnormal Toeplitz in place of the
basor Toeplitz example, a convection-diffusion CSR matrix in place of the
large sparse nonnormal examples, rectangular banded foldings after the
rectangular definition of Sec. 1).
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence

import numpy as np

EPS_4 = (1e-1, 1e-2, 1e-3, 1e-4)
EPS_6 = (1e-1, 1e-2, 1e-3, 1e-4, 1e-5, 1e-6)


def cn(rng: np.random.Generator, size) -> np.ndarray:
    """CN(0,1) draws: real parts first, then imaginary parts."""
    re = rng.standard_normal(size)
    im = rng.standard_normal(size)
    return (re + 1j * im) / math.sqrt(2.0)


@dataclasses.dataclass
class Workload:
    """One pseudospectrum problem: a matrix, a region, a grid, eps levels."""
    name: str
    m: int
    n: int
    kind: str                       # "dense" or "csr"
    region: tuple                   # (re_lo, re_hi, im_lo, im_hi)
    nx: int
    ny: int
    eps: tuple
    dense: Optional[np.ndarray] = None      # complex128, Fortran order, m x n
    rowptr: Optional[np.ndarray] = None     # int64, m + 1
    colind: Optional[np.ndarray] = None     # int32, nnz
    vals: Optional[np.ndarray] = None       # complex128, nnz
    z_center: Optional[complex] = None      # region centre (base-preconditioner site)
    info: dict = dataclasses.field(default_factory=dict)

    @property
    def npts(self) -> int:
        return self.nx * self.ny

    def to_dense(self) -> np.ndarray:
        if self.dense is not None:
            return self.dense
        A = np.zeros((self.m, self.n), dtype=np.complex128, order="F")
        rows = np.repeat(np.arange(self.m), np.diff(self.rowptr))
        A[rows, self.colind] = self.vals
        return A


def _bbox_pad(lo_re, hi_re, lo_im, hi_im, frac=0.10):
    wr = hi_re - lo_re
    wi = hi_im - lo_im
    return (lo_re - frac * wr, hi_re + frac * wr, lo_im - frac * wi, hi_im + frac * wi)


def triangular_disk(seed: int = 1001, n: int = 100, grid: int = 50, eps=EPS_4,
                    name: str = "dense-triangular") -> Workload:
    """Dense n x n C = diag(lambda) + N, upper triangular.

    lambda_i = sqrt(u_i) exp(2 pi i v_i) with u, v ~ U[0,1) (uniform in the
    unit disk); N has CN(0,1)/sqrt(n) entries strictly above the diagonal.
    Draw order: u (n), v (n), then an n x n CN(0,1) block of which the strict
    upper triangle is kept.  Region [-2,2]^2, grid x grid points."""
    rng = np.random.default_rng(seed)
    u = rng.random(n)
    v = rng.random(n)
    lam = np.sqrt(u) * np.exp(2j * np.pi * v)
    N = np.triu(cn(rng, (n, n)), k=1) / math.sqrt(n)
    C = np.asfortranarray(np.diag(lam) + N)
    return Workload(name=name, m=n, n=n, kind="dense", region=(-2.0, 2.0, -2.0, 2.0),
                    nx=grid, ny=grid, eps=tuple(eps), dense=C, z_center=0j,
                    info={"eigenvalues": lam, "seed": seed})


def toeplitz_band(seed: int = 1002, n: int = 4000, grid: int = 200, eps=EPS_6,
                  name: str = "dense-toeplitz") -> Workload:
    """Dense n x n nonnormal banded Toeplitz C with C[i, j] = t_{j-i} for
    -1 <= j - i <= 3 (one sub- and three superdiagonals, upper Hessenberg),
    the five constants t_{-1}, t_0, ..., t_3 drawn from CN(0,1) in that order.
    Stored dense.  Region: bounding box of the numerical range W(C), i.e. the
    extreme eigenvalues of (C + C^*)/2 and of (C - C^*)/(2i), each side
    widened by 10% of that axis's extent."""
    from scipy.linalg import eig_banded
    rng = np.random.default_rng(seed)
    t = cn(rng, 5)                      # t[d + 1] = t_d, d = -1..3
    C = np.zeros((n, n), dtype=np.complex128, order="F")
    idx = np.arange(n)
    for d in range(-1, 4):
        i = idx[max(0, -d): n - max(0, d)]
        C[i, i + d] = t[d + 1]
    # Hermitian parts in upper band storage (bandwidth 3):
    # H = (C + C^*)/2 has H[i, i+d] = (t_d + conj(t_{-d}))/2.
    def herm_band(sign):
        ab = np.zeros((4, n), dtype=np.complex128)
        for d in range(0, 4):
            td = t[d + 1]
            tmd = t[-d + 1] if -d >= -1 else 0.0
            if sign > 0:
                val = (td + np.conj(tmd)) / 2.0
            else:
                val = (td - np.conj(tmd)) / 2j
            ab[3 - d, d:] = val
        return ab
    ext = []
    for sign in (+1, -1):
        ab = herm_band(sign)
        lo = eig_banded(ab, lower=False, eigvals_only=True, select="i", select_range=(0, 0))[0]
        hi = eig_banded(ab, lower=False, eigvals_only=True, select="i",
                        select_range=(n - 1, n - 1))[0]
        ext.append((lo, hi))
    region = _bbox_pad(ext[0][0], ext[0][1], ext[1][0], ext[1][1])
    zc = complex(0.5 * (region[0] + region[1]), 0.5 * (region[2] + region[3]))
    return Workload(name=name, m=n, n=n, kind="dense", region=region, nx=grid, ny=grid,
                    eps=tuple(eps), dense=C, z_center=zc,
                    info={"toeplitz": t, "kl": 1, "ku": 3, "seed": seed})


def convection_diffusion(seed: int = 1003, N: int = 500, grid: int = 100, eps=EPS_6,
                         peclet: float = 50.0, name: str = "csr-convdiff",
                         region_override: Optional[Sequence[float]] = None) -> Workload:
    """Sparse CSR C = diag(exp(i phi)) A, n = N^2.

    A is the centred 5-point convection-diffusion stencil on an N x N grid
    (natural ordering, index i + N j, Dirichlet boundary), scaled by h^2 with
    h = 1/(N+1): diagonal 4, west/south -1 - beta, east/north -1 + beta with
    beta = Pe h / (2 sqrt 2) for the wind (1, 1)/sqrt 2 and global Peclet
    number Pe.  phi_i ~ U[0, 2 pi) is drawn once per row.  Region:
    [rho - w, rho + w] x [-w, w] with w = 0.1 rho, rho the largest
    eigenvalue modulus (ARPACK, which='LM'); the grid is grid x grid."""
    rng = np.random.default_rng(seed)
    n = N * N
    h = 1.0 / (N + 1)
    beta = peclet * h / (2.0 * math.sqrt(2.0))
    phi = rng.random(n) * 2.0 * np.pi
    ph = np.exp(1j * phi)
    ii = np.arange(n) % N
    jj = np.arange(n) // N
    rows, cols, vals = [], [], []
    def add(mask, off, val):
        r = np.nonzero(mask)[0]
        rows.append(r)
        cols.append(r + off)
        vals.append(np.full(r.size, val, dtype=np.complex128))
    add(jj > 0, -N, -1.0 - beta)           # south
    add(ii > 0, -1, -1.0 - beta)           # west
    add(np.ones(n, bool), 0, 4.0)          # centre
    add(ii < N - 1, +1, -1.0 + beta)       # east
    add(jj < N - 1, +N, -1.0 + beta)       # north
    r = np.concatenate(rows)
    c = np.concatenate(cols)
    v = np.concatenate(vals)
    order = np.lexsort((c, r))
    r, c, v = r[order], c[order], v[order]
    v = v * ph[r]
    rowptr = np.zeros(n + 1, dtype=np.int64)
    np.add.at(rowptr, r + 1, 1)
    rowptr = np.cumsum(rowptr)
    wl = Workload(name=name, m=n, n=n, kind="csr", region=(0, 0, 0, 0), nx=grid, ny=grid,
                  eps=tuple(eps), rowptr=rowptr, colind=c.astype(np.int32),
                  vals=v.astype(np.complex128), info={"N": N, "beta": beta, "seed": seed})
    if region_override is not None:
        wl.region = tuple(float(x) for x in region_override)
    else:
        import scipy.sparse as sp
        import scipy.sparse.linalg as spla
        A = sp.csr_matrix((wl.vals, wl.colind, wl.rowptr), shape=(n, n))
        lam = spla.eigs(A, k=1, which="LM", return_eigenvectors=False,
                        v0=np.ones(n, dtype=np.complex128), tol=1e-8)
        rho = float(np.abs(lam[0]))
        w = 0.1 * rho
        wl.region = (rho - w, rho + w, -w, w)
        wl.info["rho"] = rho
    wl.z_center = complex(0.5 * (wl.region[0] + wl.region[1]), 0.5 * (wl.region[2] + wl.region[3]))
    return wl


def folding(seed: int, n: int, grid: int = 64, eps=EPS_6, bw: int = 4,
            name: str = "csr-folding") -> Workload:
    """Rectangular banded folding: m = n + bw rows, entry (row j, col k) =
    a_{j-k} for |j - k| <= bw, with the 2 bw + 1 Toeplitz constants
    a_{-bw}..a_{bw} ~ CN(0,1) drawn in that order: the section of rows
    0..n+bw-1 and columns 0..n-1 of the banded Toeplitz matrix, so that every
    column from bw on holds its 2 bw + 1 entries and the first bw columns lose
    the ones above row 0.
    Region: bounding box of the symbol curve sum_d a_d e^{i d theta},
    widened by 10% per axis.  Stored CSR."""
    rng = np.random.default_rng(seed)
    a = cn(rng, 2 * bw + 1)                # a[d + bw] = a_d
    m = n + bw
    rows, cols, vals = [], [], []
    for d in range(-bw, bw + 1):
        k = np.arange(n)
        j = k + d
        ok = (j >= 0) & (j < m)
        rows.append(j[ok]); cols.append(k[ok]); vals.append(np.full(ok.sum(), a[d + bw]))
    r = np.concatenate(rows); c = np.concatenate(cols); v = np.concatenate(vals)
    order = np.lexsort((c, r))
    r, c, v = r[order], c[order], v[order]
    rowptr = np.zeros(m + 1, dtype=np.int64)
    np.add.at(rowptr, r + 1, 1)
    rowptr = np.cumsum(rowptr)
    th = np.linspace(0, 2 * np.pi, 4096, endpoint=False)
    sym = sum(a[d + bw] * np.exp(1j * d * th) for d in range(-bw, bw + 1))
    region = _bbox_pad(sym.real.min(), sym.real.max(), sym.imag.min(), sym.imag.max())
    zc = complex(0.5 * (region[0] + region[1]), 0.5 * (region[2] + region[3]))
    return Workload(name=name, m=m, n=n, kind="csr", region=region, nx=grid, ny=grid,
                    eps=tuple(eps), rowptr=rowptr, colind=c.astype(np.int32),
                    vals=v.astype(np.complex128), z_center=zc,
                    info={"toeplitz": a, "bw": bw, "seed": seed})


def batched_uneven(seed: int = 1004, n_dense: int = 192, n_fold: int = 64, grid: int = 64,
                   dense_range=(64, 1024), fold_range=(1000, 20000)) -> List[Workload]:
    """Many matrices of uneven size in one batch: n_dense dense triangular
    matrices (as ``triangular_disk``) with n ~ U{dense_range}, and n_fold
    rectangular foldings with n ~ U{fold_range}; each on a grid x grid grid.
    Sizes are drawn first (dense sizes, then folding sizes), then every
    matrix uses its own seed 10 * seed + index."""
    rng = np.random.default_rng(seed)
    nd = rng.integers(dense_range[0], dense_range[1] + 1, size=n_dense)
    nf = rng.integers(fold_range[0], fold_range[1] + 1, size=n_fold)
    out = []
    for i, n in enumerate(nd):
        out.append(triangular_disk(seed=10 * seed + i, n=int(n), grid=grid, eps=EPS_6,
                                   name="dense-%d" % i))
    for i, n in enumerate(nf):
        out.append(folding(seed=10 * seed + n_dense + i, n=int(n), grid=grid,
                           name="fold-%d" % i))
    return out


def grid_coords(wl: Workload):
    """(xs, ys) of the grid, both ends included (linspace)."""
    re_lo, re_hi, im_lo, im_hi = wl.region
    xs = np.linspace(re_lo, re_hi, wl.nx) if wl.nx > 1 else np.array([re_lo])
    ys = np.linspace(im_lo, im_hi, wl.ny) if wl.ny > 1 else np.array([im_lo])
    return xs, ys


def sample_indices(npts: int, k: int, seed: int) -> np.ndarray:
    """k distinct grid indices drawn uniformly by seed (sorted)."""
    rng = np.random.default_rng(seed)
    k = min(k, npts)
    return np.sort(rng.choice(npts, size=k, replace=False))


WORKLOADS = {
    "dense-triangular-n100": lambda: triangular_disk(),
    "dense-toeplitz-n4000": lambda: toeplitz_band(),
    "csr-convdiff-n250000": lambda: convection_diffusion(),
}


def serving_requests(seed: int = 1005, n_req: int = 512, dense_range=(256, 4096), sparse_N_range=(100, 447),
                     grid_range=(32, 128), eps=EPS_6) -> List[Workload]:
    """A stream of pseudospectrum requests: each one dense (as
    ``triangular_disk``, n ~ U{dense_range}, region [-2,2]^2) with probability
    1/2, else sparse (as ``convection_diffusion``, N ~ U{sparse_N_range}, n =
    N^2, region near its spectral boundary); grid side s ~ U{grid_range}.
    Per request i the draws, in order, are: kind (u < 1/2 is dense), size,
    grid side; request i's matrix then uses seed 10 * seed + i."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n_req):
        dense = rng.random() < 0.5
        size = int(rng.integers(dense_range[0], dense_range[1] + 1)) if dense else \
            int(rng.integers(sparse_N_range[0], sparse_N_range[1] + 1))
        s = int(rng.integers(grid_range[0], grid_range[1] + 1))
        if dense:
            out.append(triangular_disk(seed=10 * seed + i, n=size, grid=s, eps=eps, name="req-%d-dense" % i))
        else:
            out.append(convection_diffusion(seed=10 * seed + i, N=size, grid=s, eps=eps,
                                            name="req-%d-convdiff" % i))
    return out
