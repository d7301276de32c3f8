"""Python binding of the MI355X pseudospectra library (libps.so).

Argument marshalling only: every step of the computation runs in the HIP
kernels of ``libps.so``.  The names follow the C ABI in ``include/ps.h``:
``ps_create``, ``ps_grid``, ``ps_eval``, ``ps_destroy``.  Importing this
package never builds anything; ``build.build()`` (or
``__graft_entry__.build()``) compiles the library.  If ``libps.so`` is missing
the functions raise: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import math
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libps.so")

PS_OK = 0
PS_WARN_UNCERTIFIED = 1
PS_DENSE = 0
PS_CSR = 1
FLAG_ACCEPTED = 1
FLAG_REFINED = 2
FLAG_UNCERTIFIED = 4
FLAG_PROJ_REFINED = 8
FLAG_REBUILD = 16
FLAG_CERTIFIED = 32
FLAG_LIPSCHITZ = 64
NCLASS = 9          # PS_NCLASS: event-timed kernel classes in ps_stats


class ps_matrix_desc(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("m", ctypes.c_int64), ("n", ctypes.c_int64),
                ("dense", ctypes.c_void_p), ("ld", ctypes.c_int64),
                ("rowptr", ctypes.c_void_p), ("colind", ctypes.c_void_p), ("vals", ctypes.c_void_p),
                ("nnz", ctypes.c_int64), ("on_device", ctypes.c_int32)]


class ps_params(ctypes.Structure):
    _fields_ = [("r", ctypes.c_int32), ("k_max", ctypes.c_int32), ("rbar", ctypes.c_int32),
                ("kbar_max", ctypes.c_int32), ("max_iters", ctypes.c_int32), ("precond", ctypes.c_int32),
                ("tiles_x", ctypes.c_int32), ("tiles_y", ctypes.c_int32), ("tile_points", ctypes.c_int32),
                ("tile_mem_gb", ctypes.c_int32), ("site_mem_gb", ctypes.c_int32), ("batch", ctypes.c_int32),
                ("traversal", ctypes.c_int32),
                ("recycle", ctypes.c_int32), ("eta", ctypes.c_double), ("eta_svd", ctypes.c_double),
                ("eta_proj", ctypes.c_double), ("omega", ctypes.c_double), ("tau_min", ctypes.c_double),
                ("tau_max", ctypes.c_double), ("zdag_re", ctypes.c_double), ("zdag_im", ctypes.c_double),
                ("seed", ctypes.c_uint64), ("eta_abs", ctypes.c_double), ("rho_small", ctypes.c_double),
                ("profile", ctypes.c_int32),
                ("verbose", ctypes.c_int32), ("tol_abs", ctypes.c_double), ("esc_iters", ctypes.c_int32),
                ("cert_recycled", ctypes.c_int32), ("reg_base", ctypes.c_double), ("lipschitz", ctypes.c_int32),
                ("fact_blas", ctypes.c_int32)]


class ps_stats(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int64) for n in (
        "points", "accepted", "refined", "uncertified", "lobpcg_iters", "proj_accepted",
        "proj_refined", "proj_iters", "rebuilds", "mv_M", "sv_F", "rounds", "certified", "lipschitz_redo",
        "guard_rejects", "cert_tests", "builds_shared", "builds_private", "ritz_jobs", "store_updates",
        "precond_iters", "repairs", "mv_update", "ic_retries")] + \
        [(n, ctypes.c_double) for n in ("t_total_ms", "t_ritz_ms", "t_lobpcg_ms", "t_update_ms",
                                        "t_precond_ms")] + \
        [("k_launches", ctypes.c_int64 * NCLASS), ("k_ms", ctypes.c_double * NCLASS),
         ("k_flops", ctypes.c_double * NCLASS), ("k_bytes", ctypes.c_double * NCLASS)]

    def as_dict(self):
        out = {}
        for name, _ in self._fields_:
            v = getattr(self, name)
            out[name] = list(v) if name.startswith("k_") else v
        return out


_lib = None


def load():
    """Load libps.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError("libps.so not built: run paper_2606_26785_amd/build.py (no CPU fallback)")
    lib = ctypes.CDLL(LIB_PATH)
    P = ctypes.c_void_p
    lib.ps_default_params.argtypes = [ctypes.POINTER(ps_params)]
    lib.ps_default_params.restype = None
    lib.ps_create.argtypes = [ctypes.POINTER(ps_matrix_desc), ctypes.POINTER(ps_params), P,
                              ctypes.POINTER(P)]
    lib.ps_create.restype = ctypes.c_int
    lib.ps_grid.argtypes = [ctypes.c_double] * 4 + [ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(P)]
    lib.ps_grid.restype = ctypes.c_int
    lib.ps_eval.argtypes = [P, P, P, ctypes.c_int32, P, P, P, ctypes.POINTER(ps_stats)]
    lib.ps_eval.restype = ctypes.c_int
    lib.ps_grid_destroy.argtypes = [P]
    lib.ps_grid_destroy.restype = None
    lib.ps_destroy.argtypes = [P]
    lib.ps_destroy.restype = None
    lib.ps_strerror.argtypes = [ctypes.c_int]
    lib.ps_strerror.restype = ctypes.c_char_p
    lib.ps_last_error.argtypes = []
    lib.ps_last_error.restype = ctypes.c_char_p
    lib.ps_debug_apply.argtypes = [P, ctypes.c_int32, ctypes.c_double, ctypes.c_double, P, ctypes.c_int32, P]
    lib.ps_debug_apply.restype = ctypes.c_int
    lib.ps_debug_precond.argtypes = [P, ctypes.c_double, ctypes.c_double, P, P]
    lib.ps_debug_precond.restype = ctypes.c_int
    lib.ps_debug_twolevel.argtypes = [P] + [ctypes.c_double] * 4 + [P, P, P, P, P]
    lib.ps_debug_twolevel.restype = ctypes.c_int
    lib.ps_debug_site.argtypes = [P, P, P]
    lib.ps_debug_site.restype = ctypes.c_int
    lib.ps_debug_store.argtypes = [P, ctypes.c_int32, P, P, P, P, P, P, P]
    lib.ps_debug_store.restype = ctypes.c_int
    lib.ps_debug_ritz.argtypes = [P, ctypes.c_int32, ctypes.c_double, ctypes.c_double, P, P, P]
    lib.ps_debug_ritz.restype = ctypes.c_int
    lib.ps_apply_noalloc.argtypes = [P, ctypes.c_int32, ctypes.c_double, ctypes.c_double, P, ctypes.c_int64,
                                     ctypes.c_int32, P, ctypes.c_int64]
    lib.ps_apply_noalloc.restype = ctypes.c_int
    lib.ps_debug_order.argtypes = [ctypes.c_int32] * 6 + [P, P]
    lib.ps_debug_order.restype = ctypes.c_int
    lib.ps_debug_sparse_site.argtypes = [P, ctypes.c_double, ctypes.c_double, ctypes.c_int32, P, ctypes.c_int32,
                                         P, P]
    lib.ps_debug_sparse_site.restype = ctypes.c_int
    lib.ps_debug_inertia.argtypes = [P, ctypes.c_double, ctypes.c_double, ctypes.c_double, P]
    lib.ps_debug_inertia.restype = ctypes.c_int
    lib.ps_debug_norm.argtypes = [P]
    lib.ps_debug_norm.restype = ctypes.c_double
    _lib = lib
    return lib


class PSError(RuntimeError):
    def __init__(self, status, where):
        lib = load()
        msg = "%s: %s (%s)" % (where, lib.ps_strerror(status).decode(), lib.ps_last_error().decode())
        super().__init__(msg)
        self.status = status


def _check(status, where):
    if status < 0:
        raise PSError(status, where)
    return status


def default_params(**overrides) -> ps_params:
    p = ps_params()
    load().ps_default_params(ctypes.byref(p))
    for k, v in overrides.items():
        if not hasattr(p, k):
            raise KeyError(k)
        setattr(p, k, v)
    return p


class Matrix:
    """A ps_matrix handle (owns the device copy of C and the solver state)."""

    def __init__(self, handle, keep):
        self.handle = handle
        self._keep = keep

    def close(self):
        if self.handle:
            load().ps_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def norm_estimate(self) -> float:
        return float(load().ps_debug_norm(self.handle))


class Grid:
    def __init__(self, handle, nx, ny):
        self.handle = handle
        self.nx = nx
        self.ny = ny

    def close(self):
        if self.handle:
            load().ps_grid_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _ptr(a):
    return ctypes.c_void_p(a.ctypes.data) if isinstance(a, np.ndarray) else ctypes.c_void_p(a.data_ptr())


def ps_create(dense=None, csr=None, m=None, n=None, params: ps_params | None = None, stream=None) -> Matrix:
    """Create a handle from a dense complex matrix (host numpy array, any
    order) or a CSR triple (rowptr int64, colind int32, vals complex128)."""
    lib = load()
    d = ps_matrix_desc()
    keep = []
    if dense is not None:
        A = np.asfortranarray(np.asarray(dense), dtype=np.complex128)
        keep.append(A)
        d.kind = PS_DENSE
        d.m, d.n = A.shape
        d.ld = A.shape[0]
        d.dense = _ptr(A)
        d.on_device = 0
    else:
        rowptr, colind, vals = csr
        rowptr = np.ascontiguousarray(rowptr, dtype=np.int64)
        colind = np.ascontiguousarray(colind, dtype=np.int32)
        vals = np.ascontiguousarray(vals, dtype=np.complex128)
        keep += [rowptr, colind, vals]
        d.kind = PS_CSR
        d.m = int(m)
        d.n = int(n)
        d.rowptr = _ptr(rowptr)
        d.colind = _ptr(colind)
        d.vals = _ptr(vals)
        d.nnz = int(vals.size)
        d.on_device = 0
    h = ctypes.c_void_p()
    s = ctypes.c_void_p(stream) if stream is not None else ctypes.c_void_p(0)
    _check(lib.ps_create(ctypes.byref(d), ctypes.byref(params) if params is not None else None, s,
                         ctypes.byref(h)), "ps_create")
    mat = Matrix(h, keep)
    mat.shape = (int(d.m), int(d.n))
    return mat


def ps_grid(re_lo, re_hi, im_lo, im_hi, nx, ny) -> Grid:
    h = ctypes.c_void_p()
    _check(load().ps_grid(float(re_lo), float(re_hi), float(im_lo), float(im_hi), int(nx), int(ny),
                          ctypes.byref(h)), "ps_grid")
    return Grid(h, int(nx), int(ny))


@dataclass
class EvalResult:
    sigma: np.ndarray        # (ny, nx) flattened as j * nx + i
    member: np.ndarray       # (n_eps, npts) uint8
    flags: np.ndarray        # npts uint8
    stats: dict
    status: int


def ps_eval(mat: Matrix, grid: Grid, eps=()) -> EvalResult:
    lib = load()
    npts = grid.nx * grid.ny
    eps = np.ascontiguousarray(np.asarray(eps, dtype=np.float64).reshape(-1))
    sigma = np.empty(npts, dtype=np.float64)
    member = np.empty((max(eps.size, 1), npts), dtype=np.uint8)
    flags = np.empty(npts, dtype=np.uint8)
    st = ps_stats()
    status = lib.ps_eval(mat.handle, grid.handle, _ptr(eps) if eps.size else None, int(eps.size),
                         _ptr(sigma), _ptr(member), _ptr(flags), ctypes.byref(st))
    _check(status, "ps_eval")
    return EvalResult(sigma, member[:eps.size], flags, st.as_dict(), status)


def ps_destroy(mat: Matrix):
    mat.close()


def debug_apply(mat: Matrix, X: np.ndarray, z: complex = 0j, herm: bool = False) -> np.ndarray:
    """Y = C(z) X (herm False) or C(z)^* X (herm True) on the device (test hook)."""
    X = np.asfortranarray(X, dtype=np.complex128)
    w = X.shape[1]
    m, n = mat.shape
    Y = np.empty((n if herm else m, w), dtype=np.complex128, order="F")
    _check(load().ps_debug_apply(mat.handle, int(herm), float(np.real(z)), float(np.imag(z)), _ptr(X), w,
                                 _ptr(Y)), "ps_debug_apply")
    return Y


def apply_noalloc(mat: Matrix, X_ptr: int, ldx: int, w: int, Y_ptr: int, ldy: int, z: complex = 0j,
                  herm: bool = False) -> None:
    """Y = C(z) X or C(z)^* X on device arrays (integer device addresses,
    column-major, leading dimensions in complex elements); only enqueues the
    work on the handle's stream and allocates nothing."""
    _check(load().ps_apply_noalloc(mat.handle, int(herm), float(np.real(z)), float(np.imag(z)),
                                   ctypes.c_void_p(int(X_ptr)), int(ldx), int(w), ctypes.c_void_p(int(Y_ptr)),
                                   int(ldy)), "ps_apply_noalloc")


def debug_sparse_site(mat: Matrix, z: complex, X: np.ndarray, trans: int = 0):
    """(Y, alpha): Y = F^{-1} X (trans 0) or F^{-*} X (trans 1) for the
    sparse base site built at z (test hook)."""
    X = np.asfortranarray(X, dtype=np.complex128)
    Y = np.empty_like(X)
    a = np.zeros(1)
    _check(load().ps_debug_sparse_site(mat.handle, float(np.real(z)), float(np.imag(z)), int(trans), _ptr(X),
                                       X.shape[1], _ptr(Y), _ptr(a)), "ps_debug_sparse_site")
    return Y, float(a[0])


def debug_inertia(mat: Matrix, z: complex, mu: float) -> bool:
    """True when N(z) - mu I is positive definite by the library's inertia
    test (test hook)."""
    pd = np.zeros(1, dtype=np.int32)
    _check(load().ps_debug_inertia(mat.handle, float(np.real(z)), float(np.imag(z)), float(mu), _ptr(pd)),
           "ps_debug_inertia")
    return bool(pd[0])


def debug_order(nx: int, ny: int, tx: int, ty: int, b: int, traversal: int):
    """Traversal plan (host only): list of per-tile arrays of point indices."""
    order = np.empty(nx * ny, dtype=np.int32)
    start = np.empty(tx * ty + 1, dtype=np.int32)
    _check(load().ps_debug_order(nx, ny, tx, ty, b, traversal, _ptr(order), _ptr(start)), "ps_debug_order")
    return [order[start[t]:start[t + 1]] for t in range(tx * ty)]


def create_from_workload(wl, params: ps_params | None = None, stream=None) -> Matrix:
    """Handle for a ``workloads.Workload``."""
    if wl.kind == "dense":
        return ps_create(dense=wl.dense, params=params, stream=stream)
    return ps_create(csr=(wl.rowptr, wl.colind, wl.vals), m=wl.m, n=wl.n, params=params, stream=stream)


def debug_precond(mat: Matrix, z: complex):
    """(F^{-1}, gamma) of the dense base preconditioner built at z (test hook)."""
    m, n = mat.shape
    F = np.empty((n, n), dtype=np.complex128, order="F")
    g = np.zeros(1)
    _check(load().ps_debug_precond(mat.handle, float(np.real(z)), float(np.imag(z)), _ptr(F), _ptr(g)),
           "ps_debug_precond")
    return F, float(g[0])


def debug_twolevel(mat: Matrix, zdag: complex, z: complex, W: np.ndarray):
    """(Y = K_Ebar^{-1} W, Ebar, Lambda_bar, iterations, d, gamma) of the
    two-level preconditioner built at a site z_dag and refined at z (test hook)."""
    m, n = mat.shape
    W = np.asfortranarray(W, dtype=np.complex128)
    r = W.shape[1]
    Y = np.empty((n, r), dtype=np.complex128, order="F")
    E = np.empty((n, r), dtype=np.complex128, order="F")
    lam = np.empty(r)
    it = np.zeros(1, dtype=np.int32)
    lib = load()
    _check(lib.ps_debug_twolevel(mat.handle, float(np.real(zdag)), float(np.imag(zdag)), float(np.real(z)),
                                 float(np.imag(z)), _ptr(W), _ptr(Y), _ptr(E), _ptr(lam), _ptr(it)),
           "ps_debug_twolevel")
    d = np.zeros(1)
    g = np.zeros(1)
    _check(lib.ps_debug_site(mat.handle, _ptr(d), _ptr(g)), "ps_debug_site")
    return Y, E, lam, int(it[0]), float(d[0]), float(g[0])


def debug_store(mat: Matrix, tile: int, k_max: int):
    """(k, V, W1, W3, W4, R_A, R_res) of a tile's recycled store (test hook)."""
    m, n = mat.shape
    K = k_max
    V = np.empty((n, K), np.complex128, order="F")
    W1 = np.empty((m, K), np.complex128, order="F")
    W3 = np.empty((n, K), np.complex128, order="F")
    W4 = np.empty((n, K), np.complex128, order="F")
    RA = np.empty((2 * K, 2 * K), np.complex128, order="F")
    Rr = np.empty((4 * K, 4 * K), np.complex128, order="F")
    k = np.zeros(1, np.int32)
    _check(load().ps_debug_store(mat.handle, int(tile), _ptr(k), _ptr(V), _ptr(W1), _ptr(W3), _ptr(W4), _ptr(RA),
                                 _ptr(Rr)), "ps_debug_store")
    return int(k[0]), V, W1, W3, W4, RA, Rr


def debug_ritz(mat: Matrix, tile: int, z: complex, k: int, k_max: int):
    """(xi, residual norms, G) of the Ritz stage on a tile's store (test hook)."""
    xi = np.empty(k)
    res = np.empty(k)
    G = np.empty((k_max, k), np.complex128, order="F")
    _check(load().ps_debug_ritz(mat.handle, int(tile), float(np.real(z)), float(np.imag(z)), _ptr(xi), _ptr(res),
                                _ptr(G)), "ps_debug_ritz")
    return xi, res, G[:k, :]
