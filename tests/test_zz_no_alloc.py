"""ps_apply_noalloc (marked gpu): the operator apply that allocates nothing
(its workspace is the library's static per-GPU array) against the
allocating ps_debug_apply, called through the C ABI on device arrays: two
calls in a row on each handle, the second with a smaller input, for a dense
and a CSR handle.  Both compute Y = C(z) X (or C(z)^* X) with different
split-K depths, so they agree to rounding: |Y - Y_ref| <= 1e-13 (||C||_F +
|z|) ||x|| per column (a bound far above the rounding of a length-n complex
dot product)."""
import numpy as np
import pytest

import workloads

P = pytest.importorskip("paper_2606_26785_amd")
torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu


def _dev(A):
    """Column-major complex128 device copy of A (torch stores the transpose
    row-major)."""
    return torch.from_numpy(np.ascontiguousarray(A.T)).to("cuda")


def _noalloc(mat, X, z, herm):
    m, n = mat.shape
    rows_out = n if herm else m
    rows_in = m if herm else n
    w = X.shape[1]
    dX = _dev(X)
    dY = torch.full((w, rows_out), complex(np.nan, np.nan), dtype=torch.complex128, device="cuda")
    P.apply_noalloc(mat, dX.data_ptr(), rows_in, w, dY.data_ptr(), rows_out, z=z, herm=herm)
    torch.cuda.synchronize()
    return dY.cpu().numpy().T


def _check_pair(mat, A, X, z, herm):
    Y = _noalloc(mat, X, z, herm)
    Yr = P.debug_apply(mat, X, z=z, herm=herm)
    scale = (np.linalg.norm(A) + abs(z)) * np.linalg.norm(X, axis=0)
    assert np.isfinite(Y).all()
    assert (np.abs(Y - Yr).max(axis=0) <= 1e-13 * scale).all()
    # and the definition, C(z) = C - z [I_n; 0]
    m, n = A.shape
    Cz = A - z * np.eye(m, n)
    ref = (Cz.conj().T if herm else Cz) @ X
    assert (np.abs(Y - ref).max(axis=0) <= 1e-13 * scale).all()


def _rand(rng, rows, w):
    return (rng.standard_normal((rows, w)) + 1j * rng.standard_normal((rows, w))) / np.sqrt(2.0)


def test_noalloc_dense_two_calls():
    wl = workloads.triangular_disk(seed=1001, n=300, grid=4)
    mat = P.create_from_workload(wl)
    rng = np.random.default_rng(11)
    try:
        print("dense n=300: w=24 then w=5 (adjoint)", flush=True)
        _check_pair(mat, wl.dense, _rand(rng, 300, 24), 0.3 - 0.7j, False)
        _check_pair(mat, wl.dense, _rand(rng, 300, 5), -1.1 + 0.2j, True)
    finally:
        mat.close()


def test_noalloc_csr_two_calls():
    wl = workloads.folding(seed=7, n=500, grid=4)
    mat = P.create_from_workload(wl)
    A = wl.to_dense()
    rng = np.random.default_rng(12)
    try:
        print("csr folding n=500 m=504: w=16 then w=3 (adjoint)", flush=True)
        _check_pair(mat, A, _rand(rng, 500, 16), 0.5 + 0.5j, False)
        _check_pair(mat, A, _rand(rng, 504, 3), 0.1 - 0.2j, True)
    finally:
        mat.close()


def test_noalloc_rejects_bad_sizes():
    wl = workloads.triangular_disk(seed=1001, n=64, grid=4)
    mat = P.create_from_workload(wl)
    try:
        X = torch.zeros((8, 64), dtype=torch.complex128, device="cuda")
        Y = torch.zeros((8, 64), dtype=torch.complex128, device="cuda")
        with pytest.raises(P.PSError):
            P.apply_noalloc(mat, X.data_ptr(), 64, 65, Y.data_ptr(), 64)      # w > 64
        with pytest.raises(P.PSError):
            P.apply_noalloc(mat, X.data_ptr(), 63, 8, Y.data_ptr(), 64)       # ldx < n
        with pytest.raises(P.PSError):
            P.apply_noalloc(mat, 0, 64, 8, Y.data_ptr(), 64)                  # NULL X
    finally:
        mat.close()
