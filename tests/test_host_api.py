"""Host-side argument checks of the C ABI.  Every case here is rejected before
the library touches the GPU, so these run without one."""
import numpy as np
import pytest

P = pytest.importorskip("paper_2606_26785_amd")

PS_EINVAL, PS_EUNSUPPORTED = -1, -5


def _status(fn, *a, **k):
    with pytest.raises(P.PSError) as e:
        fn(*a, **k)
    return e.value.status


def _dense(m=6, n=4, seed=0):
    rng = np.random.default_rng(seed)
    return rng.standard_normal((m, n)) + 1j * rng.standard_normal((m, n))


def test_grid_arguments():
    assert _status(P.ps_grid, 0, 1, 0, 1, 0, 3) == PS_EINVAL
    assert _status(P.ps_grid, 0, 1, 0, 1, 3, 0) == PS_EINVAL
    assert _status(P.ps_grid, 0, float("nan"), 0, 1, 3, 3) == PS_EINVAL
    assert _status(P.ps_grid, 0, 1, float("inf"), 1, 3, 3) == PS_EINVAL
    g = P.ps_grid(-1, 1, -2, 2, 1, 1)
    assert g.nx == 1 and g.ny == 1
    g.close()


def test_create_shape_and_values():
    assert _status(P.ps_create, dense=_dense(3, 4)) == PS_EINVAL          # m < n
    C = _dense()
    C[2, 1] = np.nan
    assert _status(P.ps_create, dense=C) == PS_EINVAL                      # non-finite entry


@pytest.mark.parametrize("field,value", [("r", 3), ("r", 18), ("k_max", 12), ("k_max", 128), ("rbar", 5),
                                         ("kbar_max", 20), ("kbar_max", 72), ("max_iters", 0),
                                         ("batch", 0), ("eta", 0.0), ("eta_svd", -1.0), ("omega", 0.5),
                                         ("eta_abs", 2e-8), ("tol_abs", -1.0), ("esc_iters", -1), ("precond", 3),
                                         ("eta_proj", 0.0), ("tau_max", 0.5), ("reg_base", -1.0),
                                         ("tile_points", 0)])
def test_create_rejects_bad_params(field, value):
    params = P.default_params(**{field: value})
    assert _status(P.ps_create, dense=_dense(), params=params) == PS_EINVAL


def test_two_level_block_sizes_must_match():
    params = P.default_params(precond=2, rbar=4)
    assert _status(P.ps_create, dense=_dense(), params=params) == PS_EINVAL


def test_rectangular_csr_accepts_a_preconditioner():
    # the incomplete Cholesky base factors N(z) = C(z)^* C(z), which is
    # n x n for any m >= n: the parameters pass validation (on a machine
    # without a GPU the call then fails only for want of a device)
    rowptr = np.array([0, 1, 2, 3, 4, 4, 4], dtype=np.int64)
    colind = np.array([0, 1, 2, 3], dtype=np.int32)
    vals = np.ones(4, dtype=np.complex128)
    for pc in (1, 2):
        params = P.default_params(precond=pc)
        st = _status(P.ps_create, csr=(rowptr, colind, vals), m=6, n=4, params=params)
        assert st not in (PS_EINVAL, PS_EUNSUPPORTED)


def test_error_text():
    lib = P.load()
    assert lib.ps_strerror(PS_EINVAL).decode() == "invalid argument"
    with pytest.raises(P.PSError) as e:
        P.ps_grid(0, 1, 0, 1, 0, 0)
    assert "nx and ny" in str(e.value)
