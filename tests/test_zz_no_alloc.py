"""The allocation-free eigensolver entry point (pt_heev_noalloc) against the
allocating one (pt_test_heev): the same kernels on the same input, so the
eigenvalues, the number of selected vectors and the selected vectors agree
bit for bit.  Two calls in a row on one device, the second smaller, share
the library's static scratch array."""
import ctypes

import numpy as np
import pytest

from tests.conftest import gpu_available
from tests.helpers import ensure_library

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _lib():
    if not gpu_available():
        pytest.skip("no GPU")
    ensure_library()


def _alloc_heev(a, rule, eps, cap):
    from paper_2201_05529_amd import binding as B
    L = B.lib()
    L.pt_test_heev.restype = ctypes.c_int
    n = a.shape[0]
    af = B._cplx(a)
    w = np.zeros(n)
    v = np.zeros(2 * n * n)
    nv = ctypes.c_int32()
    st = L.pt_test_heev(n, B._dptr(af), rule, ctypes.c_double(eps), cap, B._dptr(w), B._dptr(v), ctypes.byref(nv))
    assert st == 0
    return w, v.view(np.complex128).reshape(n, n), nv.value


def _gram(n, rank, seed):
    rng = np.random.default_rng(seed)
    c = rng.normal(size=(rank, n)) + 1j * rng.normal(size=(rank, n))
    g = c.conj().T @ c
    return 0.5 * (g + g.conj().T)


@pytest.mark.parametrize("rule,eps,cap", [(4, 0.0, 0), (1, 1e-7, 0), (2, 1e-7, 20)])
def test_noalloc_matches_allocating_entry_point_twice(rule, eps, cap):
    from paper_2201_05529_amd import binding as B
    for n, rank, seed in ((200, 150, 1), (96, 96, 2)):   # the second call is smaller
        print(f"noalloc rule={rule} n={n}", flush=True)
        a = _gram(n, rank, seed + 10 * rule)
        w0, v0, k0 = _alloc_heev(a, rule, eps, cap)
        w1, v1, k1, status = B.heev_noalloc(a, rule, eps, cap)
        assert status == 0
        assert k1 == k0
        assert np.array_equal(w1, w0)
        assert np.array_equal(v1[:, :k1], v0[:, :k0])
        # and the decomposition itself holds
        res = a @ v1[:, :k1] - v1[:, :k1] * w1[:k1]
        assert np.abs(res).max() < 1e-10 * np.abs(w1).max()


def test_noalloc_rejects_sizes_beyond_its_scratch():
    from paper_2201_05529_amd import binding as B
    with pytest.raises(B.PtTebdError) as e:
        B.heev_noalloc(np.eye(257, dtype=np.complex128))
    assert e.value.status == -1
