"""CPU-side checks of the C-ABI library: it loads, exports every declared
symbol, validates its inputs, and its host helpers (bath coefficients,
PT-MPO builder) agree with the oracle.  No GPU calls."""
import ctypes
import itertools
import os
import re

import numpy as np
import pytest

from oracle import bath, ptmpo
from paper_2201_05529_amd import workloads as W
from tests.helpers import ROOT, ensure_library


@pytest.fixture(scope="module")
def B():
    ensure_library()
    from paper_2201_05529_amd import binding
    return binding


def test_exports_every_declared_symbol(B):
    names = set()
    for hname in sorted(os.listdir(os.path.join(ROOT, "include"))):
        if hname.endswith(".h"):
            header = open(os.path.join(ROOT, "include", hname)).read()
            names |= set(re.findall(r"\b(pt_(?:tebd|mpo|bath|test)_\w+)\s*\(", header))
    assert len(names) >= 16
    lib = ctypes.CDLL(B.LIB_PATH)
    for n in sorted(names):
        assert hasattr(lib, n), n


@pytest.mark.parametrize("cutoff", ["exp", "gauss"])
def test_bath_eta_matches_oracle(B, cutoff):
    for (a, wc, t, dt, k) in [(0.16, 4.0, 2.0, 0.05, 20), (0.05, 4.0, 1.0, 0.1, 10), (0.08, 4.0, 0.0, 0.1, 5)]:
        e1 = B.bath_eta(a, wc, t, dt, k, cutoff)
        e2 = bath.eta_coefficients(a, wc, t, dt, k, cutoff)
        assert np.abs(e1 - e2).max() < 1e-12


def _direct(eta, sigma, m):
    return np.array([ptmpo.influence_functional(p, eta, sigma)
                     for p in itertools.product(range(4), repeat=m)]).reshape([4] * m)


def test_library_ptmpo_equals_influence_functional(B):
    eta = bath.eta_coefficients(0.2, 4.0, 1.3, 0.15, 3)
    pt = B.build_ptmpo(0.2, 4.0, 1.3, 0.15, 6, 3, 1e-13, 1000, W.SZ)
    assert pt["diagonal"] and pt["bond_dims"][0] == 1 and pt["bond_dims"][-1] == 1
    got = ptmpo.contract_all_paths(pt["tensors"], 4)
    ref = _direct(eta, np.array([1.0, -1.0]), 6)
    # eps = 1e-13: only the discarded tails below 1e-13 of each window's
    # largest singular value separate the two
    assert np.abs(got - ref).max() < 1e-11 * np.abs(ref).max()


def test_library_ptmpo_dense_coupling(B):
    # sigma^x coupling: rotate the library's dense tensors back to the
    # coupling eigenbasis and compare with the influence functional there
    eta = bath.eta_coefficients(0.2, 4.0, 1.3, 0.15, 2)
    pt = B.build_ptmpo(0.2, 4.0, 1.3, 0.15, 4, 2, 1e-13, 1000, W.SX)
    assert not pt["diagonal"]
    sigma, u = np.linalg.eigh(W.SX)
    w = np.kron(u, u.conj())
    acc = np.ones((1, 1), dtype=np.complex128)
    for p in pt["tensors"]:
        q = np.einsum("xa,efab,by->efxy", w.conj().T, p, w)   # W^dag P W
        acc = np.einsum("pe,efxx->pxf", acc, q).reshape(-1, p.shape[1])
    got = acc[:, 0].reshape([4] * 4)
    assert np.abs(got - _direct(eta, sigma, 4)).max() < 1e-8


def test_library_ptmpo_truncated_matches_oracle_builder(B):
    # both builders compress the same influence functional with eps: their
    # contractions over all paths agree to about eps
    eta = bath.eta_coefficients(0.3, 4.0, 1.0, 0.2, 4)
    lib_pt = B.build_ptmpo(0.3, 4.0, 1.0, 0.2, 6, 4, 1e-6, 1000, W.SZ)
    ora = ptmpo.tempo_mpo(eta, np.array([1.0, -1.0]), 6, 1e-6)
    a = ptmpo.contract_all_paths(lib_pt["tensors"], 4)
    b = ptmpo.contract_all_paths(ora, 4)
    assert np.linalg.norm(a - b) / np.linalg.norm(b) < 1e-5


def _random_path_sum(tensors, rng_seed):
    """sum over all paths of prod_k P_k[x_k] v_k[x_k] for seeded random
    complex v_k (a contraction that probes every slot of the PT-MPO)."""
    rng = np.random.default_rng(rng_seed)
    acc = np.ones(1, dtype=np.complex128)
    for p in tensors:
        v = rng.normal(size=4) + 1j * rng.normal(size=4)
        acc = acc @ np.einsum("efx,x->ef", p, v)
    return acc[0]


@pytest.mark.parametrize("m,k_cut", [(14, 3), (20, 5)])
def test_library_ptmpo_long_horizon_matches_oracle_builder(B, m, k_cut):
    # horizons well past the memory cutoff: the window slides over the slots
    # (the N=21 workload runs 100 steps with a 10-step memory)
    alpha, wc, temp, dt = 0.05, 4.0, 1.0, 0.1
    eta = bath.eta_coefficients(alpha, wc, temp, dt, k_cut)
    lib_pt = B.build_ptmpo(alpha, wc, temp, dt, m, k_cut, 1e-7, 24, W.SZ)
    ora = ptmpo.tempo_mpo(eta, np.array([1.0, -1.0]), m, 1e-7, xi_max=24)
    assert lib_pt["bond_dims"] == [1] + [t.shape[1] for t in ora]
    # trace preservation of the bath: the cap at step 0 (bond dimension 1,
    # so free of the gauge of the inner bonds) is 1 up to the truncation
    # (here mostly the xi cap of 24)
    cl = ptmpo.caps(lib_pt["tensors"], 2)
    co = ptmpo.caps(ora, 2)
    assert abs(cl[0][0] - 1.0) < 1e-3 and abs(cl[0][0] - co[0][0]) < 1e-9
    for seed in range(3):
        a, b = _random_path_sum(lib_pt["tensors"], seed), _random_path_sum(ora, seed)
        assert abs(a - b) < 1e-9 * abs(b)


def _config(B, **over):
    n = over.pop("n_sites", 3)
    hs = np.zeros((n, 2, 2), dtype=np.complex128)
    hb = np.array([W.xyz_bond(1, 1, 1)] * max(n - 1, 1), dtype=np.complex128)
    r0 = np.array([W.UP] * n, dtype=np.complex128)
    keep = [B._cplx(hs), B._cplx(hb), B._cplx(r0)]
    cfg = B.Config()
    cfg.n_sites, cfg.d, cfg.dt = n, 2, 0.1
    cfg.h_site, cfg.h_bond, cfg.rho0 = [B._dptr(k) for k in keep]
    cfg.n_lindblad, cfg.lindblad, cfg.n_baths, cfg.baths = 0, None, 0, None
    cfg.chi_max, cfg.xi_max, cfg.svd_rel_cutoff, cfg.precision, cfg.seed = 16, 4, 1e-7, 0, 1
    for k, v in over.items():
        setattr(cfg, k, v)
    return cfg, keep


def _ws(B, cfg):
    size = ctypes.c_size_t()
    return B.lib().pt_tebd_workspace_size(ctypes.byref(cfg), ctypes.byref(size)), size.value


def test_validation_rejects_bad_configs(B):
    cfg, keep = _config(B)
    st, size = _ws(B, cfg)
    assert st == 0 and size > 0
    for field, val in [("n_sites", 0), ("d", 3), ("dt", -0.1), ("chi_max", 0), ("svd_rel_cutoff", -1.0),
                       ("precision", 7)]:
        bad, k2 = _config(B)
        setattr(bad, field, val)
        assert _ws(B, bad)[0] == -1, field
    # non-Hermitian site Hamiltonian
    hs = np.zeros((3, 2, 2), dtype=np.complex128)
    hs[0, 0, 1] = 1.0
    arr = B._cplx(hs)
    bad, k2 = _config(B)
    bad.h_site = B._dptr(arr)
    assert _ws(B, bad)[0] == -1


def test_validation_rejects_bad_baths(B):
    cfg, keep = _config(B)
    t = np.ones((1, 2, 4), dtype=np.complex128)
    flat = B._cplx(t)
    tptr = (ctypes.POINTER(ctypes.c_double) * 1)(B._dptr(flat))
    for dims, expect in [([1, 2], 0), ([2, 2], -1), ([1, 9], -1)]:
        d = np.array(dims, dtype=np.int32)
        bath_s = (B.Bath * 1)()
        bath_s[0].site, bath_s[0].n_steps, bath_s[0].diagonal = 1, 1, 1
        bath_s[0].bond_dims = d.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
        bath_s[0].tensors = tptr
        bath_s[0].caps = None
        cfg.n_baths, cfg.baths = 1, bath_s
        assert _ws(B, cfg)[0] == expect, dims
    nan = np.full((1, 2, 4), np.nan, dtype=np.complex128)
    nflat = B._cplx(nan)
    nptr = (ctypes.POINTER(ctypes.c_double) * 1)(B._dptr(nflat))
    d = np.array([1, 2], dtype=np.int32)
    bath_s = (B.Bath * 1)()
    bath_s[0].site, bath_s[0].n_steps, bath_s[0].diagonal = 1, 1, 1
    bath_s[0].bond_dims = d.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
    bath_s[0].tensors = nptr
    cfg.n_baths, cfg.baths = 1, bath_s
    assert _ws(B, cfg)[0] == -4
