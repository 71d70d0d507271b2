"""GPU PT-MPO construction (pt_mpo_build_ohmic_batch, Appendix B.1) against
the oracle: without truncation the PT-MPO contracted over all paths is the
influence functional itself; with eps_TEMPO and the xi cap it agrees with
the oracle's builder to about eps; many baths in one call are independent
work items; a chain stepped with GPU-built PT-MPOs matches the oracle."""
import itertools

import numpy as np
import pytest

from oracle import bath, ptmpo
from oracle import pt_tebd as opt
from paper_2201_05529_amd import workloads as W
from tests.conftest import gpu_available
from tests.helpers import ensure_library

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _lib():
    if not gpu_available():
        pytest.skip("no GPU")
    ensure_library()


def _direct(eta, sigma, m):
    return np.array([ptmpo.influence_functional(p, eta, sigma)
                     for p in itertools.product(range(4), repeat=m)]).reshape([4] * m)


def _random_path_sum(tensors, seed):
    rng = np.random.default_rng(seed)
    acc = np.ones(1, dtype=np.complex128)
    for p in tensors:
        v = rng.normal(size=4) + 1j * rng.normal(size=4)
        acc = acc @ np.einsum("efx,x->ef", p, v)
    return acc[0]


def test_gpu_ptmpo_untruncated_equals_influence_functional():
    from paper_2201_05529_amd import binding as B
    params = [(0.2, 1.3, 0.15), (0.1, 0.7, 0.1), (0.3, 2.0, 0.15)]
    baths = [{"alpha": a, "wc": 4.0, "temperature": t, "coupling_op": W.SZ} for a, t, _ in params]
    for dt in (0.15,):
        pts = B.build_ptmpo_batch(baths, dt, 6, 3, 1e-13, 64)
        for (a, t, _), pt in zip(params, pts):
            eta = bath.eta_coefficients(a, 4.0, t, dt, 3)
            got = ptmpo.contract_all_paths(pt["tensors"], 4)
            ref = _direct(eta, np.array([1.0, -1.0]), 6)
            err = np.abs(got - ref).max() / np.abs(ref).max()
            print(f"alpha {a} T {t}: relative error {err:.1e}", flush=True)
            assert pt["bond_dims"][0] == 1 and pt["bond_dims"][-1] == 1
            assert err < 1e-10


def test_gpu_ptmpo_dense_coupling():
    from paper_2201_05529_amd import binding as B
    eta = bath.eta_coefficients(0.2, 4.0, 1.3, 0.15, 2)
    pt = B.build_ptmpo_batch([{"alpha": 0.2, "wc": 4.0, "temperature": 1.3, "coupling_op": W.SX}],
                             0.15, 4, 2, 1e-13, 64)[0]
    assert not pt["diagonal"]
    sigma, u = np.linalg.eigh(W.SX)
    w = np.kron(u, u.conj())
    acc = np.ones((1, 1), dtype=np.complex128)
    for p in pt["tensors"]:
        q = np.einsum("xa,efab,by->efxy", w.conj().T, p, w)
        acc = np.einsum("pe,efxx->pxf", acc, q).reshape(-1, p.shape[1])
    got = acc[:, 0].reshape([4] * 4)
    assert np.abs(got - _direct(eta, sigma, 4)).max() < 1e-8


@pytest.mark.parametrize("m,k_cut", [(14, 3), (30, 10)])
def test_gpu_ptmpo_long_horizon_matches_oracle_builder(m, k_cut):
    from paper_2201_05529_amd import binding as B
    alpha, wc, dt = 0.05, 4.0, 0.1
    temps = [1.0, 0.6]
    pts = B.build_ptmpo_batch([{"alpha": alpha, "wc": wc, "temperature": t, "coupling_op": W.SZ} for t in temps],
                              dt, m, k_cut, 1e-7, 24)
    for t, pt in zip(temps, pts):
        eta = bath.eta_coefficients(alpha, wc, t, dt, k_cut)
        ora = ptmpo.tempo_mpo(eta, np.array([1.0, -1.0]), m, 1e-7, xi_max=24)
        cl, co = ptmpo.caps(pt["tensors"], 2), ptmpo.caps(ora, 2)
        print(f"T {t}: dims gpu {max(pt['bond_dims'])} oracle {max(p.shape[1] for p in ora)}; "
              f"cap0 {cl[0][0]:.10f} vs {co[0][0]:.10f}", flush=True)
        assert abs(cl[0][0] - co[0][0]) < 1e-6
        for seed in range(3):
            a, b = _random_path_sum(pt["tensors"], seed), _random_path_sum(ora, seed)
            assert abs(a - b) < 1e-6 * abs(b)


def test_chain_with_gpu_ptmpo_matches_oracle():
    # the N = 3 workload stepped with the GPU-built PT-MPO, against the
    # oracle stepped with the oracle-built one: the two builders differ by
    # about eps_TEMPO, which bounds the observable difference
    from paper_2201_05529_amd import binding as B
    from oracle.build import problem_from_workload
    wl = W.xyz3()
    b = wl["baths"][0]
    pt = B.build_ptmpo_batch([b], wl["dt"], wl["n_steps"], b["k_cut"], wl["eps_tempo"], wl["xi_max"])[0]
    ch = B.Chain(wl["h_site"], wl["h_bond"], wl["rho0"], wl["dt"], baths=[{"site": 0, "tensors": pt["tensors"]}],
                 chi_max=wl["chi_max"], xi_max=wl["xi_max"], eps=wl["eps"])
    prob, _ = problem_from_workload(wl)
    eng = opt.Engine(prob)
    err = 0.0
    for _ in range(wl["n_steps"]):
        ch.step(1)
        eng.step(1)
        v, _tr = ch.observe(range(3), np.array([W.SZ] * 3))
        err = max(err, np.abs(v - np.array([eng.expectation(s, W.SZ) for s in range(3)])).max())
    print(f"xyz3 with the GPU PT-MPO: max |d<sz>| {err:.1e}", flush=True)
    assert err < 1e-5


def test_builds_of_different_lengths_in_one_call_equal_single_builds():
    # a bath's own length: builds advance in lockstep and each stops at its
    # own length, so every build equals the build made alone
    from paper_2201_05529_amd import binding as B
    specs = [{"alpha": 0.1, "wc": 4.0, "temperature": 1.2, "coupling_op": W.SZ, "n_steps": 7},
             {"alpha": 0.2, "wc": 4.0, "temperature": 0.8, "coupling_op": W.SZ, "n_steps": 12},
             {"alpha": 0.15, "wc": 4.0, "temperature": 2.0, "coupling_op": W.SZ, "n_steps": 3}]
    together = B.build_ptmpo_batch(specs, 0.1, 12, 4, 1e-9, 32)
    for spec, pt in zip(specs, together):
        alone = B.build_ptmpo_batch([dict(spec, n_steps=None)], 0.1, spec["n_steps"], 4, 1e-9, 32)[0]
        assert len(pt["tensors"]) == spec["n_steps"]
        assert pt["bond_dims"] == alone["bond_dims"]
        for a, b in zip(pt["tensors"], alone["tensors"]):
            assert np.array_equal(a, b)
