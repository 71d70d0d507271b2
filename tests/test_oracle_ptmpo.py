"""Pins of oracle/ptmpo.py."""
import itertools

import numpy as np
import pytest

from oracle import bath, ptmpo
from oracle import liouville as lv
from oracle.pt_tebd import truncation_rank

SIGMA_Z_EIG = np.array([1.0, -1.0])


def direct_if(eta, sigma, m):
    d2 = len(sigma) ** 2
    return np.array([ptmpo.influence_functional(p, eta, sigma)
                     for p in itertools.product(range(d2), repeat=m)]).reshape([d2] * m)


def brute_factor_product(eta, sigma, path):
    # the influence functional written out as one exponent (independent of
    # influence_matrix): sum over ordered pairs k >= k' of the
    # Feynman-Vernon discretised exponent
    sp = np.repeat(sigma, len(sigma))
    sm = np.tile(sigma, len(sigma))
    k_cut = len(eta) - 1
    phi = 0.0 + 0.0j
    for k in range(len(path)):
        for kp in range(max(0, k - k_cut), k + 1):
            e = eta[k - kp]
            x, y = path[k], path[kp]
            phi += (sp[x] - sm[x]) * (e * sp[y] - np.conj(e) * sm[y])
    return np.exp(-phi)


def test_influence_functional_matches_exponent_sum():
    eta = bath.eta_coefficients(0.1, 4.0, 1.0, 0.1, 3)
    rng = np.random.default_rng(0)
    for _ in range(20):
        path = list(rng.integers(0, 4, size=6))
        assert np.isclose(ptmpo.influence_functional(path, eta, SIGMA_Z_EIG),
                          brute_factor_product(eta, SIGMA_Z_EIG, path), rtol=1e-13)


@pytest.mark.parametrize("k_cut,m", [(1, 4), (2, 4), (3, 5), (4, 4)])
def test_history_mpo_equals_direct_if(k_cut, m):
    eta = bath.eta_coefficients(0.2, 4.0, 1.3, 0.15, k_cut)
    h = ptmpo.history_mpo(eta, SIGMA_Z_EIG, m)
    assert h[0].shape[0] == 1 and h[-1].shape[1] == 1
    got = ptmpo.contract_all_paths(h, 4)
    assert np.abs(got - direct_if(eta, SIGMA_Z_EIG, m)).max() < 1e-13


@pytest.mark.parametrize("k_cut,m", [(2, 5), (4, 5), (3, 6)])
def test_tempo_mpo_equals_direct_if(k_cut, m):
    eta = bath.eta_coefficients(0.2, 4.0, 1.3, 0.15, k_cut)
    t = ptmpo.tempo_mpo(eta, SIGMA_Z_EIG, m, 1e-14)
    got = ptmpo.contract_all_paths(t, 4)
    ref = direct_if(eta, SIGMA_Z_EIG, m)
    assert np.abs(got - ref).max() < 1e-11 * np.abs(ref).max()


def test_tempo_truncation_error_tracks_eps():
    eta = bath.eta_coefficients(0.3, 4.0, 1.0, 0.2, 5)
    ref = direct_if(eta, SIGMA_Z_EIG, 6)
    errs = []
    for eps in (1e-3, 1e-5, 1e-7):
        got = ptmpo.contract_all_paths(ptmpo.tempo_mpo(eta, SIGMA_Z_EIG, 6, eps), 4)
        errs.append(np.linalg.norm(got - ref) / np.linalg.norm(ref))
    assert errs[0] > errs[1] > errs[2]
    assert errs[2] < 1e-6


def test_zero_coupling_gives_identity():
    eta = np.zeros(4, dtype=np.complex128)
    t = ptmpo.tempo_mpo(eta, SIGMA_Z_EIG, 6, 1e-10)
    assert all(p.shape[:2] == (1, 1) for p in t)
    assert np.allclose(np.abs(ptmpo.contract_all_paths(t, 4)), 1.0)


def test_history_caps_are_all_ones():
    eta = bath.eta_coefficients(0.2, 4.0, 1.3, 0.15, 3)
    caps = ptmpo.caps(ptmpo.history_mpo(eta, SIGMA_Z_EIG, 6), 2)
    for c in caps:
        assert np.allclose(c, 1.0, atol=1e-14)


def test_caps_give_the_shorter_influence_functional():
    # containment: the first k slots of the M-step PT capped with c^(k) equal
    # the influence functional of k steps (all later factors trace to one)
    eta = bath.eta_coefficients(0.25, 4.0, 1.0, 0.1, 4)
    m = 6
    t = ptmpo.tempo_mpo(eta, SIGMA_Z_EIG, m, 1e-14)
    caps = ptmpo.caps(t, 2)
    for k in (2, 4, 5):
        acc = np.ones((1, 1), dtype=np.complex128)
        for p in t[:k]:
            acc = np.einsum("pe,efx->pxf", acc, p).reshape(-1, p.shape[1])
        got = (acc @ caps[k]).reshape([4] * k)
        assert np.abs(got - direct_if(eta, SIGMA_Z_EIG, k)).max() < 1e-11


def test_rotation_to_computational_basis():
    # sigma^z handled through eigh (permuted eigenbasis) must equal the
    # diagonal computational-basis tensors
    eta = bath.eta_coefficients(0.2, 4.0, 1.3, 0.15, 2)
    diag = ptmpo.history_mpo(eta, SIGMA_Z_EIG, 4)
    sigma_eigh, _ = np.linalg.eigh(lv.SIGMA_Z)
    rot = ptmpo.to_computational_basis(ptmpo.history_mpo(eta, sigma_eigh, 4), lv.SIGMA_Z)
    got_d = ptmpo.contract_all_paths(diag, 4)
    acc = np.ones((1, 1), dtype=np.complex128)
    for p in rot:
        acc = np.einsum("pe,efxx->pxf", acc, p).reshape(-1, p.shape[1])
    assert np.abs(acc[:, 0].reshape([4] * 4) - got_d).max() < 1e-13


def oracle_problem_small(wl):
    from oracle.build import problem_from_workload
    prob, _ = problem_from_workload(wl, n_steps=2)
    return prob


def test_read_out_survives_a_scale_beyond_the_double_range():
    # the chain log-scale and the tensors may each leave the double range
    # (the N = 21 workload reaches log-scale -714 by step 54) while the
    # observable stays finite: shift scale between them and read out again
    from oracle import pt_tebd
    from paper_2201_05529_amd import workloads as W
    wl = W.random_small_chain(9, 4, with_bath_sites=(1,), k_cut=2, eps=1e-10, xi_max=16)
    prob = oracle_problem_small(wl)
    eng = pt_tebd.Engine(prob)
    eng.step(2)
    ref = [eng.expectation(s, W.SZ) for s in range(4)]
    tr = eng.trace()
    shift = 300.0  # exp(4 * 300) overflows a double, exp(-4 * 300) underflows
    eng.mps.log_scale -= 4 * shift
    for n in range(4):
        eng.mps.gammas[n] = eng.mps.gammas[n] * np.exp(shift)
    got = [eng.expectation(s, W.SZ) for s in range(4)]
    assert np.allclose(got, ref, rtol=1e-12, atol=1e-14)
    assert abs(eng.trace() - tr) < 1e-12
