"""Pins of oracle/gates.py."""
import numpy as np
import scipy.linalg

from oracle import brute, gates, liouville as lv
from paper_2201_05529_amd import workloads as W


def chain(n, seed=0, field=True):
    wl = W.random_small_chain(seed, n, field=field)
    return wl["h_site"], wl["h_bond"]


def test_kprime_weights_sum_to_chain_hamiltonian():
    for n in (2, 3, 5):
        h_site, h_bond = chain(n, seed=n)
        total = np.zeros((2 ** n, 2 ** n), dtype=np.complex128)
        for b in range(n - 1):
            wl, wr = gates.site_weights(b, n)
            kp = h_bond[b] + wl * np.kron(h_site[b], np.eye(2)) + wr * np.kron(np.eye(2), h_site[b + 1])
            total += lv.embed_bond_operator(kp, b, n, 2)
        expect = sum(lv.embed_site_operator(h_site[s], s, n, 2) for s in range(n)) \
            + sum(lv.embed_bond_operator(h_bond[b], b, n, 2) for b in range(n - 1))
        assert np.allclose(total, expect, atol=1e-13)


def test_two_site_gate_equals_dense_expm():
    # N = 2: the single (odd) bond carries exp(L_chain dt/2); compare against
    # the dense whole-chain Liouvillian built independently with kron.
    h_site, h_bond = chain(2, seed=7)
    dt = 0.13
    g = gates.chain_gates(h_site, h_bond, None, dt, 2)[0]
    dense = scipy.linalg.expm(brute.dense_chain_liouvillian(h_site, h_bond, None, 2) * dt / 2)
    assert np.allclose(g, dense, atol=1e-13)


def test_unitary_gate_is_u_kron_uconj():
    h_site, h_bond = chain(3, seed=3)
    dt = 0.2
    gs = gates.chain_gates(h_site, h_bond, None, dt, 2)
    for b, g in enumerate(gs):
        wl, wr = gates.site_weights(b, 3)
        kp = h_bond[b] + wl * np.kron(h_site[b], np.eye(2)) + wr * np.kron(np.eye(2), h_site[b + 1])
        w, v = np.linalg.eigh(kp)
        u = (v * np.exp(-1j * w * gates.bond_tau(b, dt))) @ v.conj().T
        nat = np.kron(u, u.conj())
        assert np.allclose(g, lv.superop_to_site_major(nat, 2), atol=1e-13)


def test_gates_trace_and_hermiticity_preserving():
    rng = np.random.default_rng(5)
    h_site, h_bond = chain(4, seed=4)
    lind = [[0.3 * W.SX + 0.1j * W.SZ], [], [0.2 * W.SY], []]
    gs = gates.chain_gates(h_site, h_bond, lind, 0.1, 2)
    t2 = np.kron(lv.trace_vector(2), lv.trace_vector(2))
    for g in gs:
        assert np.allclose(t2 @ g, t2, atol=1e-13)
        m = rng.normal(size=(4, 4)) + 1j * rng.normal(size=(4, 4))
        rho = m + m.conj().T
        v_sm = lv.superop_to_site_major(np.eye(16), 2) @ lv.vec(rho)  # identity perm check
        p = lv.two_site_natural_to_site_major(2)
        out_sm = g @ lv.vec(rho)[p]
        out_nat = np.empty_like(out_sm)
        out_nat[p] = out_sm
        r = out_nat.reshape(4, 4)
        assert np.allclose(r, r.conj().T, atol=1e-12)
        assert v_sm.shape == (16,)


def test_commuting_chain_gates_reproduce_half_step_exactly():
    # Ising ZZ bonds + z fields commute: E(dt/4) O(dt/2) E(dt/4) == exp(L dt/2)
    n, dt = 4, 0.3
    h_site = np.array([0.5 * f * W.SZ for f in (0.3, -0.7, 1.1, 0.2)])
    h_bond = np.array([0.25 * j * np.kron(W.SZ, W.SZ) for j in (1.0, 0.6, 1.4)])
    gs = gates.chain_gates(h_site, h_bond, None, dt, 2)
    v = np.ones(1)
    rng = np.random.default_rng(2)
    for _ in range(n):
        m = rng.normal(size=(2, 2)) + 1j * rng.normal(size=(2, 2))
        v = np.kron(v, lv.vec(m @ m.conj().T))
    psi = v.reshape([4] * n)
    for sub in gates.half_step_sublayers(n):
        for b in sub:
            psi = np.moveaxis(np.tensordot(gs[b].reshape(4, 4, 4, 4), psi, axes=([2, 3], [b, b + 1])),
                              [0, 1], [b, b + 1])
    dense = scipy.linalg.expm(brute.dense_chain_liouvillian(h_site, h_bond, None, 2) * dt / 2) @ v
    assert np.allclose(psi.reshape(-1), dense, atol=1e-12)


def test_sublayer_order():
    assert gates.half_step_sublayers(2) == [[0]]
    assert gates.half_step_sublayers(3) == [[1], [0], [1]]
    assert gates.half_step_sublayers(5) == [[1, 3], [0, 2], [1, 3]]
    assert gates.bond_tau(0, 0.4) == 0.2 and gates.bond_tau(1, 0.4) == 0.1
