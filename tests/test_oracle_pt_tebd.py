"""Pins of oracle/pt_tebd.py against brute force, dense expm and closed forms."""
import numpy as np
import pytest

from oracle import bath, brute, closed_forms as cf, ptmpo, pt_tebd
from oracle import liouville as lv
from oracle.build import problem_from_workload
from paper_2201_05529_amd import workloads as W

SZ, SX, SY = W.SZ, W.SX, W.SY


def problem_no_bath(wl, eps=1e-13, chi_max=None, lindblad=None):
    return pt_tebd.Problem(wl["h_site"], wl["h_bond"], wl["rho0"], wl["dt"],
                           lindblad=lindblad, chi_max=chi_max, eps=eps)


@pytest.mark.parametrize("n", [1, 2, 3, 4, 5])
def test_zero_coupling_same_split_matches_dense(n):
    wl = W.random_small_chain(10 + n, n)
    eng = pt_tebd.Engine(problem_no_bath(wl))
    bf = brute.BruteForce(wl["h_site"], wl["h_bond"], wl["rho0"], wl["dt"])
    for _ in range(4):
        eng.step()
        bf.step()
        for s in range(n):
            for op in (SX, SY, SZ):
                assert abs(eng.expectation(s, op) - bf.expectation(s, op)) < 1e-11
        assert abs(eng.trace() - 1.0) < 1e-12


def test_zero_coupling_converges_to_exact_evolution_second_order():
    # Markovian reduction: without a PT the network is Liouville-space TEBD;
    # against the dense exp(L t) the error scales as dt^2
    wl = W.random_small_chain(3, 4)
    lind = [[0.2 * (SX - 1j * SY) / 2], [], [0.1 * SZ], []]
    t_final = 0.8
    errs = []
    for m in (4, 8, 16):
        wl2 = dict(wl, dt=t_final / m)
        eng = pt_tebd.Engine(problem_no_bath(wl2, lindblad=lind))
        eng.step(m)
        exact = brute.exact_evolution(wl["h_site"], wl["h_bond"], lind, wl["rho0"], t_final, 2)
        errs.append(max(abs(eng.expectation(s, SZ) - brute.site_major_expectation(exact, 4, s, SZ, 2))
                        for s in range(4)))
    assert errs[0] / errs[1] > 3.0 and errs[1] / errs[2] > 3.0


def test_lindblad_same_split_matches_brute():
    wl = W.random_small_chain(21, 3)
    lind = [[0.3 * (SX - 1j * SY) / 2], [0.2 * SZ], [0.25 * (SX + 1j * SY) / 2]]
    eng = pt_tebd.Engine(problem_no_bath(wl, lindblad=lind))
    bf = brute.BruteForce(wl["h_site"], wl["h_bond"], wl["rho0"], wl["dt"], lindblad=lind)
    eng.step(5)
    bf.step(5)
    for s in range(3):
        assert abs(eng.expectation(s, SZ) - bf.expectation(s, SZ)) < 1e-11


@pytest.mark.parametrize("n,bath_sites,k_cut,m", [(1, (0,), 3, 6), (2, (0,), 3, 5), (3, (0,), 3, 5),
                                                  (3, (0, 2), 2, 4), (2, (0, 1), 2, 5)])
def test_history_pt_tebd_matches_brute_force(n, bath_sites, k_cut, m):
    wl = W.random_small_chain(30 + n, n, with_bath_sites=bath_sites, k_cut=k_cut, eps=1e-12)
    prob, _ = problem_from_workload(wl, form="history", n_steps=m)
    eng = pt_tebd.Engine(prob)
    baths = [{"site": b["site"], "coupling_op": b["coupling_op"],
              "eta": bath.eta_coefficients(b["alpha"], b["wc"], b["temperature"], wl["dt"], k_cut)}
             for b in wl["baths"]]
    bf = brute.BruteForce(wl["h_site"], wl["h_bond"], wl["rho0"], wl["dt"], baths=baths)
    for _ in range(m):
        eng.step()
        bf.step()
        for s in range(n):
            for op in (SX, SZ):
                assert abs(eng.expectation(s, op) - bf.expectation(s, op)) < 1e-9
        assert abs(eng.trace() - bf.trace()) < 1e-9


def test_dense_coupling_pt_tebd_matches_brute_force():
    # coupling through sigma^x: PT tensors are dense in the computational basis
    wl = W.random_small_chain(44, 2, with_bath_sites=(1,), k_cut=2, eps=1e-12)
    wl["baths"][0]["coupling_op"] = SX.copy()
    prob, _ = problem_from_workload(wl, form="history", n_steps=4)
    eng = pt_tebd.Engine(prob)
    b = wl["baths"][0]
    bf = brute.BruteForce(wl["h_site"], wl["h_bond"], wl["rho0"], wl["dt"], baths=[{
        "site": 1, "coupling_op": SX,
        "eta": bath.eta_coefficients(b["alpha"], b["wc"], b["temperature"], wl["dt"], 2)}])
    eng.step(4)
    bf.step(4)
    for s in range(2):
        assert abs(eng.expectation(s, SZ) - bf.expectation(s, SZ)) < 1e-9


def test_ch_sequence_equals_theta_svd():
    wl = W.random_small_chain(50, 3, with_bath_sites=(0, 2), k_cut=3, eps=1e-12, random_state=True)
    prob, _ = problem_from_workload(wl, form="tempo", n_steps=6)
    a = pt_tebd.Engine(prob, mode="ch")
    b = pt_tebd.Engine(prob, mode="theta")
    for _ in range(6):
        a.step()
        b.step()
        for s in range(3):
            assert abs(a.expectation(s, SZ) - b.expectation(s, SZ)) < 1e-9
        for la, lb in zip(a.mps.lams, b.mps.lams):
            assert la.shape == lb.shape and np.allclose(la, lb, atol=1e-9)


def test_pure_dephasing_closed_form():
    h, alpha, wc, temp, dt, m = 0.9, 0.15, 4.0, 1.2, 0.1, 7
    plus = 0.5 * np.array([[1, 1], [1, 1]], dtype=np.complex128)
    wl = W.make_chain("deph", 1, [], [h], [plus], dt, m,
                      [W.bath(0, alpha, wc, temp, m - 1)], chi_max=4, xi_max=4 ** 7, eps=1e-13)
    prob, _ = problem_from_workload(wl, form="history", n_steps=m)
    eng = pt_tebd.Engine(prob)
    for k in range(1, m + 1):
        eng.step()
        rho = eng.reduced_density_matrix()
        expect = cf.pure_dephasing_coherence(0.5, h, k * dt, cf.g_closed_form_exp(k * dt, alpha, wc, temp))
        assert abs(rho[0, 1] - expect) < 1e-12
        assert abs(rho[0, 0] - 0.5) < 1e-12


@pytest.mark.parametrize("n", [3, 4])
def test_ising_zz_chain_closed_form(n):
    jz, alpha, wc, temp, dt, m = 1.3, 0.1, 4.0, 1.0, 0.15, 5
    plus = 0.5 * np.array([[1, 1], [1, 1]], dtype=np.complex128)
    bonds = [0.25 * jz * np.kron(SZ, SZ)] * (n - 1)
    wl = W.make_chain("ising", n, bonds, [0.0] * n, [plus] * n, dt, m,
                      [W.bath(s, alpha, wc, temp, m - 1) for s in range(n)],
                      chi_max=4 ** n, xi_max=4 ** m, eps=1e-13)
    prob, _ = problem_from_workload(wl, form="tempo", n_steps=m)
    eng = pt_tebd.Engine(prob)
    for k in range(1, m + 1):
        eng.step()
        g = cf.g_closed_form_exp(k * dt, alpha, wc, temp)
        for s in range(n):
            nb = (s > 0) + (s < n - 1)
            assert abs(eng.expectation(s, SX) - cf.ising_zz_sigma_x(jz, k * dt, nb, g)) < 1e-10


def test_correlation_special_cases():
    wl = W.random_small_chain(60, 3, with_bath_sites=(0,), k_cut=3, eps=1e-12)
    prob, _ = problem_from_workload(wl, form="tempo", n_steps=8)
    eng = pt_tebd.Engine(prob)
    eng.step(2)
    # C(0) = <B A>
    c = eng.correlate(1, SX, 1, SX, 0)
    assert abs(c[0] - 1.0) < 1e-12
    c = eng.correlate(0, SY, 2, SZ, 0)
    assert abs(c[0] - _two_point(eng, 0, SY, 2, SZ)) < 1e-12
    # A = 1 gives the plain expectation value at later times
    c = eng.correlate(1, np.eye(2), 2, SZ, 3)
    ref = []
    probe = pt_tebd.Engine(prob)
    probe.mps = eng.mps.copy()
    for j in range(4):
        ref.append(probe.expectation(2, SZ))
        probe.step()
    assert np.allclose(c, ref, atol=1e-12)
    assert eng.mps.step == 2   # the main state is untouched


def test_brute_force_correlation_matches_hilbert_space():
    # pin of BruteForce.correlate_multi on its own: a closed chain (no bath,
    # no GKSL terms) evolved with the exact propagator, against the
    # Heisenberg-picture two-point function Tr[B U(tau) A rho(t) U(tau)^dag]
    # (and Tr[B U (rho A) U^dag] for the right-acting insertion) computed in
    # Hilbert space from the eigendecomposition of H
    wl = W.random_small_chain(61, 3)
    n, dt = 3, wl["dt"]
    bf = brute.BruteForce(wl["h_site"], wl["h_bond"], wl["rho0"], dt, split="exact")
    bf.step(2)
    h = sum(lv.embed_site_operator(wl["h_site"][i], i, n, 2) for i in range(n))
    h = h + sum(lv.embed_bond_operator(wl["h_bond"][b], b, n, 2) for b in range(n - 1))
    w, v = np.linalg.eigh(h)

    def u(t):
        return (v * np.exp(-1j * w * t)) @ v.conj().T

    rho0 = wl["rho0"][0]
    for r in wl["rho0"][1:]:
        rho0 = np.kron(rho0, r)
    rho_t = u(2 * dt) @ rho0 @ u(2 * dt).conj().T
    a = lv.embed_site_operator(SX, 0, n, 2)
    b = lv.embed_site_operator(SZ, 2, n, 2)
    for side in ("L", "R"):
        c = bf.correlate_multi([(0, 0, SX, side)], 2, SZ, 5)
        x0 = a @ rho_t if side == "L" else rho_t @ a
        ref = [np.trace(b @ u(j * dt) @ x0 @ u(j * dt).conj().T) / np.trace(rho_t) for j in range(6)]
        assert np.abs(c - np.array(ref)).max() < 1e-12
    # three-time form: A at t, C at t + 2 dt, B read from t + 2 dt on
    cop = lv.embed_site_operator(SY, 1, n, 2)
    c = bf.correlate_multi([(0, 0, SX, "L"), (2, 1, SY, "L")], 2, SZ, 3)
    x2 = cop @ (u(2 * dt) @ (a @ rho_t) @ u(2 * dt).conj().T)
    ref = [np.trace(b @ u(j * dt) @ x2 @ u(j * dt).conj().T) / np.trace(rho_t) for j in range(4)]
    assert np.abs(c - np.array(ref)).max() < 1e-12


@pytest.mark.parametrize("n,bath_sites,k_cut", [(2, (0,), 3), (3, (0, 2), 2), (3, (1,), 3)])
def test_correlate_matches_brute_force_with_baths(n, bath_sites, k_cut):
    # Engine.correlate / correlate_multi against the dense augmented state
    # with the exact history PT-MPO, no truncation: insertions after a few
    # steps, propagated through later bath interactions
    m = 9
    wl = W.random_small_chain(62 + n, n, with_bath_sites=bath_sites, k_cut=k_cut, eps=1e-13)
    prob, _ = problem_from_workload(wl, form="history", n_steps=m)
    eng = pt_tebd.Engine(prob)
    baths = [{"site": b["site"], "coupling_op": b["coupling_op"],
              "eta": bath.eta_coefficients(b["alpha"], b["wc"], b["temperature"], wl["dt"], k_cut)}
             for b in wl["baths"]]
    bf = brute.BruteForce(wl["h_site"], wl["h_bond"], wl["rho0"], wl["dt"], baths=baths)
    eng.step(2)
    bf.step(2)
    c_gpu_form = eng.correlate(0, SX, n - 1, SZ, 5)
    c_ref = bf.correlate_multi([(0, 0, SX, "L")], n - 1, SZ, 5)
    assert np.abs(c_gpu_form - c_ref).max() < 1e-10
    assert abs(c_ref[0]) > 1e-3 or abs(c_ref[3]) > 1e-3   # a non-trivial correlation
    for ins in ([(0, n - 1, SY, "R")], [(0, 0, SX, "L"), (2, n - 1, SY, "L")],
                [(1, 0, SZ, "R"), (3, 0, SX, "L")]):
        c = eng.correlate_multi(ins, 0, SZ, 3)
        r = bf.correlate_multi(ins, 0, SZ, 3)
        assert np.abs(c - r).max() < 1e-10, ins
    assert eng.mps.step == 2 and bf.step_index == 2


def _two_point(eng, sa, a, sb, b):
    rho = eng.reduced_density_matrix()
    n = eng.mps.n_sites
    op = lv.embed_site_operator(b, sb, n, 2) @ lv.embed_site_operator(a, sa, n, 2)
    return np.trace(op @ rho) / np.trace(rho)


def test_trace_and_hermiticity_untruncated():
    wl = W.random_small_chain(70, 3, with_bath_sites=(1,), k_cut=3, eps=1e-13)
    prob, _ = problem_from_workload(wl, form="history", n_steps=6)
    eng = pt_tebd.Engine(prob)
    for _ in range(6):
        eng.step()
        rho = eng.reduced_density_matrix()
        assert abs(np.trace(rho) - 1.0) < 1e-12
        assert np.abs(rho - rho.conj().T).max() < 1e-12


def test_xy_chain_conserves_total_sz():
    # isotropic XY + z field + sigma^z baths: [H, S^z_tot] = 0 (Sec. IV)
    n = 6
    wl = W.make_chain("xy", n, [W.xyz_bond(1.0, 1.0, 0.0)] * (n - 1), [1.0] * n,
                      [W.DOWN] * 2 + [W.UP] + [W.DOWN] * 3, 0.1, 6,
                      [W.bath(s, 0.1, 4.0, 1.0, 3) for s in range(n)], chi_max=16, xi_max=16, eps=1e-7)
    prob, _ = problem_from_workload(wl)
    eng = pt_tebd.Engine(prob)
    for _ in range(6):
        eng.step()
        tot = sum(eng.expectation(s, SZ) for s in range(n))
        assert abs(tot - (-4.0)) < 1e-7


def test_truncation_error_shrinks_with_eps():
    wl = W.random_small_chain(80, 5, with_bath_sites=(0, 4), k_cut=3, eps=1e-12)
    prob_ref, cache = problem_from_workload(wl, form="tempo", n_steps=6)
    ref = pt_tebd.run(prob_ref, 6, [(s, SZ) for s in range(5)])["obs"]
    errs = []
    for eps in (1e-3, 1e-5, 1e-7):
        prob, _ = problem_from_workload(dict(wl, eps=eps), form="tempo", n_steps=6, pt_cache=cache)
        got = pt_tebd.run(prob, 6, [(s, SZ) for s in range(5)])["obs"]
        errs.append(np.abs(got - ref).max())
    assert errs[0] >= errs[1] >= errs[2]
    assert errs[2] < 1e-5


@pytest.mark.slow
def test_weak_coupling_relaxes_to_gibbs():
    # one spin, H = (e/2) sigma^z, coupled through sigma^x: the steady state
    # approaches the Gibbs state at the bath temperature with a deviation that
    # grows about linearly in alpha (Sec. III.A, weak-coupling comparison).
    # The inverted state (the Gibbs state of -H) is much further away: this
    # pins the sign of Im eta (a sign error relaxes towards the inverted state).
    e, temp, dt, k_cut, m = 1.0, 1.0, 0.25, 8, 60
    gibbs = cf.gibbs_state(0.5 * e * SZ, temp)
    inverted = cf.gibbs_state(-0.5 * e * SZ, temp)
    alphas = (0.02, 0.04, 0.08)
    dists, inv = [], []
    for alpha in alphas:
        wl = W.make_chain("gibbs", 1, [], [e], [W.UP], dt, m,
                          [W.bath(0, alpha, 4.0, temp, k_cut, coupling=SX)], chi_max=4,
                          xi_max=48, eps=1e-8, eps_tempo=1e-8)
        prob, _ = problem_from_workload(wl, n_steps=m)
        eng = pt_tebd.Engine(prob)
        eng.step(m)
        rho = eng.reduced_density_matrix()
        rho = rho / np.trace(rho)
        dists.append(cf.trace_distance(rho, gibbs))
        inv.append(cf.trace_distance(rho, inverted))
    assert dists[0] < dists[1] < dists[2]
    slope = np.polyfit(np.log(alphas), np.log(dists), 1)[0]
    assert 0.5 < slope < 1.3
    assert max(dists) < 0.2 * min(inv)
