"""Pin of the oracle's correlated initial states (Appendix A.1: the
augmented legs of the initial MPS have dimension > 1 when the chain and an
environment start correlated).

An environment that is one ancilla qubit has an exact PT-MPO: each tensor is
the joint propagator exp(L^E dt) of site and ancilla, with the ancilla's
Liouville index as the bond (the last tensor traces the ancilla out).  Start
site 0 and the ancilla in an entangled mixed state: the site's initial
augmented tensor is their joint vec(rho) with the ancilla index as the
augmented leg.  PT-TEBD with that tensor must equal the dense evolution of
chain plus ancilla under the same splitting (chain half-step, exp(L^E dt),
chain half-step), step by step.  A product start written the same way must
equal the ordinary uncorrelated run."""
import numpy as np
import scipy.linalg

from oracle import gates as gt
from oracle import liouville as lv
from oracle import pt_tebd as opt

SX = np.array([[0, 1], [1, 0]], dtype=np.complex128)
SZ = np.array([[1, 0], [0, -1]], dtype=np.complex128)
I2 = np.eye(2, dtype=np.complex128)


def ancilla_model(dt=0.1, m=8, g=0.7, wa=1.3):
    h_e = g * np.kron(SX, SX) + 0.5 * wa * np.kron(I2, SZ)
    e_sm = lv.superop_to_site_major(scipy.linalg.expm(lv.hamiltonian_liouvillian(h_e) * dt), 2)
    e4 = e_sm.reshape(4, 4, 4, 4)                   # [s_out, a_out, s_in, a_in]
    p = e4.transpose(3, 1, 0, 2).copy()             # P[a_in, a_out, s_out, s_in]
    t = lv.trace_vector(2)
    p_last = np.einsum("soti,o->ist", e4, t)[:, None, :, :]
    return [p] * (m - 1) + [p_last], e_sm


def joint_to_augmented(rho_joint):
    v = lv.vec(rho_joint)[lv.two_site_natural_to_site_major(2)]
    return v.reshape(4, 4)                          # R[s, a]


def chain():
    h_site = [0.5 * 0.4 * SZ, -0.5 * 0.3 * SZ]
    h_bond = [np.kron(SX, SX) + 0.8 * np.kron(SZ, SZ)]
    return h_site, h_bond


def brute(h_site, h_bond, r0, rho1, e_sm, dt, m):
    x = np.einsum("sa,t->sta", r0, lv.vec(rho1))     # [s0, s1, a]
    g = gt.chain_gates(h_site, h_bond, None, dt, 2)
    t = lv.trace_vector(2)
    o = lv.observable_vector(SZ)
    out = []

    def half(x):
        for sub in gt.half_step_sublayers(2):
            for b in sub:
                x = np.einsum("uv,vA->uA", g[b], x.reshape(16, 4)).reshape(4, 4, 4)
        return x

    for k in range(m + 1):
        if k:
            x = half(x)
            x = np.einsum("uv,vB->uB", e_sm, x.transpose(0, 2, 1).reshape(16, 4)).reshape(4, 4, 4).transpose(0, 2, 1)
            x = half(x)
        tr = np.einsum("sta,s,t,a->", x, t, t, t)
        out.append([np.einsum("sta,s,t,a->", x, o, t, t) / tr, np.einsum("sta,s,t,a->", x, t, o, t) / tr, tr])
    return np.array(out)


def run_oracle(h_site, h_bond, rho0, tensors, dt, m, initial=None):
    bath = {"site": 0, "tensors": tensors}
    if initial is not None:
        bath["initial"] = initial
    eng = opt.Engine(opt.Problem(h_site, h_bond, rho0, dt, baths=[bath], eps=1e-14))
    out = []
    for k in range(m + 1):
        if k:
            eng.step(1)
        out.append([eng.expectation(0, SZ), eng.expectation(1, SZ), eng.trace()])
    return np.array(out)


def test_correlated_start_matches_dense_evolution_with_the_ancilla():
    dt, m = 0.1, 8
    tensors, e_sm = ancilla_model(dt, m)
    phi = np.array([1, 0, 0, 1], dtype=np.complex128) / np.sqrt(2)
    rho_joint = 0.7 * np.outer(phi, phi.conj()) + 0.3 * np.eye(4) / 4
    r0 = joint_to_augmented(rho_joint)
    h_site, h_bond = chain()
    down = np.diag([0.0, 1.0]).astype(np.complex128)
    ref = brute(h_site, h_bond, r0, down, e_sm, dt, m)
    got = run_oracle(h_site, h_bond, [np.eye(2) / 2, down], tensors, dt, m, initial=r0)
    assert np.abs(got - ref).max() < 1e-12
    # the correlation matters: the marginals alone give another trajectory
    rho_s = np.trace(rho_joint.reshape(2, 2, 2, 2), axis1=1, axis2=3)
    rho_a = np.trace(rho_joint.reshape(2, 2, 2, 2), axis1=0, axis2=2)
    prod = brute(h_site, h_bond, np.outer(lv.vec(rho_s), lv.vec(rho_a)), down, e_sm, dt, m)
    assert np.abs(prod - ref).max() > 1e-3


def test_product_start_written_as_augmented_tensor_equals_the_ordinary_start():
    dt, m = 0.1, 6
    tensors, e_sm = ancilla_model(dt, m)
    rho_s = np.array([[0.8, 0.1j], [-0.1j, 0.2]])
    rho_a = np.array([[0.3, 0.2], [0.2, 0.7]], dtype=np.complex128)
    h_site, h_bond = chain()
    down = np.diag([0.0, 1.0]).astype(np.complex128)
    aug = run_oracle(h_site, h_bond, [np.eye(2) / 2, down], tensors, dt, m,
                     initial=np.outer(lv.vec(rho_s), lv.vec(rho_a)))
    # the ordinary form: the ancilla state absorbed into the first tensor
    first = np.einsum("i,iosa->osa", lv.vec(rho_a), tensors[0])[None]
    plain = run_oracle(h_site, h_bond, [rho_s, down], [first] + tensors[1:], dt, m)
    assert np.abs(aug - plain).max() < 1e-12
