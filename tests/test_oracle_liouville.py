"""Pins of oracle/liouville.py: the super-operator constructions are checked
against explicit matrix products (not against the kron formulas)."""
import numpy as np

from oracle import liouville as lv

RNG = np.random.default_rng(1)


def rand_c(*shape):
    return RNG.normal(size=shape) + 1j * RNG.normal(size=shape)


def test_sandwich_matches_matrix_products():
    for d in (2, 3):
        a, b, rho = rand_c(d, d), rand_c(d, d), rand_c(d, d)
        assert np.allclose(lv.sandwich(a, b) @ lv.vec(rho), lv.vec(a @ rho @ b), atol=1e-13)


def test_hamiltonian_liouvillian_is_commutator():
    h = rand_c(2, 2)
    h = h + h.conj().T
    rho = rand_c(2, 2)
    assert np.allclose(lv.hamiltonian_liouvillian(h) @ lv.vec(rho),
                       lv.vec(-1j * (h @ rho - rho @ h)), atol=1e-13)


def test_gksl_dissipator_matches_definition():
    l_op, rho = rand_c(2, 2), rand_c(2, 2)
    ldl = l_op.conj().T @ l_op
    expect = l_op @ rho @ l_op.conj().T - 0.5 * (ldl @ rho + rho @ ldl)
    assert np.allclose(lv.gksl_dissipator(l_op) @ lv.vec(rho), lv.vec(expect), atol=1e-13)
    # trace preservation of the generator: t . (D vec rho) = 0
    assert abs(lv.trace_vector(2) @ (lv.gksl_dissipator(l_op) @ lv.vec(rho))) < 1e-13


def test_observable_vector_gives_trace():
    op, rho = rand_c(2, 2), rand_c(2, 2)
    assert np.isclose(lv.observable_vector(op) @ lv.vec(rho), np.trace(op @ rho))
    assert np.isclose(lv.trace_vector(2) @ lv.vec(rho), np.trace(rho))


def test_two_site_permutation_on_product_states():
    # a product state r1 (x) r2 in natural order must become the kron of the
    # site vectors in site-major order
    r1, r2 = rand_c(2, 2), rand_c(2, 2)
    natural = lv.vec(np.kron(r1, r2))
    p = lv.two_site_natural_to_site_major(2)
    assert np.allclose(natural[p], np.kron(lv.vec(r1), lv.vec(r2)))


def test_chain_permutation_on_product_states():
    rs = [rand_c(2, 2) for _ in range(3)]
    natural = lv.vec(np.kron(np.kron(rs[0], rs[1]), rs[2]))
    p = lv.chain_natural_to_site_major(3, 2)
    expect = np.kron(np.kron(lv.vec(rs[0]), lv.vec(rs[1])), lv.vec(rs[2]))
    assert np.allclose(natural[p], expect)


def test_site_major_superop_acts_like_partial_operator():
    # (A (x) 1) rho (B (x) 1) on a product state only touches site 1
    a, b = rand_c(2, 2), rand_c(2, 2)
    one = np.eye(2)
    sop = lv.superop_to_site_major(lv.sandwich(np.kron(a, one), np.kron(b, one)), 2)
    r1, r2 = rand_c(2, 2), rand_c(2, 2)
    got = sop @ np.kron(lv.vec(r1), lv.vec(r2))
    assert np.allclose(got, np.kron(lv.vec(a @ r1 @ b), lv.vec(r2)))
