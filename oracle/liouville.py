"""Liouville-space conventions (Appendix A.1; the paper leaves the vectorisation
order unspecified, so the reading below is ours).

* Basis of one spin-1/2: index 0 = up, 1 = down; sigma^z = diag(1, -1);
  spin operators s^gamma = sigma^gamma / 2 (Sec. III, XYZ chain Hamiltonian).
* Row-major vectorisation: vec(rho)[i*d + j] = rho[i, j].  Then
  A rho B  ->  (A kron B^T) vec(rho).
* Hamiltonian part of a Liouvillian: -i[H, .] -> -i (H kron 1 - 1 kron H^T).
* GKSL part (Appendix A.1, GKSL extension of the system Liouvillian):
  L rho L^dag - 1/2 {L^dag L, rho}
  -> L kron conj(L) - 1/2 (L^dag L kron 1 + 1 kron (L^dag L)^T).
* Two-site objects are built in the natural order of the two-site density
  matrix, row index (i_n i_{n+1}), column index (j_n j_{n+1}), and then
  permuted to the site-major Liouville order (i_n j_n)(i_{n+1} j_{n+1}) that
  the MPS legs use.

Pinned by tests/test_oracle_liouville.py (sandwich identity against explicit
matrix products, trace preservation, Hermiticity preservation, permutation
against an explicit partial-trace construction).
"""
import numpy as np

SIGMA_X = np.array([[0, 1], [1, 0]], dtype=np.complex128)
SIGMA_Y = np.array([[0, -1j], [1j, 0]], dtype=np.complex128)
SIGMA_Z = np.array([[1, 0], [0, -1]], dtype=np.complex128)
IDENTITY2 = np.eye(2, dtype=np.complex128)


def vec(rho):
    """Row-major vectorisation of a square matrix."""
    return np.asarray(rho, dtype=np.complex128).reshape(-1)


def unvec(v, d):
    return np.asarray(v, dtype=np.complex128).reshape(d, d)


def sandwich(a, b):
    """Super-operator of rho -> a rho b."""
    return np.kron(a, b.T)


def left_mult(a):
    """Super-operator of rho -> a rho (left-acting C^L of Appendix A.4)."""
    return sandwich(a, np.eye(a.shape[0], dtype=np.complex128))


def right_mult(a):
    """Super-operator of rho -> rho a (right-acting C^R of Appendix A.4)."""
    return sandwich(np.eye(a.shape[0], dtype=np.complex128), a)


def hamiltonian_liouvillian(h):
    """-i[h, .] in row-major Liouville space."""
    one = np.eye(h.shape[0], dtype=np.complex128)
    return -1j * (np.kron(h, one) - np.kron(one, h.T))


def gksl_dissipator(l_op):
    """L . L^dag - 1/2 {L^dag L, .} in row-major Liouville space."""
    one = np.eye(l_op.shape[0], dtype=np.complex128)
    ldl = l_op.conj().T @ l_op
    return np.kron(l_op, l_op.conj()) - 0.5 * (np.kron(ldl, one) + np.kron(one, ldl.T))


def trace_vector(d):
    """t with t . vec(rho) = Tr rho."""
    return vec(np.eye(d))


def observable_vector(op):
    """o with o . vec(rho) = Tr[op rho] = sum_ij op[j, i] rho[i, j]."""
    return vec(np.asarray(op, dtype=np.complex128).T)


def two_site_natural_to_site_major(d):
    """Permutation p such that v_site_major = v_natural[p].

    Natural index:     ((i1 * d + i2) * d*d) + (j1 * d + j2)
    Site-major index:  ((i1 * d + j1) * d*d) + (i2 * d + j2)
    """
    p = np.empty(d ** 4, dtype=np.int64)
    for i1 in range(d):
        for j1 in range(d):
            for i2 in range(d):
                for j2 in range(d):
                    sm = ((i1 * d + j1) * d * d) + (i2 * d + j2)
                    nat = ((i1 * d + i2) * d * d) + (j1 * d + j2)
                    p[sm] = nat
    return p


def superop_to_site_major(sop, d):
    """Re-index a two-site super-operator from natural to site-major order."""
    p = two_site_natural_to_site_major(d)
    return sop[np.ix_(p, p)]


def chain_natural_to_site_major(n_sites, d):
    """Permutation for an N-site density matrix: natural (i_1..i_N, j_1..j_N)
    row-major vec -> site-major (i_1 j_1, ..., i_N j_N)."""
    dims_nat = [d] * (2 * n_sites)
    idx = np.arange(d ** (2 * n_sites)).reshape(dims_nat)
    order = []
    for n in range(n_sites):
        order += [n, n_sites + n]
    return idx.transpose(order).reshape(-1)


def embed_site_operator(op, site, n_sites, d):
    """op acting on one site of an N-site chain (Hilbert space)."""
    out = np.eye(1, dtype=np.complex128)
    for n in range(n_sites):
        out = np.kron(out, op if n == site else np.eye(d, dtype=np.complex128))
    return out


def embed_bond_operator(op2, bond, n_sites, d):
    """Two-site operator (natural order) acting on sites bond, bond+1."""
    out = np.eye(d ** bond, dtype=np.complex128)
    out = np.kron(out, op2)
    return np.kron(out, np.eye(d ** (n_sites - bond - 2), dtype=np.complex128))
