"""Chain propagators of PT-TEBD (Appendix A.1).

The on-site system terms are absorbed into the nearest-neighbour couplings
(the K' definition of Appendix A.1): the first bond takes the whole first
site term plus half of the second, the last bond half of the second-to-last
plus the whole last site term, every other bond half of each neighbour.
Readings where the paper is silent or ambiguous:

* N = 2: both special cases apply to the single bond; it takes both site
  terms in full (K' = K + H_1 + H_2).
* N = 1: there is no bond; each chain half-step is the single-site propagator
  exp(L^S dt/2).
* GKSL terms of a site are shared between its bonds with the same weights as
  the site Hamiltonian.
* Second-order splitting among the chain sites (Appendix A.1, last paragraph
  of the construction): each chain half-step exp(L_chain dt/2) becomes
  E(dt/4) O(dt/2) E(dt/4), with bonds numbered from 1; "even" bonds are
  2, 4, ... and act first, "odd" bonds 1, 3, ... act in the middle with the
  merged dt/2 gate.  With 0-based bond index b the odd bonds are b = 0, 2, 4
  and the even bonds b = 1, 3, 5.

Gates are computed with scipy.linalg.expm and returned in site-major order,
G[(s', t'), (s, t)] with s = i*d + j.

Pinned by tests/test_oracle_gates.py: the product of all gates at tau equal
to exp(L_chain tau) for commuting bond terms; N = 2 gate against the dense
expm of a kron-built two-site Liouvillian; trace preservation; Hermiticity
preservation; eigen-decomposition form for unitary gates.
"""
import numpy as np
import scipy.linalg

from . import liouville as lv


def site_weights(bond, n_sites):
    """Weights (w_left, w_right) with which the two site terms enter K'."""
    if n_sites == 2:
        return 1.0, 1.0
    if bond == 0:
        return 1.0, 0.5
    if bond == n_sites - 2:
        return 0.5, 1.0
    return 0.5, 0.5


def bond_liouvillian(h_site, h_bond, lindblad, bond, n_sites, d):
    """Two-site Liouvillian of K'_{b,b+1} (plus weighted GKSL terms),
    natural two-site order."""
    one = np.eye(d, dtype=np.complex128)
    wl, wr = site_weights(bond, n_sites)
    kp = (np.asarray(h_bond[bond], dtype=np.complex128)
          + wl * np.kron(h_site[bond], one)
          + wr * np.kron(one, h_site[bond + 1]))
    lsup = lv.hamiltonian_liouvillian(kp)
    if lindblad is not None:
        for l_op in lindblad[bond]:
            lsup = lsup + wl * lv.gksl_dissipator(np.kron(l_op, one))
        for l_op in lindblad[bond + 1]:
            lsup = lsup + wr * lv.gksl_dissipator(np.kron(one, l_op))
    return lsup


def site_liouvillian(h_site, lindblad, site):
    lsup = lv.hamiltonian_liouvillian(np.asarray(h_site[site], dtype=np.complex128))
    if lindblad is not None:
        for l_op in lindblad[site]:
            lsup = lsup + lv.gksl_dissipator(l_op)
    return lsup


def bond_tau(bond, dt):
    """Time argument of the gate on 0-based bond b: odd (1-based) bonds carry
    the merged dt/2 gate, even (1-based) bonds the dt/4 gates."""
    return dt / 2.0 if bond % 2 == 0 else dt / 4.0


def chain_gates(h_site, h_bond, lindblad, dt, d):
    """List of site-major gates, one per bond (each bond uses one tau only)."""
    n_sites = len(h_site)
    gates = []
    for b in range(n_sites - 1):
        lsup = bond_liouvillian(h_site, h_bond, lindblad, b, n_sites, d)
        lsm = lv.superop_to_site_major(lsup, d)
        gates.append(scipy.linalg.expm(lsm * bond_tau(b, dt)))
    return gates


def single_site_half_step(h_site, lindblad, dt):
    """N = 1 only: exp(L^S dt / 2)."""
    return scipy.linalg.expm(site_liouvillian(h_site, lindblad, 0) * (dt / 2.0))


def half_step_sublayers(n_sites):
    """The three sublayers of one chain half-step as lists of 0-based bonds:
    E (even, 1-based), O (odd, 1-based), E.  Empty sublayers are dropped."""
    even = [b for b in range(n_sites - 1) if b % 2 == 1]
    odd = [b for b in range(n_sites - 1) if b % 2 == 0]
    return [s for s in (even, odd, even) if s]
