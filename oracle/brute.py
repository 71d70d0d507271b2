"""Dense full-Liouville-space references (small chains only).

These share the physics conventions of the oracle (row-major vec, site-major
MPS index, same gate schedule, same influence factors) but none of the MPS
machinery: the whole chain density matrix is one dense vector of length
d^(2N), and each bath's recent history of Liouville indices is kept as
explicit extra tensor axes (an i-QUAPI style augmented density tensor).
With no truncation this is what PT-TEBD with the exact history PT-MPO must
reproduce, which pins the two-site update, the PT absorption, the caps and
the observables of pt_tebd.py.

* ``dense_chain_liouvillian``: L_chain = sum_n L^S_n + sum_n L^K_{n,n+1}
  (Appendix A.1) built with kron products in the natural order and permuted
  to site-major order.
* ``exact_evolution``: exp(L_chain t) vec(rho0), the Markovian/zero-coupling
  reference (Sec. II.A: without a PT the network is TEBD in Liouville space).
* ``BruteForce``: step-by-step propagation with the same splitting as the
  PT-TEBD schedule (or the exact chain half-step propagator), bath factors
  applied in the coupling eigenbasis.

It is pinned on its own terms in tests/test_oracle_pt_tebd.py: the
zero-coupling dense expm of an independently built Liouvillian, and the
closed forms of closed_forms.py (through the PT-TEBD runs it must match).
``BruteForce.correlate_multi`` inserts left- or right-acting single-site
super-operators into the dense augmented state (eq.
two-time-corr-decomposed); its own pin is a two-point function of a
bath-free chain evaluated as Tr[B e^{L t} A rho] with the dense propagator.
"""
import numpy as np
import scipy.linalg

from . import gates as gt
from . import liouville as lv
from . import ptmpo


def dense_chain_liouvillian(h_site, h_bond, lindblad, d):
    """Site-major L_chain for the whole chain (4^N x 4^N for spins)."""
    n_sites = len(h_site)
    dim = d ** n_sites
    h_tot = np.zeros((dim, dim), dtype=np.complex128)
    for n in range(n_sites):
        h_tot += lv.embed_site_operator(np.asarray(h_site[n], dtype=np.complex128), n, n_sites, d)
    for b in range(n_sites - 1):
        h_tot += lv.embed_bond_operator(np.asarray(h_bond[b], dtype=np.complex128), b, n_sites, d)
    lsup = lv.hamiltonian_liouvillian(h_tot)
    if lindblad is not None:
        for n in range(n_sites):
            for l_op in lindblad[n]:
                lsup = lsup + lv.gksl_dissipator(lv.embed_site_operator(l_op, n, n_sites, d))
    perm = lv.chain_natural_to_site_major(n_sites, d)
    return lsup[np.ix_(perm, perm)]


def product_state_vector(rho0):
    v = np.ones(1, dtype=np.complex128)
    for r in rho0:
        v = np.kron(v, lv.vec(r))
    return v


def exact_evolution(h_site, h_bond, lindblad, rho0, t, d):
    lsup = dense_chain_liouvillian(h_site, h_bond, lindblad, d)
    return scipy.linalg.expm(lsup * t) @ product_state_vector(rho0)


class BruteForce:
    """Dense augmented state psi[s_0..s_{N-1}, history axes].

    baths: list of dict(site, eta (array K+1), coupling_op (d x d Hermitian)).
    split: 'trotter' applies the PT-TEBD gate schedule, 'exact' applies
    exp(L_chain dt/2) for each chain half-step.
    """

    def __init__(self, h_site, h_bond, rho0, dt, baths=(), lindblad=None,
                 d=2, split="trotter"):
        self.d, self.d2 = d, d * d
        self.n_sites = len(h_site)
        self.dt = dt
        self.split = split
        self.psi = product_state_vector(rho0).reshape([self.d2] * self.n_sites)
        self.labels = [("site", n) for n in range(self.n_sites)]
        self.baths = []
        for i, bath in enumerate(baths):
            op = np.asarray(bath["coupling_op"], dtype=np.complex128)
            sigma, u = np.linalg.eigh(op)
            w = np.kron(u, u.conj())     # eigenbasis vec -> computational vec
            eta = np.asarray(bath["eta"], dtype=np.complex128)
            b = [ptmpo.influence_matrix(eta[k], sigma) for k in range(len(eta))]
            self.baths.append({"id": i, "site": bath["site"], "w": w, "b": b,
                               "k_cut": len(eta) - 1, "hist": 0})
        self.step_index = 0
        if split == "trotter":
            if self.n_sites > 1:
                self.gates = gt.chain_gates(h_site, h_bond, lindblad, dt, d)
            else:
                self.site_prop = gt.single_site_half_step(h_site, lindblad, dt)
        else:
            lsup = dense_chain_liouvillian(h_site, h_bond, lindblad, d)
            self.half = scipy.linalg.expm(lsup * (dt / 2.0))

    # -- axis helpers ---------------------------------------------------------
    def _axis(self, label):
        return self.labels.index(label)

    def _apply_on_axes(self, mat, labels):
        """psi <- mat applied on the listed axes (mat acts on their product)."""
        axes = [self._axis(lab) for lab in labels]
        k = len(axes)
        rest = [i for i in range(self.psi.ndim) if i not in axes]
        t = np.transpose(self.psi, axes + rest)
        shape = t.shape
        t = mat @ t.reshape(self.d2 ** k, -1)
        t = t.reshape(shape)
        inv = np.argsort(axes + rest)
        self.psi = np.transpose(t, inv)

    def _half_step(self):
        if self.split == "exact":
            shape = self.psi.shape
            order = [self._axis(("site", n)) for n in range(self.n_sites)]
            rest = [i for i in range(self.psi.ndim) if i not in order]
            t = np.transpose(self.psi, order + rest)
            tshape = t.shape
            t = (self.half @ t.reshape(self.d2 ** self.n_sites, -1)).reshape(tshape)
            self.psi = np.transpose(t, np.argsort(order + rest))
            assert self.psi.shape == shape
            return
        if self.n_sites == 1:
            self._apply_on_axes(self.site_prop, [("site", 0)])
            return
        for sublayer in gt.half_step_sublayers(self.n_sites):
            for bond in sublayer:
                self._apply_on_axes(self.gates[bond], [("site", bond), ("site", bond + 1)])

    def _bath_step(self, bath):
        site_lab = ("site", bath["site"])
        self._apply_on_axes(bath["w"].conj().T, [site_lab])     # to eigenbasis
        ax = self._axis(site_lab)
        shape = [1] * self.psi.ndim
        shape[ax] = self.d2
        self.psi = self.psi * np.diag(bath["b"][0]).reshape(shape)
        for delta in range(1, bath["hist"] + 1):
            hax = self._axis(("hist", bath["id"], delta))
            shape = [1] * self.psi.ndim
            shape[ax] = self.d2
            shape[hax] = self.d2
            fac = bath["b"][delta]
            if ax > hax:
                fac = fac.T
            self.psi = self.psi * fac.reshape(shape)
        # forget the oldest entry once it has met its last partner
        if bath["hist"] == bath["k_cut"] and bath["k_cut"] > 0:
            hax = self._axis(("hist", bath["id"], bath["k_cut"]))
            self.psi = self.psi.sum(axis=hax)
            del self.labels[hax]
            bath["hist"] -= 1
        # shift history labels and record the current index
        if bath["k_cut"] > 0:
            for delta in range(bath["hist"], 0, -1):
                i = self._axis(("hist", bath["id"], delta))
                self.labels[i] = ("hist", bath["id"], delta + 1)
            ax = self._axis(site_lab)
            copy = np.zeros((self.d2, self.d2))
            np.fill_diagonal(copy, 1.0)
            self.psi = np.expand_dims(self.psi, -1)
            self.labels.append(("hist", bath["id"], 1))
            shape = [1] * self.psi.ndim
            shape[ax] = self.d2
            shape[-1] = self.d2
            self.psi = self.psi * copy.reshape(shape)
            bath["hist"] += 1
        self._apply_on_axes(bath["w"], [site_lab])              # back

    def step(self, n=1):
        for _ in range(n):
            self._half_step()
            for bath in self.baths:
                self._bath_step(bath)
            self._half_step()
            self.step_index += 1

    def insert(self, site, op, side="L"):
        """Apply C rho (side "L") or rho C (side "R") on one site of the
        augmented state (every history axis is untouched)."""
        op = np.asarray(op, dtype=np.complex128)
        sop = lv.left_mult(op) if side == "L" else lv.right_mult(op)
        self._apply_on_axes(sop, [("site", site)])

    def correlate_multi(self, insertions, site_b, op_b, n_steps):
        """Same contract as the PT-TEBD oracle's correlate_multi: a copy of
        the dense augmented state receives the insertions (m_p, n_p, C_p,
        side_p) at step offsets m_p and is propagated; out[j] is
        Tr[B X] / Tr rho(t) at offset m_P + j."""
        import copy as _copy
        tr0 = self.trace()
        fork = _copy.deepcopy(self)
        offset = 0
        for m, site, op, side in insertions:
            fork.step(m - offset)
            offset = m
            fork.insert(site, op, side)
        out = []
        for j in range(n_steps + 1):
            if j:
                fork.step(1)
            out.append(fork.unnormalised(site_b, op_b) / tr0)
        return np.array(out)

    def unnormalised(self, site, op):
        """Tr[op_site X] without dividing by Tr X."""
        v = self.chain_vector().reshape([self.d2] * self.n_sites)
        t = lv.trace_vector(self.d)
        o = lv.observable_vector(op)
        for n in range(self.n_sites - 1, -1, -1):
            v = v @ (o if n == site else t)
        return v

    def chain_vector(self):
        """Site-major vec(rho_chain): every history axis summed (all-ones caps)."""
        order = [self._axis(("site", n)) for n in range(self.n_sites)]
        rest = tuple(i for i in range(self.psi.ndim) if i not in order)
        t = self.psi.sum(axis=rest) if rest else self.psi
        # remaining axes are the site axes in their current relative order
        remaining = [i for i in range(self.psi.ndim) if i in order]
        perm = [remaining.index(o) for o in order]
        return np.transpose(t, perm).reshape(-1)

    def expectation(self, site, op):
        v = self.chain_vector().reshape([self.d2] * self.n_sites)
        t = lv.trace_vector(self.d)
        o = lv.observable_vector(op)
        num = v
        den = v
        for n in range(self.n_sites - 1, -1, -1):
            num = num @ (o if n == site else t)
            den = den @ t
        return num / den

    def trace(self):
        v = self.chain_vector().reshape([self.d2] * self.n_sites)
        t = lv.trace_vector(self.d)
        for _ in range(self.n_sites):
            v = v @ t
        return v


def site_major_expectation(vec_sm, n_sites, site, op, d):
    v = np.asarray(vec_sm).reshape([d * d] * n_sites)
    t = lv.trace_vector(d)
    o = lv.observable_vector(op)
    num, den = v, v
    for n in range(n_sites - 1, -1, -1):
        num = num @ (o if n == site else t)
        den = den @ t
    return num / den
