"""Plain PT-TEBD on an augmented MPS (Appendix A), complex128.

State (augmented MPS in Vidal form, Appendix A.1 last paragraph):
  Gamma_n[a, s, e, b]  a = left bond, s = Liouville index of site n (d^2),
                       e = augmented leg (bond of the site's PT-MPO, 1 if the
                       site has no bath), b = right bond
  lam[n]               bond vector left of site n; lam[0] = lam[N] = [1]
  log_scale            real; the represented vec(rho) is exp(log_scale) times
                       the contraction (our bookkeeping, the paper is silent)

One time step (eq. propagator-env with the chain half-steps split as in
Appendix A.1):  H(dt/2) -> absorb P_k on every bath site -> H(dt/2), where
H(dt/2) = E(dt/4) O(dt/2) E(dt/4) over bonds (see gates.py).

Two-site gate (Appendix A.2, Fig. tensor-network-contraction (c)-(h)):
  (c-d) B_L = lam_{n-1} Gamma_n  as (a,e) x (s,b);  B_R = Gamma_{n+1} lam_{n+1}
        as (b,t) x (f,c)
  (d-e) truncated SVDs B_L ~ U_L S_L V_L^dag, B_R ~ U_R S_R V_R^dag (eps only)
  (e-f) D[l,s',t',r] = sum_{s,t,b} (S_L V_L^dag)[l,s,b] lam_n[b]
                       G[s't',st] (U_R S_R)[b,t,r]
  (f-g) truncated SVD of D as (l,s') x (t',r): eps rule, then the chi_max cap
  (g-h) Gamma_n' = lam_{n-1}^-1 U_L U^D, Gamma_{n+1}' = V^D^dag V_R^dag lam_{n+1}^-1
  The new bond vector is S^D / ||S^D||_2 and log ||S^D||_2 goes to log_scale.

Truncation (Appendix A.2): the smallest rank with the 2-norm of the
discarded singular values strictly below eps times the largest.  Readings:
exact zeros are never kept, the rank is at least 1, the eps rule comes first
and the chi_max cap second.  Where a cut falls inside a run of singular
values whose neighbours are within a relative gap of 1e-6, the kept subspace
is not a well-defined function of the matrix: a backward-stable SVD with
unit roundoff u turns the kept and discarded vectors of a pair with
relative gap g into each other by an angle of order u / (g sigma_r /
sigma_1), which moves the truncated state by about u sigma_1 / g.  Such runs
are therefore kept or dropped whole: an eps cut inside one moves to its end
(the discarded tail only shrinks, so the eps condition still holds) and a
cap that splits one moves to its start.  Without this, two LAPACK drivers
(gesdd and gesvd) following the minimal rule end up 6e-6 apart in
<sigma^z> on the N = 5 workload within 60 steps; with it they agree to
3e-12 (tests/test_oracle_truncation.py).

PT absorption (Appendix A.2, Fig. tensor-network-contraction (i)-(j)):
  Gamma_n[a,s,e',b] <- sum_{e, s_in} P_k[e,e',s,s_in] Gamma_n[a,s_in,e,b].

Observables (Appendix A.3, Fig. tensor-network-contraction (k)-(l)): contract
the cap c^(k) into each bath site, then <O_n> = Tr[O_n rho] / Tr rho, with
Tr[O rho] = vec(O^T) . vec(rho).

Two-time correlations (Appendix A.4, eq. two-time-corr-decomposed): the
left super-operator A.  is applied to a copy of the full augmented state,
which is propagated with its own log_scale; C(j) = Tr[B X(t + j dt)] /
Tr rho(t) (never normalised by the trace of X).

Pinned by tests/test_oracle_pt_tebd.py against brute.py (dense full
Liouville space with the bath history kept explicitly), the zero-coupling
dense expm, and the closed forms of closed_forms.py.
"""
import copy

import numpy as np

from . import gates as gt
from . import liouville as lv


TIE_TOLERANCE = 1e-6  # relative gap below which neighbouring singular values form one run


def truncation_rank(sv, eps, chi_max=None, tie=TIE_TOLERANCE):
    """Truncated rank for descending singular values ``sv`` (Appendix A.2);
    tie = 0 gives the minimal rank without the run reading."""
    sv = np.asarray(sv, dtype=np.float64)
    n_pos = int(np.count_nonzero(sv > 0.0))
    if n_pos == 0:
        return 1
    sv = sv[:n_pos]
    tail = np.sqrt(np.cumsum((sv ** 2)[::-1])[::-1])  # tail[c] = ||sv[c:]||
    rank = n_pos
    for c in range(1, n_pos):
        if tail[c] < eps * sv[0]:
            rank = c
            break
    # an eps cut inside a run moves to the run's end
    while rank < n_pos and sv[rank - 1] - sv[rank] < tie * sv[rank - 1]:
        rank += 1
    if chi_max is not None and rank > chi_max:
        rank = chi_max
        # a cap that splits a run moves to the run's start
        while rank > 1 and sv[rank - 1] - sv[rank] < tie * sv[rank - 1]:
            rank -= 1
    return rank


class AugmentedMPS:
    def __init__(self, rho0, d, initial=None):
        """Product initial state; ``initial`` maps a bath site to its initial
        augmented tensor R[s, e] for a chain site initially correlated with
        its environment (Appendix A.1: augmented legs of dimension > 1 at the
        start), which replaces that site's rho0."""
        self.d = d
        self.d2 = d * d
        self.n_sites = len(rho0)
        self.gammas = [lv.vec(r).reshape(1, self.d2, 1, 1).copy() for r in rho0]
        for site, r in (initial or {}).items():
            r = np.asarray(r, dtype=np.complex128)
            self.gammas[site] = r.reshape(1, self.d2, r.shape[-1], 1).copy()
        self.lams = [np.ones(1) for _ in range(self.n_sites + 1)]
        self.log_scale = 0.0
        self.step = 0

    def copy(self):
        return copy.deepcopy(self)

    def bond_dims(self):
        return [lam.shape[0] for lam in self.lams[1:-1]]

    def xi_dims(self):
        return [g.shape[2] for g in self.gammas]


def svd(mat, driver="gesdd"):
    """Thin SVD by LAPACK: numpy's default divide-and-conquer driver, or
    scipy's gesvd (QR iteration), a second correct implementation used to
    measure how far two LAPACK drivers' trajectories drift apart."""
    if driver == "gesdd":
        return np.linalg.svd(mat, full_matrices=False)
    import scipy.linalg
    return scipy.linalg.svd(mat, full_matrices=False, lapack_driver=driver)


def two_site_update(mps, bond, gate, eps, chi_max, stats=None, driver="gesdd", tie=TIE_TOLERANCE):
    """Appendix A.2 sequence (c)-(h) on sites bond, bond+1."""
    d2 = mps.d2
    g_l, g_r = mps.gammas[bond], mps.gammas[bond + 1]
    lam_l, lam_c, lam_r = mps.lams[bond], mps.lams[bond + 1], mps.lams[bond + 2]
    a, _, e, b = g_l.shape
    _, _, f, c = g_r.shape

    # (c-d)
    b_l = (lam_l[:, None, None, None] * g_l).transpose(0, 2, 1, 3).reshape(a * e, d2 * b)
    b_r = (g_r * lam_r[None, None, None, :]).reshape(b * d2, f * c)

    # (d-e)
    u_l, s_l, vh_l = svd(b_l, driver)
    n_l = truncation_rank(s_l, eps, tie=tie)
    u_r, s_r, vh_r = svd(b_r, driver)
    n_r = truncation_rank(s_r, eps, tie=tie)
    x_mat = (s_l[:n_l, None] * vh_l[:n_l]).reshape(n_l, d2, b)      # [l, s, b]
    y_mat = (u_r[:, :n_r] * s_r[None, :n_r]).reshape(b, d2, n_r)    # [b, t, r]

    # (e-f)
    x_lam = x_mat * lam_c[None, None, :]
    pair = np.einsum("lsb,btr->lstr", x_lam, y_mat)                 # [l, s, t, r]
    gate4 = gate.reshape(d2, d2, d2 * d2)                           # [s', t', (s,t)]
    d_ten = np.einsum("uvk,lkr->luvr", gate4, pair.reshape(n_l, d2 * d2, n_r))
    d_mat = d_ten.reshape(n_l * d2, d2 * n_r)

    # (f-g)
    u_d, s_d, vh_d = svd(d_mat, driver)
    chi = truncation_rank(s_d, eps, chi_max, tie=tie)
    norm = np.linalg.norm(s_d[:chi])
    mps.lams[bond + 1] = s_d[:chi] / norm
    mps.log_scale += np.log(norm)

    # (g-h)
    new_l = (u_l[:, :n_l] @ u_d[:, :chi].reshape(n_l, d2 * chi)).reshape(a, e, d2, chi)
    new_l = new_l / lam_l[:, None, None, None]
    mps.gammas[bond] = new_l.transpose(0, 2, 1, 3).copy()
    new_r = (vh_d[:chi].reshape(chi * d2, n_r) @ vh_r[:n_r]).reshape(chi, d2, f, c)
    mps.gammas[bond + 1] = new_r / lam_r[None, None, None, :]

    if stats is not None:
        stats.append({"bond": bond, "l": n_l, "r": n_r, "chi": chi,
                      "discarded": float(np.linalg.norm(s_d[chi:]) / s_d[0])})


def two_site_update_theta(mps, bond, gate, eps, chi_max):
    """Slow reference form of the same update: build the full two-site theta,
    apply the gate and split it with one truncated SVD (the textbook TEBD
    step that the (c)-(h) sequence reorganises)."""
    d2 = mps.d2
    g_l, g_r = mps.gammas[bond], mps.gammas[bond + 1]
    lam_l, lam_c, lam_r = mps.lams[bond], mps.lams[bond + 1], mps.lams[bond + 2]
    a, _, e, _ = g_l.shape
    _, _, f, c = g_r.shape
    theta = np.einsum("a,asez,z,ztfc,c->aestfc", lam_l, g_l, lam_c, g_r, lam_r)
    gate4 = gate.reshape(d2, d2, d2, d2)
    theta = np.einsum("uvst,aestfc->aeuvfc", gate4, theta)
    mat = theta.reshape(a * e * d2, d2 * f * c)
    u, s, vh = np.linalg.svd(mat, full_matrices=False)
    chi = truncation_rank(s, eps, chi_max)
    norm = np.linalg.norm(s[:chi])
    mps.lams[bond + 1] = s[:chi] / norm
    mps.log_scale += np.log(norm)
    new_l = u[:, :chi].reshape(a, e, d2, chi) / lam_l[:, None, None, None]
    mps.gammas[bond] = new_l.transpose(0, 2, 1, 3).copy()
    mps.gammas[bond + 1] = vh[:chi].reshape(chi, d2, f, c) / lam_r[None, None, None, :]


def apply_site_superop(mps, site, sop):
    """Gamma_n[a,s,e,b] <- sum_{s''} sop[s,s''] Gamma_n[a,s'',e,b]."""
    mps.gammas[site] = np.einsum("st,atez->asez", sop, mps.gammas[site])


def absorb_pt(mps, site, tensor):
    """Appendix A.2 (i)-(j): the PT-MPO bond becomes the new augmented leg."""
    g = mps.gammas[site]
    if tensor.ndim == 3:   # diagonal P[e, e', s]
        mps.gammas[site] = np.einsum("efs,asez->asfz", tensor, g)
    else:                  # dense P[e, e', s_out, s_in]
        mps.gammas[site] = np.einsum("efst,atez->asfz", tensor, g)


class Problem:
    """Explicit inputs of one chain (arrays only; no physics parameters)."""

    def __init__(self, h_site, h_bond, rho0, dt, baths=(), lindblad=None,
                 chi_max=None, eps=1e-7, d=2):
        self.d = d
        self.h_site = [np.asarray(h, dtype=np.complex128) for h in h_site]
        self.h_bond = [np.asarray(h, dtype=np.complex128) for h in h_bond]
        self.rho0 = [np.asarray(r, dtype=np.complex128) for r in rho0]
        self.dt = float(dt)
        self.lindblad = lindblad
        self.chi_max = chi_max
        self.eps = float(eps)
        # bath: dict(site=int, tensors=[P_k], caps=[c_k] or None)
        self.baths = []
        for bath in baths:
            caps = bath.get("caps")
            if caps is None:
                from .ptmpo import caps as make_caps
                caps = make_caps(bath["tensors"], d)
            self.baths.append({"site": int(bath["site"]), "tensors": bath["tensors"], "caps": caps,
                               "initial": bath.get("initial")})
        self.n_sites = len(self.h_site)
        if self.n_sites > 1:
            self.gates = gt.chain_gates(self.h_site, self.h_bond, lindblad, self.dt, d)
        else:
            self.site_prop = gt.single_site_half_step(self.h_site, lindblad, self.dt)


class Engine:
    def __init__(self, problem, mode="ch", svd_driver="gesdd", tie=TIE_TOLERANCE):
        self.p = problem
        self.mode = mode
        self.svd_driver = svd_driver
        self.tie = tie
        self.mps = AugmentedMPS(problem.rho0, problem.d,
                                {b["site"]: b["initial"] for b in problem.baths if b.get("initial") is not None})
        self.stats = []

    def _gate(self, mps, bond):
        if self.mode == "ch":
            two_site_update(mps, bond, self.p.gates[bond], self.p.eps, self.p.chi_max, self.stats,
                            self.svd_driver, self.tie)
        else:
            two_site_update_theta(mps, bond, self.p.gates[bond], self.p.eps, self.p.chi_max)

    def _half_step(self, mps):
        if self.p.n_sites == 1:
            apply_site_superop(mps, 0, self.p.site_prop)
            return
        for sublayer in gt.half_step_sublayers(self.p.n_sites):
            for bond in sublayer:
                self._gate(mps, bond)

    def step_state(self, mps):
        """One full time step k -> k+1 of eq. propagator-env."""
        self._half_step(mps)
        k = mps.step + 1
        for bath in self.p.baths:
            absorb_pt(mps, bath["site"], bath["tensors"][k - 1])
        self._half_step(mps)
        mps.step = k

    def step(self, n=1):
        for _ in range(n):
            self.step_state(self.mps)

    def capped_sites(self, mps):
        """Gamma-hat_n[a, s, b] with the cap of the current step contracted."""
        caps = {bath["site"]: bath["caps"][mps.step] for bath in self.p.baths}
        out = []
        for n, g in enumerate(mps.gammas):
            cap = caps.get(n, np.ones(g.shape[2], dtype=np.complex128))
            out.append(np.einsum("asez,e->asz", g, cap))
        return out

    def contract(self, mps, site_vectors):
        """sum over the chain of lam_0 G^_0(v_0) lam_1 ... lam_N times
        exp(log_scale), with v_n the vector contracted into site n."""
        hats = self.capped_sites(mps)
        left = np.ones(1, dtype=np.complex128)
        log_acc = mps.log_scale
        for n, h in enumerate(hats):
            left = (left * mps.lams[n]) @ np.einsum("asz,s->az", h, site_vectors[n])
            # keep the running vector at unit scale; its scale goes to the
            # logarithm (the chain's log-scale and the tensors' own growth
            # can each exceed the double range although their product does not)
            nrm = np.abs(left).max()
            if nrm > 0.0:
                left = left / nrm
                log_acc += np.log(nrm)
        left = left * mps.lams[-1]
        return np.exp(log_acc) * left.sum()

    def trace(self, mps=None):
        mps = self.mps if mps is None else mps
        t = lv.trace_vector(self.p.d)
        return self.contract(mps, [t] * mps.n_sites)

    def expectation(self, site, op, mps=None):
        """Tr[op_site rho] / Tr rho."""
        mps = self.mps if mps is None else mps
        t = lv.trace_vector(self.p.d)
        vecs = [t] * mps.n_sites
        vecs[site] = lv.observable_vector(op)
        return self.contract(mps, vecs) / self.trace(mps)

    def reduced_density_matrix(self, mps=None):
        """Full chain density matrix (natural order) from the capped MPS;
        small chains only."""
        mps = self.mps if mps is None else mps
        hats = self.capped_sites(mps)
        acc = np.ones((1, 1), dtype=np.complex128)  # [physical, bond]
        for n, h in enumerate(hats):
            acc = np.einsum("pa,a,asz->psz", acc, mps.lams[n], h).reshape(-1, h.shape[2])
        vec_sm = np.exp(mps.log_scale) * (acc @ mps.lams[-1])
        perm = lv.chain_natural_to_site_major(mps.n_sites, self.p.d)
        vec_nat = np.empty_like(vec_sm)
        vec_nat[perm] = vec_sm
        dim = self.p.d ** mps.n_sites
        return vec_nat.reshape(dim, dim)

    def correlate(self, site_a, op_a, site_b, op_b, n_steps):
        """C(j) = Tr[B X(t + j dt)] / Tr rho(t), j = 0..n_steps, where
        X(t) = A rho(t) is propagated from a copy of the augmented state."""
        return self.correlate_multi([(0, site_a, op_a, "L")], site_b, op_b, n_steps)

    def correlate_multi(self, insertions, site_b, op_b, n_steps):
        """Multi-time correlation of eq. two-time-corr-decomposed, from the
        current step t: a copy X of the augmented state is propagated, and
        at step offset m_p (non-decreasing, m_1 >= 0) the super-operator of
        C_p acts on site n_p, from the left (C rho, side "L") or, for
        out-of-time-ordered correlations, from the right (rho C, side "R").
        insertions = [(m_p, n_p, C_p, side_p), ...].  Returns
        out[j] = Tr[B X(t + (m_P + j) dt)] / Tr rho(t), j = 0..n_steps, with
        m_P the last offset.  Never normalised by the trace of X."""
        tr0 = self.trace()
        fork = self.mps.copy()
        t = lv.trace_vector(self.p.d)
        vecs = [t] * fork.n_sites
        vecs[site_b] = lv.observable_vector(op_b)
        offset = 0
        for m, site, op, side in insertions:
            if m < offset:
                raise ValueError("insertion offsets must be non-decreasing")
            for _ in range(m - offset):
                self.step_state(fork)
            offset = m
            op = np.asarray(op, dtype=np.complex128)
            sop = lv.left_mult(op) if side == "L" else lv.right_mult(op)
            apply_site_superop(fork, site, sop)
        out = [self.contract(fork, vecs) / tr0]
        for _ in range(n_steps):
            self.step_state(fork)
            out.append(self.contract(fork, vecs) / tr0)
        return np.array(out)


def run(problem, n_steps, observables, mode="ch"):
    """Propagate n_steps and record <op_site> for each (site, op) in
    ``observables`` plus Tr rho at steps 0..n_steps."""
    eng = Engine(problem, mode)
    obs = np.zeros((n_steps + 1, len(observables)), dtype=np.complex128)
    trace = np.zeros(n_steps + 1, dtype=np.complex128)
    chis = []

    def record(k):
        trace[k] = eng.trace()
        for i, (site, op) in enumerate(observables):
            obs[k, i] = eng.expectation(site, op)
        chis.append(eng.mps.bond_dims())

    record(0)
    for k in range(1, n_steps + 1):
        eng.step(1)
        record(k)
    return {"obs": obs, "trace": trace, "chi": chis, "engine": eng}
