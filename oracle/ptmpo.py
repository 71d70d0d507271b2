"""Process-tensor MPO (PT-MPO) of a Gaussian bath: influence functional,
exact history-form MPO, TEMPO-style compressed MPO and cap tensors.

Paper: the PT as a multilinear map stored as an MPO with bond dimension xi
(Sec. II.A; Appendix A.1, Fig. tensor-network-construction (b)); PT-MPOs of
Gaussian baths are built with PT-TEMPO with convergence parameters dt, the
memory cutoff Delta K_max and the truncation threshold eps_TEMPO (Appendix
B.1); caps remove the augmented leg by tracing later time slots (the
containment property, Appendix A.3, Fig. tensor-network-contraction (a,b)).

Conventions (our reading; the paper defers the construction to its refs):

* Work in the eigenbasis of the coupling operator S with eigenvalues sigma.
  A Liouville index x = i*d + j carries s+ = sigma_i and s- = sigma_j.
* Influence factor between the step-k index x and the step-(k-D) index x':
    b_D(x, x') = exp[-(s+ - s-)(eta_D s'+ - conj(eta_D) s'-)],   D >= 0,
  with the same-step factor b_0(x, x).
* Discretised influence functional with memory cutoff K:
    I(x_1..x_M) = prod_k prod_{D=0}^{min(K, k-1)} b_D(x_k, x_{k-D}).
* A PT-MPO tensor is P_k[e, e', x] (diagonal in the Liouville index in the
  eigenbasis of S), with xi_0 = xi_M = 1.  In the computational basis the
  tensor is W diag(P_k) W^dag with W = U kron conj(U), U the eigenvectors.
* Caps (backward recursion, our reading of the missing figure): c^(M) = [1],
  c^(k-1)[e] = sum_{e', s_out, s_in} P_k[e, e', s_out, s_in] t[s_out]
  (t[s_in]/d) c^(k)[e']  -- trace the output, feed the maximally mixed input.

Pinned by tests/test_oracle_ptmpo.py: the history MPO contracted over every
path equals the direct evaluation of I(x); the compressed MPO matches it to
~eps_TEMPO; alpha = 0 gives the identity with xi = 1; caps of the history
MPO are all-ones; the causality identity of the caps; the pure-dephasing
closed form of closed_forms.py.
"""
import itertools

import numpy as np


def liouville_charges(sigma):
    """(s+, s-) for each Liouville index x = i*d + j."""
    sigma = np.asarray(sigma, dtype=np.float64)
    d = sigma.shape[0]
    return np.repeat(sigma, d), np.tile(sigma, d)


def influence_matrix(eta_delta, sigma):
    """b[x, x'] = b_D(x, x') for one coefficient eta_D."""
    sp, sm = liouville_charges(sigma)
    return np.exp(-np.outer(sp - sm, eta_delta * sp - np.conj(eta_delta) * sm))


def influence_functional(path, eta, sigma):
    """Direct evaluation of I(x_1..x_M) for one path (list of Liouville
    indices); len(eta) - 1 is the memory cutoff K."""
    k_cut = len(eta) - 1
    b = [influence_matrix(eta[delta], sigma) for delta in range(k_cut + 1)]
    val = 1.0 + 0.0j
    for k in range(len(path)):
        val *= b[0][path[k], path[k]]
        for delta in range(1, min(k_cut, k) + 1):
            val *= b[delta][path[k], path[k - delta]]
    return val


def history_mpo(eta, sigma, n_steps):
    """Exact PT-MPO whose bond after step k holds the last min(k, K)
    Liouville indices (base-d^2 digits, most recent least significant).
    Returns a list of n_steps tensors P_k[e, e', x]."""
    k_cut = len(eta) - 1
    d2 = len(sigma) ** 2
    b = [influence_matrix(eta[delta], sigma) for delta in range(k_cut + 1)]
    tensors = []
    for k in range(1, n_steps + 1):
        m_in = min(k - 1, k_cut)
        m_out = 0 if k == n_steps else min(k, k_cut)
        xi_in, xi_out = d2 ** m_in, d2 ** m_out
        p = np.zeros((xi_in, xi_out, d2), dtype=np.complex128)
        for e in range(xi_in):
            digits = [(e // d2 ** j) % d2 for j in range(m_in)]  # digits[D-1] = x_{k-D}
            for x in range(d2):
                val = b[0][x, x]
                for delta in range(1, m_in + 1):
                    val *= b[delta][x, digits[delta - 1]]
                e_out = (x + d2 * e) % xi_out if xi_out > 1 else 0
                p[e, e_out, x] += val
        tensors.append(p)
    return tensors


def _truncation(sv, eps, cap):
    """Smallest rank with ||discarded||_2 < eps * max(sv), at most cap."""
    sv = sv[sv > 0.0]
    if sv.size == 0:
        return 1
    tail = np.sqrt(np.cumsum((sv ** 2)[::-1])[::-1])  # tail[c] = norm(sv[c:])
    rank = sv.size
    for c in range(1, sv.size):
        if tail[c] < eps * sv[0]:
            rank = c
            break
    return min(rank, cap) if cap else rank


def tempo_mpo(eta, sigma, n_steps, eps, xi_max=None):
    """TEMPO-style PT-MPO built forward in time.

    The PT is held as an MPS over time slots (physical leg x_k).  At step k a
    new slot with the same-step factor b_0 is appended, the couplings
    b_D(x_k, x_{k-D}) for D = 1..K are multiplied in through a bond-d^2 copy
    MPO that carries x_k back to slot k-K, and the window k-K..k is
    recompressed: right-to-left LQ sweep, then left-to-right truncated SVDs
    (threshold eps relative to the largest singular value, cap xi_max).
    Slots left of the window are final.  No scale factor is ever dropped.
    """
    k_cut = len(eta) - 1
    d2 = len(sigma) ** 2
    b = [influence_matrix(eta[delta], sigma) for delta in range(k_cut + 1)]
    mps = []  # tensors T[a, x, c]
    for k in range(1, n_steps + 1):
        new = np.zeros((1, d2, 1), dtype=np.complex128)
        new[0, :, 0] = np.diag(b[0])
        mps.append(new)
        m = min(k_cut, k - 1)
        if m == 0:
            continue
        last = len(mps) - 1
        # copy MPO: slot k emits x_k on a new bond of dim d2
        t = mps[last]
        a, _, c = t.shape
        out = np.zeros((a * d2, d2, c), dtype=np.complex128)
        for x in range(d2):
            out.reshape(a, d2, d2, c)[:, x, x, :] = t[:, x, :]
        mps[last] = out
        for delta in range(1, m + 1):
            j = last - delta
            t = mps[j]
            a, _, c = t.shape
            fac = b[delta]  # fac[x_k, x_j]
            if delta < m:
                out = np.zeros((a, d2, d2, c, d2), dtype=np.complex128)
                for xk in range(d2):
                    out[:, xk, :, :, xk] = t * fac[xk][None, :, None]
                mps[j] = out.reshape(a * d2, d2, c * d2)
                # layout: left bond (a, xk), right bond (c, xk)
            else:
                out = np.zeros((a, d2, c, d2), dtype=np.complex128)
                for xk in range(d2):
                    out[:, :, :, xk] = t * fac[xk][None, :, None]
                mps[j] = out.reshape(a, d2, c * d2)
        _recompress_window(mps, last - m, last, eps, xi_max)
    return [t.transpose(0, 2, 1).copy() for t in mps]  # P_k[e, e', x]


def _recompress_window(mps, lo, hi, eps, xi_max):
    # right-to-left LQ: make slots hi..lo+1 right-orthonormal
    for j in range(hi, lo, -1):
        t = mps[j]
        a, x, c = t.shape
        q, r = np.linalg.qr(t.reshape(a, x * c).conj().T)  # t^dag = q r -> t = r^dag q^dag
        mps[j] = q.conj().T.reshape(-1, x, c)
        mps[j - 1] = np.tensordot(mps[j - 1], r.conj().T, axes=([2], [0]))
    # left-to-right truncated SVD
    for j in range(lo, hi):
        t = mps[j]
        a, x, c = t.shape
        u, s, vh = np.linalg.svd(t.reshape(a * x, c), full_matrices=False)
        keep = _truncation(s, eps, xi_max)
        mps[j] = u[:, :keep].reshape(a, x, keep)
        sv = s[:keep, None] * vh[:keep]
        mps[j + 1] = np.tensordot(sv, mps[j + 1], axes=([1], [0]))


def to_computational_basis(tensors, coupling_op):
    """Dense P_k[e, e', s_out, s_in] in the computational basis for a general
    Hermitian coupling operator (eigenbasis tensors given as P_k[e, e', x])."""
    _, u = np.linalg.eigh(coupling_op)
    w = np.kron(u, u.conj())
    out = []
    for p in tensors:
        out.append(np.einsum("ax,efx,bx->efab", w, p, w.conj()))
    return out


def coupling_eigensystem(coupling_op):
    """(sigma, diagonal) for a coupling operator: for a diagonal operator the
    computational basis is kept (sigma = its diagonal), otherwise the eigh
    eigenbasis is used and the tensors must be rotated."""
    op = np.asarray(coupling_op, dtype=np.complex128)
    if np.allclose(op, np.diag(np.diag(op)), atol=0.0):
        return np.real(np.diag(op)).copy(), True
    sigma, _ = np.linalg.eigh(op)
    return sigma, False


def caps(tensors, d):
    """Cap vectors c^(0) .. c^(M) by backward recursion.  Accepts diagonal
    tensors P[e, e', x] or dense P[e, e', s_out, s_in]."""
    t = np.eye(d, dtype=np.complex128).reshape(-1)
    out = [None] * (len(tensors) + 1)
    out[-1] = np.ones(tensors[-1].shape[1], dtype=np.complex128)
    for k in range(len(tensors), 0, -1):
        p = tensors[k - 1]
        if p.ndim == 3:
            red = np.einsum("efx,x->ef", p, t * t / d)
        else:
            red = np.einsum("efab,a,b->ef", p, t, t / d)
        out[k - 1] = red @ out[k]
    return out


def contract_all_paths(tensors, d2):
    """Full contraction of a diagonal PT-MPO over every path (small M only):
    returns T[x_1, ..., x_M]."""
    acc = np.ones((1, 1), dtype=np.complex128)  # [paths, bond]
    for p in tensors:
        acc = np.einsum("pe,efx->pxf", acc, p).reshape(-1, p.shape[1])
    return acc[:, 0].reshape([d2] * len(tensors))


def all_paths(d2, n_steps):
    return itertools.product(range(d2), repeat=n_steps)
