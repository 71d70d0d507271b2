"""Analytically solvable special cases used as pins (they are not part of
the method; every one is derived in its docstring).

All cases have a coupling operator that commutes with every chain term, so
the chain/environment splitting (eq. propagator-env) and the even/odd split
are exact, the system path in the coupling eigenbasis is constant, and the
discretised influence functional of a constant off-diagonal path
x = (up, down) (s+ = 1, s- = -1) is exp(-4 Re sum_{k >= k'} eta_{k k'}),
where the double sum over the discretisation triangle is G(M dt).  These hold
for any dt as long as the memory cutoff K >= M - 1 and nothing is truncated.
"""
import numpy as np
import scipy.special


def g_closed_form_exp(t, alpha, wc, temperature):
    """G(t) for J(w) = 2 alpha w exp(-w/wc):
    Im G = 2 alpha [arctan(wc t) - wc t]
    Re G = alpha ln(1 + wc^2 t^2) + 2 alpha ln[Gamma(1+x)^2 / |Gamma(1+x+iy)|^2]
    with x = T/wc, y = T t (the thermal part vanishes at T = 0).
    Derivation: Im part from int_0^inf e^{-w/wc} sin(wt)/w dw = arctan(wc t);
    Re part from coth(w/2T) = 1 + 2 sum_n e^{-n w/T} and
    int_0^inf e^{-a w}(1 - cos wt)/w dw = 1/2 ln(1 + t^2/a^2), summed with the
    product formula of |Gamma(1+x+iy)|^2 / Gamma(1+x)^2."""
    im = 2.0 * alpha * (np.arctan(wc * t) - wc * t)
    re = alpha * np.log1p((wc * t) ** 2)
    if temperature > 0.0:
        x = temperature / wc
        y = temperature * t
        lg_re = scipy.special.loggamma(1.0 + x)
        lg_c = scipy.special.loggamma(1.0 + x + 1j * y)
        re += 2.0 * alpha * (2.0 * lg_re - 2.0 * np.real(lg_c))
    return re + 1j * im


def im_g_gauss_zero_temperature(t, alpha, wc):
    """Im G(t) for J(w) = 2 alpha w exp(-w^2/wc^2) (independent of T):
    2 alpha [(pi/2) erf(wc t / 2) - (sqrt(pi)/2) wc t]."""
    return 2.0 * alpha * (0.5 * np.pi * scipy.special.erf(0.5 * wc * t)
                          - 0.5 * np.sqrt(np.pi) * wc * t)


def pure_dephasing_coherence(rho_ud0, h, t, g_of_t):
    """One spin, H_S = (h/2) sigma^z, coupling sigma^z:
    rho_{up,down}(t) = rho_{up,down}(0) exp(-i h t) exp(-4 Re G(t))."""
    return rho_ud0 * np.exp(-1j * h * t) * np.exp(-4.0 * np.real(g_of_t))


def ising_zz_sigma_x(jz, t, n_neighbours, g_of_t):
    """Chain H = sum_n J_z s^z_n s^z_{n+1} (s = sigma/2), a sigma^z bath on
    every site, initial |+>^N: each neighbour in a sigma^z eigenstate shifts
    the site's level splitting by +-J_z/2, averaging to cos(J_z t/2) per
    neighbour; the site's own bath multiplies its coherence by
    exp(-4 Re G(t)); neighbours' baths only touch their coherences, which
    the partial trace removes.
    <sigma^x_n(t)> = cos(J_z t / 2)^{n_neighbours} exp(-4 Re G(t))."""
    return np.cos(0.5 * jz * t) ** n_neighbours * np.exp(-4.0 * np.real(g_of_t))


def gibbs_state(h, temperature):
    w, v = np.linalg.eigh(h)
    p = np.exp(-(w - w.min()) / temperature)
    p /= p.sum()
    return (v * p) @ v.conj().T


def trace_distance(a, b):
    return 0.5 * np.sum(np.abs(np.linalg.eigvalsh(a - b)))
