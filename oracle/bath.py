"""Gaussian bosonic bath: spectral density, correlation function and the
discretised influence coefficients eta_Delta.

Paper: the bath Hamiltonian with linear coupling through a system operator
(Sec. III.A, eq. bosonic-bath; Sec. IV, eq. bosonic-bath-XY), the ohmic
spectral density J(w) = 2 alpha w exp(-w^2/wc^2) with a Gaussian cutoff
(Sec. III.A), and the bath correlation function C(tau) of Appendix B.1.
The workloads of this library use the exponential cutoff
J(w) = 2 alpha w exp(-w/wc); both are supported (``cutoff='exp'|'gauss'``).

The paper defers the time discretisation of the bath influence to the
PT-TEMPO literature.  Our reading (piecewise-constant system path over each
step of length dt, which is exact for the symmetric chain/environment
splitting of eq. propagator-env when the coupling operator commutes with the
bath's own system term):

  G(t)    = int_0^inf dw J(w)/w^2 [coth(w/2T)(1 - cos wt) + i (sin wt - wt)]
          = int_0^t dt' int_0^t' dt'' C(t'')
  eta_0   = G(dt)                                        (same step)
  eta_D   = int_0^inf dw J(w) 2(1 - cos w dt)/w^2
              [coth(w/2T) cos(w D dt) - i sin(w D dt)]    (D >= 1)
          = G((D+1)dt) - 2 G(D dt) + G((D-1)dt)

All integrals here are done by adaptive quadrature (scipy.integrate.quad).

Pinned by tests/test_oracle_bath.py: closed form of G for the exponential
cutoff (complex log-gamma), the T -> 0 limit, the Gaussian-cutoff imaginary
part (error function), the second-difference identity for eta_D, and
sum over the discretisation triangle = G(M dt).
"""
import numpy as np
import scipy.integrate


def spectral_density(w, alpha, wc, cutoff="exp"):
    w = np.asarray(w, dtype=np.float64)
    if cutoff == "exp":
        return 2.0 * alpha * w * np.exp(-w / wc)
    if cutoff == "gauss":
        return 2.0 * alpha * w * np.exp(-(w / wc) ** 2)
    raise ValueError(cutoff)


def _upper_limit(wc, cutoff):
    return wc * (60.0 if cutoff == "exp" else 7.5)


def _coth_half(w, temperature):
    if temperature <= 0.0:
        return 1.0
    return 1.0 / np.tanh(w / (2.0 * temperature))


def _quad(f, w_max, t_scale):
    """Adaptive quadrature of f over (0, w_max), split into pieces no wider
    than one oscillation period of the widest time argument."""
    n_pieces = int(np.ceil(w_max * max(t_scale, 1.0) / np.pi)) + 1
    edges = np.linspace(0.0, w_max, n_pieces + 1)
    total = 0.0
    for lo, hi in zip(edges[:-1], edges[1:]):
        val, _ = scipy.integrate.quad(f, lo, hi, limit=200, epsabs=1e-16, epsrel=1e-14)
        total += val
    return total


def correlation_function(tau, alpha, wc, temperature, cutoff="exp"):
    """C(tau) of Appendix B.1 (bath correlation function)."""
    w_max = _upper_limit(wc, cutoff)

    def re(w):
        return spectral_density(w, alpha, wc, cutoff) * np.cos(w * tau) * _coth_half(w, temperature)

    def im(w):
        return -spectral_density(w, alpha, wc, cutoff) * np.sin(w * tau)

    return _quad(re, w_max, tau) + 1j * _quad(im, w_max, tau)


def g_function(t, alpha, wc, temperature, cutoff="exp"):
    """G(t): twice-integrated bath correlation function."""
    w_max = _upper_limit(wc, cutoff)

    def re(w):
        if w == 0.0:
            return 0.0
        jw2 = spectral_density(w, alpha, wc, cutoff) / (w * w)
        return jw2 * _coth_half(w, temperature) * 2.0 * np.sin(0.5 * w * t) ** 2

    def im(w):
        if w == 0.0:
            return 0.0
        jw2 = spectral_density(w, alpha, wc, cutoff) / (w * w)
        return jw2 * (np.sin(w * t) - w * t)

    return _quad(re, w_max, t) + 1j * _quad(im, w_max, t)


def eta_coefficients(alpha, wc, temperature, dt, k_max, cutoff="exp"):
    """eta_Delta for Delta = 0 .. k_max (memory cutoff K = k_max)."""
    w_max = _upper_limit(wc, cutoff)
    eta = np.zeros(k_max + 1, dtype=np.complex128)
    eta[0] = g_function(dt, alpha, wc, temperature, cutoff)
    for delta in range(1, k_max + 1):
        def re(w, delta=delta):
            if w == 0.0:
                return 0.0
            pref = spectral_density(w, alpha, wc, cutoff) * 4.0 * np.sin(0.5 * w * dt) ** 2 / (w * w)
            return pref * _coth_half(w, temperature) * np.cos(w * delta * dt)

        def im(w, delta=delta):
            if w == 0.0:
                return 0.0
            pref = spectral_density(w, alpha, wc, cutoff) * 4.0 * np.sin(0.5 * w * dt) ** 2 / (w * w)
            return -pref * np.sin(w * delta * dt)

        t_scale = (delta + 1) * dt
        eta[delta] = _quad(re, w_max, t_scale) + 1j * _quad(im, w_max, t_scale)
    return eta
