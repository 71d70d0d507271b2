"""Fluctuation and dissipation spectra of a stationary auto-correlation
(Sec. III.A "Checking thermalization through the fluctuation-dissipation
theorem" and Appendix B.2 "Multi-time correlations and fluctuation and
dissipation spectra").  Test infrastructure: never imported by the library.

For a Hermitian observable A at a steady state, C(tau) = <A(tau) A(0)> is
known for tau >= 0 (one left insertion of A, then propagation).  The
stationarity argument of Appendix B.2 gives C(-tau) = C(tau)^*, so on the
symmetric interval (-tau_max, tau_max):
  * fluctuations  S_A(tau)   = 1/2 <{A(tau), A(0)}> = Re C(tau)   (even in tau)
  * response      chi_A(tau) = i Theta(tau) <[A(tau), A(0)]> = -2 Theta(tau) Im C(tau)
and the spectra are S_A(w) = FT[S_A](w) and chi''_A(w) = Im FT[chi_A](w)
with FT[f](w) = integral f(tau) exp(i w tau) dtau.  The FDT states
S_A(w) / chi''_A(w) = coth(w / 2T) for a thermal state at temperature T, so
T(w) = w / (2 artanh(chi''_A(w) / S_A(w))) is an effective temperature.

Reading (the paper names a fast Fourier transform on the interval but no
quadrature): the integral over [-n dt, n dt] is taken with the trapezoid
rule on the samples tau_j = j dt; evaluated at arbitrary frequencies, so
the two halves of the interval are summed explicitly below (no FFT grid).
"""
import numpy as np


def symmetric_samples(corr, dt):
    """tau_j = j dt for j = -n..n and the continued correlation there."""
    corr = np.asarray(corr, dtype=np.complex128)
    n = len(corr) - 1
    taus = dt * np.arange(-n, n + 1)
    full = np.concatenate([np.conj(corr[:0:-1]), corr])   # C(-tau) = C(tau)^*
    return taus, full


def trapezoid_weights(m):
    w = np.ones(m)
    if m > 1:
        w[0] = w[-1] = 0.5
    return w


def spectra(corr, dt, omegas):
    """S_A(w) and chi''_A(w) at the angular frequencies omegas from
    C(tau_j) = <A(tau_j) A(0)>, j = 0..n (tau_j = j dt)."""
    taus, full = symmetric_samples(corr, dt)
    w = trapezoid_weights(len(taus))
    s_tau = full.real                                 # 1/2 <{A(tau), A}> for all tau
    chi_tau = np.where(taus >= 0.0, -2.0 * full.imag, 0.0)   # i Theta(tau) <[A(tau), A]>
    # at tau = 0 the step function takes the half value of the trapezoid
    # rule's end point of the one-sided integral; Im C(0) = 0 for Hermitian A
    s_w, chi_w = [], []
    for om in np.atleast_1d(omegas):
        ph = np.exp(1j * om * taus)
        s_w.append(dt * np.sum(w * s_tau * ph).real)
        # chi is supported on tau >= 0: its trapezoid weights are those of
        # the half interval [0, n dt]
        half = taus >= 0.0
        wh = trapezoid_weights(int(half.sum()))
        chi_w.append((dt * np.sum(wh * chi_tau[half] * ph[half])).imag)
    return np.array(s_w), np.array(chi_w)


def effective_temperature(omegas, s_w, chi_w):
    """T(w) from S/chi'' = coth(w / 2T)."""
    return np.asarray(omegas) / (2.0 * np.arctanh(np.asarray(chi_w) / np.asarray(s_w)))
