"""Pins of the oracle's fluctuation and dissipation spectra (oracle/fdt.py,
Sec. III.A and Appendix B.2).

* A damped two-level correlation C(tau) = p_u exp((i w0 - g) tau)
  + p_d exp((-i w0 - g) tau) has closed-form transforms: S(w) is a sum of
  two Lorentzians of weight 1 at +-w0 and chi''(w) their difference scaled
  by -(p_u - p_d); the trapezoid sums must reproduce them to O(dt^2).
* The paper's own check: a spin coupled to one thermal bath relaxes to a
  state whose auto-correlation obeys the fluctuation-dissipation theorem,
  S/chi'' = coth(w / 2T), i.e. the effective temperature T(w) equals the
  bath temperature (up to the discretisation of the influence functional).
"""
import numpy as np

from oracle import fdt
from oracle import pt_tebd as opt
from oracle.build import problem_from_workload
from paper_2201_05529_amd import workloads as W


def _lorentz(g, x):
    return g / (g * g + x * x)


def test_spectra_match_closed_form_lorentzians():
    w0, g, dt = 2.0, 0.5, 0.005
    beta = 0.7
    pu, pd = np.exp(-beta * w0 / 2), np.exp(beta * w0 / 2)
    pu, pd = pu / (pu + pd), pd / (pu + pd)
    tau = dt * np.arange(int(70.0 / dt) + 1)        # exp(-g tau_max) ~ 6e-16
    c = pu * np.exp((1j * w0 - g) * tau) + pd * np.exp((-1j * w0 - g) * tau)
    om = np.array([0.3, 1.0, 1.7, 2.0, 2.4, 3.5])
    s, chi = fdt.spectra(c, dt, om)
    s_ref = _lorentz(g, w0 - om) + _lorentz(g, w0 + om)
    chi_ref = -(pu - pd) * (_lorentz(g, w0 - om) - _lorentz(g, w0 + om))
    assert np.abs(s - s_ref).max() < 1e-4 * np.abs(s_ref).max()
    assert np.abs(chi - chi_ref).max() < 1e-4 * np.abs(chi_ref).max()
    # a narrow line of a thermal two-level system: S/chi'' -> coth at w0
    gn = 0.02
    tau = dt * np.arange(int(1800.0 / dt) + 1)
    c = pu * np.exp((1j * w0 - gn) * tau) + pd * np.exp((-1j * w0 - gn) * tau)
    s, chi = fdt.spectra(c, dt, np.array([w0]))
    assert abs(s[0] / chi[0] - 1.0 / np.tanh(beta * w0 / 2)) < 1e-3


def test_single_bath_steady_state_obeys_fdt():
    # H = (w0/2) sigma^z, bath coupled through sigma^x (so the spin
    # exchanges energy with it), relaxed for 20 time units; C(tau) of
    # sigma^x over a further 20 (it has decayed to ~5e-5 of C(0))
    w0, temp, dt = 1.0, 1.0, 0.2
    wl = W.make_chain("fdt1", 1, [], [w0], [W.UP], dt=dt, n_steps=200,
                      baths=[W.bath(0, 0.05, 4.0, temp, 10, coupling=W.SX)], chi_max=4, xi_max=32, eps=1e-9,
                      eps_tempo=1e-7)
    prob, _ = problem_from_workload(wl)
    eng = opt.Engine(prob)
    eng.step(100)
    c = eng.correlate(0, W.SX, 0, W.SX, 100)
    assert abs(c[0] - 1.0) < 1e-12 and np.abs(c[-10:]).max() < 1e-3
    om = np.linspace(0.2, 2.0, 10)
    s, chi = fdt.spectra(c, dt, om)
    assert (s > 0).all() and (chi > 0).all()
    t_eff = fdt.effective_temperature(om, s, chi)
    assert np.abs(t_eff / temp - 1.0).max() < 0.08
