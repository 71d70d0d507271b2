"""Pins of oracle/bath.py: quadrature against closed forms."""
import numpy as np
import pytest

from oracle import bath, closed_forms as cf


@pytest.mark.parametrize("temperature", [0.0, 0.5, 1.6, 3.0])
def test_g_quadrature_matches_closed_form(temperature):
    for t in (0.05, 0.2, 1.0, 2.5, 6.0):
        q = bath.g_function(t, 0.08, 4.0, temperature)
        c = cf.g_closed_form_exp(t, 0.08, 4.0, temperature)
        assert abs(q - c) < 1e-12 * max(1.0, abs(c))


def test_g_zero_temperature_limit():
    t = 0.7
    assert abs(bath.g_function(t, 0.2, 3.0, 0.0).real - 0.2 * np.log1p((3.0 * t) ** 2)) < 1e-12


def test_gaussian_cutoff_imaginary_part():
    for t in (0.1, 0.6, 2.0):
        for temperature in (0.0, 1.6):
            q = bath.g_function(t, 0.32, 4.0, temperature, cutoff="gauss")
            assert abs(q.imag - cf.im_g_gauss_zero_temperature(t, 0.32, 4.0)) < 1e-12


def test_eta_is_second_difference_of_g():
    dt, k = 0.1, 6
    a, wc, temp = 0.16, 4.0, 2.0
    eta = bath.eta_coefficients(a, wc, temp, dt, k)
    g = [cf.g_closed_form_exp(j * dt, a, wc, temp) for j in range(k + 2)]
    assert abs(eta[0] - g[1]) < 1e-12
    for delta in range(1, k + 1):
        assert abs(eta[delta] - (g[delta + 1] - 2 * g[delta] + g[delta - 1])) < 1e-12


def test_eta_triangle_sum_is_g():
    dt, m = 0.1, 8
    eta = bath.eta_coefficients(0.08, 4.0, 1.6, dt, m - 1)
    total = sum((m - delta) * eta[delta] for delta in range(m))
    assert abs(total - cf.g_closed_form_exp(m * dt, 0.08, 4.0, 1.6)) < 1e-11


def test_correlation_function_high_temperature_real_part_positive():
    # C(0) = int J coth > 0 and Im C(0) = 0
    c0 = bath.correlation_function(0.0, 0.08, 4.0, 1.6)
    assert c0.real > 0 and abs(c0.imag) < 1e-14
