"""Pins of the oracle's time-discretisation coefficients (paper Sec. 3.1)."""
import numpy as np
import pytest

from oracle import schemes


@pytest.mark.parametrize("dt_new,dt_old", [(0.1, 0.1), (0.2, 0.05), (0.013, 0.07)])
def test_bdf2_differentiates_quadratics_exactly(dt_new, dt_old):
    """Variable-step BDF2 is exact on quadratics: a p(t+) + b p(t) + c p(t-) = p'(t+)."""
    a, b, c, theta = schemes.coefficients(schemes.BDF2, dt_new, dt_old)
    assert theta == 1.0
    t = 0.7
    tm, tp = t - dt_old, t + dt_new
    for p, dp in ((lambda s: 1.0 + 0 * s, lambda s: 0.0),
                  (lambda s: s, lambda s: 1.0),
                  (lambda s: 3 * s * s - s, lambda s: 6 * s - 1)):
        assert abs(a * p(tp) + b * p(t) + c * p(tm) - dp(tp)) < 1e-10 * (1 + abs(a))


def test_constant_step_bdf2_and_first_step():
    a, b, c, _ = schemes.coefficients(schemes.BDF2, 0.5, 0.5)
    assert np.allclose([a, b, c], [3.0, -4.0, 1.0])  # (3/2, -2, 1/2) / dt
    a, b, c, th = schemes.coefficients(schemes.BDF2, 0.5, None)
    assert (a, b, c, th) == (2.0, -2.0, 0.0, 1.0)     # backward Euler


def test_midpoint_coefficients():
    a, b, c, th = schemes.coefficients(schemes.MP, 0.25, 0.1)
    assert (a, b, c, th) == (4.0, -4.0, 0.0, 0.5)


@pytest.mark.parametrize("scheme", [schemes.BDF2, schemes.MP])
def test_coefficients_sum_to_zero(scheme):
    """Constants are steady states: a + b + c = 0."""
    for dn, do in ((0.1, 0.1), (0.3, 0.1), (0.01, 0.5)):
        a, b, c, _ = schemes.coefficients(scheme, dn, do)
        assert abs(a + b + c) < 1e-12 * abs(a)


def test_extrapolation_is_exact_for_linear_histories():
    t_n, dt_old, dt_new = 1.0, 0.2, 0.35
    f = lambda t: 2.0 - 3.0 * t
    x = schemes.extrapolate(np.array([f(t_n)]), np.array([f(t_n - dt_old)]), dt_new, dt_old)
    assert abs(x[0] - f(t_n + dt_new)) < 1e-14
    first = schemes.extrapolate(np.array([1.5]), None, dt_new, None)
    assert first[0] == 1.5
