"""Pins of the IMEX oracle (LBDF2, LMP; Sec. 3.1.1, eq.
eqn:FCH-semidis-simplicit).

* The splitting L + N reproduces the chemical potential (whose own pins are
  finite differences of the energy).
* One step on a single small Fourier mode about a steady state multiplies it
  by the closed-form linear factor (1 - dt M q (N' + (1 - theta) l)) /
  (1 + dt M q theta l), with N' = mu' - l from the linearised chemical
  potential.
* Second order in time (self-convergence), exact mass conservation.
"""
import math

import numpy as np
import pytest

from oracle import imex, models, spectral


def _fch(tau=0.0):
    return models.FCH(0.1, 0.145, 0.2, tau)


@pytest.mark.parametrize("kind,tau", [("pfc", 0.0), ("fch", 0.0), ("fch", 0.125)])
def test_splitting_reproduces_mu(kind, tau):
    g = spectral.Grid((12, 16), (3.0, 4.0) if kind == "fch" else (12.0, 16.0))
    m = models.PFC(0.25) if kind == "pfc" else _fch(tau)
    u = -0.3 + 0.4 * np.random.default_rng(5).uniform(-1, 1, g.shape)
    lhs = imex.linear_part(m, g, u) + imex.nonlinear_part(m, g, u)
    mu = m.mu(g, u)
    assert np.max(np.abs(lhs - mu)) <= 1e-11 * np.max(np.abs(mu))


def test_linear_symbols_as_printed():
    g = spectral.Grid((8, 8), (2 * math.pi, 2 * math.pi))  # integer wavenumbers
    q = g.k2
    assert np.allclose(imex.linear_symbol(models.PFC(0.25), g), (1 - q) ** 2, rtol=0, atol=1e-14)
    m = _fch(0.125)
    k0 = 1 - 2 * 0.125 ** 2 + 0.2
    assert np.allclose(imex.linear_symbol(m, g), 0.1 ** 4 * q * q + q + k0, rtol=1e-15, atol=1e-14)


def _mode(g, kx, ky, amp):
    y, x = g.coords()
    k = 2 * math.pi * np.array([ky / g.lengths[0], kx / g.lengths[1]])
    return amp * np.cos(k[1] * x + k[0] * y), float(k @ k)


@pytest.mark.parametrize("scheme", [imex.LBDF2, imex.LMP])
@pytest.mark.parametrize("kind", ["pfc", "fch"])
def test_single_mode_linear_factor(kind, scheme):
    """About u = 0 (a steady state of both models with tau = 0): PFC
    mu'(q) = (1 - q)^2 - eps; FCH mu'(q) = eps^4 q^2 + eps^2 q (2F''(0) - eta1)
    + F''(0)^2 - eta2 F''(0) with F''(0) = -1 (F'(0) = 0)."""
    if kind == "pfc":
        g = spectral.Grid((16, 16), (32.0, 32.0))
        m = models.PFC(0.25)
        dt = 0.3
        mu1 = lambda q: (1 - q) ** 2 - m.eps
    else:
        g = spectral.Grid((16, 16), (2.0, 2.0))
        m = _fch()
        dt = 1e-3
        e2 = m.eps ** 2
        mu1 = lambda q: e2 * e2 * q * q + e2 * q * (-2.0 - m.eta1) + 1.0 + m.eta2
    delta = 1e-7
    u0, q = _mode(g, 3, 2, delta)
    u1 = imex.step(m, g, scheme, u0, None, dt, None)
    # printed symbols: (1 - q)^2, and eps^4 q^2 + kappa2 q + kappa0 with
    # kappa2 = 1, kappa0 = 1 - 2 tau^2 + eta2 = 1.2
    l = (1 - q) ** 2 if kind == "pfc" else m.eps ** 4 * q * q + q + 1.2
    theta = 1.0 if scheme == imex.LBDF2 else 0.5
    nprime = mu1(q) - l
    factor = (1 - dt * q * (nprime + (1 - theta) * l)) / (1 + dt * q * theta * l)
    assert np.max(np.abs(u1 - factor * u0)) <= 1e-9 * delta


@pytest.mark.parametrize("scheme", [imex.LBDF2, imex.LMP])
def test_second_order_in_time(scheme):
    g = spectral.Grid((16, 16), (64.0, 64.0))
    m = models.PFC(0.25)
    u0 = -0.25 + 0.5 * np.random.default_rng(4).uniform(-1, 1, g.shape)
    T = 2.0
    sols = [imex.run(m, g, scheme, u0, T / n, n) for n in (16, 32, 64, 128)]
    e = [np.max(np.abs(sols[i + 1] - sols[i])) for i in range(3)]
    ratios = [e[0] / e[1], e[1] / e[2]]
    assert all(3.6 <= r <= 4.4 for r in ratios), ratios


@pytest.mark.parametrize("scheme", [imex.LBDF2, imex.LMP])
def test_mass_conserved(scheme):
    g = spectral.Grid((32, 32), (math.pi, math.pi))
    m = _fch()
    u0 = -0.6 + 0.01 * np.random.default_rng(0).uniform(-1, 1, g.shape)
    u = imex.run(m, g, scheme, u0, 1e-3, 10)
    assert abs(u.mean() - u0.mean()) <= 1e-14
