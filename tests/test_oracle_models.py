"""Pins of the oracle's energies and chemical potentials (paper Sec. 2)."""
import numpy as np
import pytest

from oracle import models, spectral


def directional_fd(f, u, v, h):
    """Fourth-order central difference of h -> f(u + h v) at 0."""
    return (-f(u + 2 * h * v) + 8 * f(u + h * v) - 8 * f(u - h * v) + f(u - 2 * h * v)) / (12 * h)


MODELS = [
    ("pfc", dict(eps=0.25), 0.0, 0.3, (8, 8), (8.0, 8.0)),
    ("pfc", dict(eps=0.25), -0.25, 0.3, (9, 7), (10.0, 7.0)),
    ("fch", dict(eps=0.3, eta1=0.45, eta2=0.6, tau=0.0), -0.5, 0.3, (8, 8), (2.0, 2.0)),
    ("fch", dict(eps=0.3, eta1=0.45, eta2=0.6, tau=0.125), 0.1, 0.3, (7, 9), (2.0, 3.0)),
    ("fch", dict(eps=0.3, eta1=0.45, eta2=0.6, tau=0.125), 0.1, 0.3, (4, 6, 4), (2.0, 3.0, 2.0)),
]


@pytest.mark.parametrize("kind,params,mean,amp,shape,lengths", MODELS)
def test_mu_is_gradient_of_energy(kind, params, mean, amp, shape, lengths):
    """dE_N[v] = (mu_N(u), v)_N: mu_N is the discrete variational derivative."""
    g = spectral.Grid(shape, lengths)
    m = models.make_model(kind, **params)
    rng = np.random.default_rng(11)
    # smooth-ish random fields keep the FD truncation error small
    u = mean + amp * g.inv(g.fwd(rng.uniform(-1, 1, shape)) * np.exp(-0.05 * g.k2))
    for seed in range(3):
        v = np.random.default_rng(seed).standard_normal(shape)
        fd = directional_fd(lambda w: m.energy(g, w), u, v, 1e-3)
        an = g.inner(m.mu(g, u), v)
        assert abs(fd - an) <= 1e-8 * max(1.0, abs(an))


@pytest.mark.parametrize("tau", [0.0, 0.125, -0.3])
def test_double_well_derivatives(tau):
    """F' = (z^2 - 1)(z + tau) etc. are the derivatives of the printed F."""
    z = np.linspace(-2, 2, 41)
    h = 1e-4
    fd1 = (models.F(z + h, tau) - models.F(z - h, tau)) / (2 * h)
    fd2 = (models.dF(z + h, tau) - models.dF(z - h, tau)) / (2 * h)
    fd3 = (models.d2F(z + h, tau) - models.d2F(z - h, tau)) / (2 * h)
    assert np.allclose(fd1, models.dF(z, tau), atol=1e-7)
    assert np.allclose(fd2, models.d2F(z, tau), atol=1e-7)
    assert np.allclose(fd3, models.d3F(z, tau), atol=1e-7)
    # wells of the symmetric potential: F(+-1) = 0 for tau = 0, F(-1) = 0 always
    assert abs(models.F(-1.0, tau)) < 1e-15
    if tau == 0.0:
        assert abs(models.F(1.0, 0.0)) < 1e-15
        assert abs(models.F(0.0, 0.0) - 0.25) < 1e-15


def test_fch_mu_equals_system_form():
    """The reading of the FCH system: mu = (eps^2 Delta - F'' + eta1) omega + (eta1 - eta2) F'."""
    g = spectral.Grid((16, 16), (2 * np.pi, 2 * np.pi))
    m = models.FCH(0.2, 0.3, 0.5, 0.1)
    u = -0.3 + 0.2 * np.random.default_rng(2).uniform(-1, 1, g.shape)
    om = m.omega(g, u)
    alt = (m.eps ** 2 * g.lap(om) - models.d2F(u, m.tau) * om + m.eta1 * om
           + (m.eta1 - m.eta2) * models.dF(u, m.tau))
    assert np.allclose(m.mu(g, u), alt, atol=1e-11)


def test_pfc_energy_of_constant_state():
    """E_PFC(c) = |Omega| (c^4/4 + (1-eps) c^2/2) for a constant field."""
    g = spectral.Grid((8, 8), (5.0, 5.0))
    m = models.PFC(0.25)
    c = -0.3
    ref = 25.0 * (c ** 4 / 4 + 0.75 * c * c / 2)
    assert abs(m.energy(g, np.full(g.shape, c)) - ref) < 1e-13
