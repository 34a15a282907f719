"""Pins of the oracle's Fourier-collocation operators (paper Sec. 3.2)."""
import numpy as np
import pytest

from oracle import dft, spectral

CASES = [((8, 8), (1.0, 1.0)), ((6, 6), (2.0, 2.0)), ((12, 12), (3.0, 3.0)),
         ((8, 12), (2.0, 5.0)), ((7, 9), (1.5, 2.5)), ((4, 6, 8), (1.0, 2.0, 3.0))]


@pytest.mark.parametrize("shape,lengths", CASES)
@pytest.mark.parametrize("alpha", [1, 2, -1])
def test_operators_match_brute_force_sums(shape, lengths, alpha):
    """(-Delta_N)^alpha via FFT equals the explicit sums of eq. def:frac-Lap."""
    rng = np.random.default_rng(7)
    g = spectral.Grid(shape, lengths)
    w = rng.standard_normal(shape)
    ref = dft.apply_symbol(w, lengths, alpha)
    if alpha == 1:
        got = -g.lap(w)
    elif alpha == 2:
        got = g.bilap(w)
    else:
        got = g.inv_neg_lap(w)
    assert np.max(np.abs(got - ref)) <= 1e-12 * np.max(np.abs(ref))


@pytest.mark.parametrize("r", [(0, 1), (2, 3), (4, 0), (-4, 2), (4, 4), (-3, -4)])
def test_laplacian_of_grid_mode(r):
    """Delta_N cos(k.x) = -|k|^2 cos(k.x) for every grid mode, Nyquist included."""
    shape, lengths = (8, 8), (3.0, 5.0)
    g = spectral.Grid(shape, lengths)
    y, x = g.coords()
    ky, kx = 2 * np.pi * r[0] / lengths[0], 2 * np.pi * r[1] / lengths[1]
    w = np.cos(ky * y + kx * x)
    k2 = kx * kx + ky * ky
    assert np.allclose(g.lap(w), -k2 * w, rtol=0, atol=1e-12 * max(1.0, k2))
    assert np.allclose(g.bilap(w), k2 * k2 * w, rtol=0, atol=1e-12 * max(1.0, k2 * k2))


def test_inverse_laplacian_on_mean_zero_data():
    g = spectral.Grid((16, 8), (2.0, 1.0))
    w = np.random.default_rng(1).standard_normal((16, 8))
    assert np.allclose(-g.lap(g.inv_neg_lap(w)), g.proj0(w), atol=1e-12)
    assert abs(np.mean(g.inv_neg_lap(w))) < 1e-14


def test_inner_product_is_trapezoid_rule():
    """(1, 1)_N = |Omega| and (sin, sin)_N = |Omega| / 2 for a resolved mode."""
    g = spectral.Grid((10, 6), (4.0, 3.0))
    y, x = g.coords()
    one = np.ones(g.shape)
    assert abs(g.inner(one, one) - 12.0) < 1e-13
    s = np.sin(2 * np.pi * 2 * x / 3.0)
    assert abs(g.inner(s, s) - 6.0) < 1e-12


def test_negative_norm_matches_sum_over_modes():
    """||w||_{-1,N}^2 = (1/P) |Omega| sum_{r != 0} |w_hat(r)|^2 / |k|^2 (Parseval)."""
    shape, lengths = (8, 8), (2.0, 2.0)
    g = spectral.Grid(shape, lengths)
    w = np.random.default_rng(3).standard_normal(shape)
    what = np.fft.fftn(w)
    ky = 2 * np.pi * np.fft.fftfreq(8, 1 / 8) / 2.0
    K2 = ky[:, None] ** 2 + ky[None, :] ** 2
    nz = K2 > 0
    ref = 4.0 * np.sum(np.abs(what[nz]) ** 2 / K2[nz]) / 64 ** 2
    assert abs(g.neg_norm_sq(w) - ref) < 1e-12 * ref
