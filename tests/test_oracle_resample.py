"""Pins of the oracle's band-limited change of grid (the reference of the
learned guess's resampling between the solver's grid and a network's
coarser grid): exact on trigonometric polynomials inside the band, zero on
modes outside it, interpolation back to the fine grid inverts sampling for
band-limited fields, and the mean is kept."""
import numpy as np
import pytest

from oracle import fno as ofno


def trig(shape, terms):
    ny, nx = shape
    y, x = np.meshgrid(np.arange(ny) / ny, np.arange(nx) / nx, indexing="ij")
    out = np.zeros(shape)
    for a, ky, kx, ph in terms:
        out += a * np.cos(2 * np.pi * (ky * y + kx * x) + ph)
    return out


IN_BAND = [(0.3, 0, 0, 0.0), (1.0, 3, -5, 0.4), (0.5, -7, 2, 1.1), (0.25, 7, 7, -0.3)]


@pytest.mark.parametrize("fine,coarse", [((64, 32), (16, 16)), ((48, 64), (16, 32)), ((32, 32), (32, 32))])
def test_samples_band_limited_fields_exactly(fine, coarse):
    f = trig(fine, IN_BAND)
    c = ofno.band_resample(f, coarse)
    assert np.max(np.abs(c - trig(coarse, IN_BAND))) <= 1e-13


def test_drops_modes_outside_the_band():
    fine, coarse = (64, 64), (16, 16)
    out = [(1.0, 8, 0, 0.0), (1.0, 0, -8, 0.3), (0.7, 9, 3, 0.2), (0.4, 3, 20, 0.0)]  # |k| >= 16/2
    c = ofno.band_resample(trig(fine, IN_BAND + out), coarse)
    assert np.max(np.abs(c - trig(coarse, IN_BAND))) <= 1e-13


def test_interpolation_back_inverts_sampling_in_band():
    fine, coarse = (64, 48), (16, 16)
    f = trig(fine, IN_BAND)
    back = ofno.band_resample(ofno.band_resample(f, coarse), fine)
    assert np.max(np.abs(back - f)) <= 1e-13


def test_mean_is_kept():
    rng = np.random.default_rng(3)
    f = rng.uniform(-1, 1, (64, 32)) + 0.37
    c = ofno.band_resample(f, (16, 8))
    assert abs(c.mean() - f.mean()) <= 1e-14
    assert abs(ofno.band_resample(c, (64, 32)).mean() - f.mean()) <= 1e-14
