"""Pins of the float64 FNO reference: hand-written backward vs central
finite differences, and the spectral layer vs an explicit DFT sum."""
import numpy as np
import pytest

from oracle import fno


@pytest.mark.parametrize("ny,nx,width,modes,layers", [(12, 12, 4, 3, 2), (8, 10, 3, 2, 3)])
def test_backward_matches_finite_differences(ny, nx, width, modes, layers):
    rng = np.random.default_rng(0)
    theta = fno.init_params(width, modes, layers, seed=1)
    x = rng.standard_normal((2, 2, ny, nx))
    t = rng.standard_normal((2, ny, nx))
    g, _ = fno.backward(theta, x, t, width, modes, layers)
    idx = rng.choice(theta.size, 60, replace=False)
    h = 1e-6
    for i in idx:
        e = np.zeros_like(theta)
        e[i] = h
        fd = (fno.loss(theta + e, x, t, width, modes, layers)
              - fno.loss(theta - e, x, t, width, modes, layers)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-7 * max(1.0, abs(fd)) + 1e-9, (i, fd, g[i])


def test_spectral_layer_equals_explicit_mode_sum():
    """K v = sum over retained modes of R-mixed coefficients, written out as
    explicit complex exponentials (c_kx = 1 for kx = 0, 2 otherwise)."""
    rng = np.random.default_rng(3)
    ny, nx, W, M = 8, 8, 2, 2
    v = rng.standard_normal((1, W, ny, nx))
    R = rng.standard_normal((W, W, 2 * M, M)) + 1j * rng.standard_normal((W, W, 2 * M, M))
    got = fno.spectral(v, R, M)
    yy, xx = np.meshgrid(np.arange(ny), np.arange(nx), indexing="ij")
    kys = list(range(M)) + list(range(ny - M, ny))
    ref = np.zeros((1, W, ny, nx))
    for o in range(W):
        for a, ky in enumerate(kys):
            for kx in range(M):
                coef = 0.0
                for i in range(W):
                    vh = np.sum(v[0, i] * np.exp(-2j * np.pi * (ky * yy / ny + kx * xx / nx)))
                    coef += vh * R[i, o, a, kx]
                c = 1.0 if kx == 0 else 2.0
                ref[0, o] += c * np.real(coef * np.exp(2j * np.pi * (ky * yy / ny + kx * xx / nx))) / (ny * nx)
    assert np.allclose(got, ref, atol=1e-12)


def test_parameter_count_and_layout():
    W, M, L = 32, 16, 4
    assert fno.n_params(W, M, L) == fno.init_params(W, M, L).size
    # about 2.1 million complex spectral weights in the benchmark network
    assert L * W * W * 2 * M * M == 2 ** 21


@pytest.mark.parametrize("nz,ny,nx,width,modes,layers", [(6, 8, 10, 3, 2, 2), (8, 6, 8, 2, 1, 3)])
def test_backward_matches_finite_differences_3d(nz, ny, nx, width, modes, layers):
    rng = np.random.default_rng(4)
    theta = fno.init_params(width, modes, layers, seed=2, ndim=3)
    assert theta.size == fno.n_params(width, modes, layers, ndim=3)
    x = rng.standard_normal((2, 2, nz, ny, nx))
    t = rng.standard_normal((2, nz, ny, nx))
    g, _ = fno.backward(theta, x, t, width, modes, layers)
    idx = rng.choice(theta.size, 60, replace=False)
    h = 1e-6
    for i in idx:
        e = np.zeros_like(theta)
        e[i] = h
        fd = (fno.loss(theta + e, x, t, width, modes, layers)
              - fno.loss(theta - e, x, t, width, modes, layers)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-7 * max(1.0, abs(fd)) + 1e-9, (i, fd, g[i])


def test_spectral_layer_3d_equals_explicit_mode_sum():
    """3D: kz and ky from {0..M-1} U {N-M..N-1}, kx from {0..M-1}, written out
    as explicit complex exponentials."""
    rng = np.random.default_rng(5)
    nz, ny, nx, W, M = 4, 6, 6, 2, 1
    v = rng.standard_normal((1, W, nz, ny, nx))
    R = rng.standard_normal((W, W, 2 * M, 2 * M, M)) + 1j * rng.standard_normal((W, W, 2 * M, 2 * M, M))
    got = fno.spectral(v, R, M)
    zz, yy, xx = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    kzs = list(range(M)) + list(range(nz - M, nz))
    kys = list(range(M)) + list(range(ny - M, ny))
    ref = np.zeros((1, W, nz, ny, nx))
    for o in range(W):
        for a, kz in enumerate(kzs):
            for b, ky in enumerate(kys):
                for kx in range(M):
                    ph = 2j * np.pi * (kz * zz / nz + ky * yy / ny + kx * xx / nx)
                    coef = sum(np.sum(v[0, i] * np.exp(-ph)) * R[i, o, a, b, kx] for i in range(W))
                    c = 1.0 if kx == 0 else 2.0
                    ref[0, o] += c * np.real(coef * np.exp(ph)) / (nz * ny * nx)
    assert np.allclose(got, ref, atol=1e-12)
