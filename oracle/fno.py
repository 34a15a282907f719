"""Float64 Fourier neural operator: forward and hand-written backward.

TEST INFRASTRUCTURE ONLY (the reference for the GPU kernels' gradient
checks).  Not part of the paper: the learned warm start of the PAGD solve
predicts a correction to the extrapolated initial guess.

Network (width W, retained modes M per axis, L spectral layers), input
x[b, 2, Ny, Nx]:
    v0 = lift(x)            v0[b,o] = sum_i P[i,o] x[b,i] + pb[o]
    for l < L:
        s  = K_l(v)         spectral convolution: rfft2 over (y, x), keep
                            ky in {0..M-1} U {Ny-M..Ny-1}, kx in {0..M-1},
                            multiply by R_l[i,o,ky,kx] summed over i, zero
                            every other mode, irfft2
        z  = s + sum_i W_l[i,o] v[b,i] + b_l[o]
        v  = gelu(z) for l < L-1, v = z for the last layer
    y[b] = sum_i Q[i] v[b,i] + qb                       (one output channel)
gelu(z) = z (1 + erf(z / sqrt 2)) / 2.  Loss: mean over all points of
(y - t)^2.

Flat parameter layout (float32 on the device, float64 here), in order:
P[2][W], pb[W], then per layer R[W][W][2M][M][2] (re, im; index kyi < M is
ky = kyi, kyi >= M is ky = Ny - 2M + kyi), Wl[W][W], bl[W]; then Q[W], qb[1].
"""
import math

import numpy as np
from scipy.special import erf


def n_params(width, modes, layers):
    W, M = width, modes
    return 2 * W + W + layers * (W * W * 2 * M * M * 2 + W * W + W) + W + 1


def unpack(theta, width, modes, layers):
    W, M = width, modes
    p = {}
    o = 0

    def take(n, shape):
        nonlocal o
        a = theta[o:o + n].reshape(shape)
        o += n
        return a

    p["P"] = take(2 * W, (2, W))
    p["pb"] = take(W, (W,))
    p["R"], p["W"], p["b"] = [], [], []
    for _ in range(layers):
        r = take(W * W * 2 * M * M * 2, (W, W, 2 * M, M, 2))
        p["R"].append(r[..., 0] + 1j * r[..., 1])
        p["W"].append(take(W * W, (W, W)))
        p["b"].append(take(W, (W,)))
    p["Q"] = take(W, (W,))
    p["qb"] = take(1, (1,))
    assert o == theta.size
    return p


def init_params(width, modes, layers, seed=0):
    """Deterministic initial weights (scaled uniform)."""
    rng = np.random.default_rng(seed)
    W, M = width, modes
    parts = [rng.uniform(-1, 1, 2 * W) / math.sqrt(2), np.zeros(W)]
    for _ in range(layers):
        parts.append(rng.uniform(0, 1, W * W * 2 * M * M * 2) / (W * W))
        parts.append(rng.uniform(-1, 1, W * W) / math.sqrt(W))
        parts.append(np.zeros(W))
    parts += [rng.uniform(-1, 1, W) / math.sqrt(W), np.zeros(1)]
    return np.concatenate(parts)


def _kept_ky(ny, modes):
    return np.concatenate([np.arange(modes), np.arange(ny - modes, ny)])


def gelu(z):
    return 0.5 * z * (1.0 + erf(z / math.sqrt(2.0)))


def gelu_grad(z):
    return 0.5 * (1.0 + erf(z / math.sqrt(2.0))) + z * np.exp(-0.5 * z * z) / math.sqrt(2.0 * math.pi)


def spectral(v, R, modes):
    """K v for v[b, i, Ny, Nx] with weights R[i, o, 2M, M] (complex)."""
    b, _, ny, nx = v.shape
    ky = _kept_ky(ny, modes)
    vh = np.fft.rfft2(v)[:, :, ky, :modes]
    yh = np.einsum("bikl,iokl->bokl", vh, R)
    full = np.zeros((b, R.shape[1], ny, nx // 2 + 1), dtype=np.complex128)
    full[:, :, ky, :modes] = yh
    return np.fft.irfft2(full, s=(ny, nx))


def forward(theta, x, width, modes, layers):
    """Returns (y[b, Ny, Nx], cache)."""
    p = unpack(theta, width, modes, layers)
    v = np.einsum("bixy,io->boxy", x, p["P"]) + p["pb"][None, :, None, None]
    cache = {"x": x, "v": [v], "z": []}
    for l in range(layers):
        s = spectral(v, p["R"][l], modes)
        z = s + np.einsum("bixy,io->boxy", v, p["W"][l]) + p["b"][l][None, :, None, None]
        cache["z"].append(z)
        v = gelu(z) if l < layers - 1 else z
        cache["v"].append(v)
    y = np.einsum("bixy,i->bxy", v, p["Q"]) + p["qb"][0]
    return y, cache


def loss(theta, x, t, width, modes, layers):
    y, _ = forward(theta, x, width, modes, layers)
    return float(np.mean((y - t) ** 2))


def backward(theta, x, t, width, modes, layers):
    """Gradient of the loss with respect to the flat parameter vector."""
    p = unpack(theta, width, modes, layers)
    y, c = forward(theta, x, width, modes, layers)
    b, _, ny, nx = x.shape
    ky = _kept_ky(ny, modes)
    dy = 2.0 * (y - t) / y.size
    g = {"R": [None] * layers, "W": [None] * layers, "b": [None] * layers}
    v_last = c["v"][-1]
    g["Q"] = np.einsum("bixy,bxy->i", v_last, dy)
    g["qb"] = np.array([dy.sum()])
    dv = np.einsum("bxy,i->bixy", dy, p["Q"])
    for l in reversed(range(layers)):
        z = c["z"][l]
        dz = dv * gelu_grad(z) if l < layers - 1 else dv
        v_in = c["v"][l]
        g["b"][l] = dz.sum(axis=(0, 2, 3))
        g["W"][l] = np.einsum("bixy,boxy->io", v_in, dz)
        dv_in = np.einsum("boxy,io->bixy", dz, p["W"][l])
        # spectral path: s = irfft2(place(vh_kept @ R)); real loss gradient
        # through irfft2 is rfft2 with the Hermitian weights of the half
        # spectrum (1/(Ny Nx) per mode, doubled for 0 < kx < Nx/2).
        dfull = np.fft.rfft2(dz) / (ny * nx)
        wk = np.full(nx // 2 + 1, 2.0)
        wk[0] = 1.0
        if nx % 2 == 0:
            wk[-1] = 1.0
        dyh = np.conj(dfull[:, :, ky, :modes]) * wk[None, None, None, :modes]
        # dyh holds dL/d(yh) in the convention dL = Re(sum dyh * d yh)
        vh = np.fft.rfft2(v_in)[:, :, ky, :modes]
        # yh = sum_i vh R  ->  dR = sum_b vh * dyh  (same convention)
        g["R"][l] = np.einsum("bikl,bokl->iokl", vh, dyh)
        dvh = np.einsum("bokl,iokl->bikl", dyh, p["R"][l])
        # vh_k = sum_x v e^{-i phi_k}, so d(Re sum_k dvh_k vh_k)/dv(x) =
        # Re(sum_k dvh_k e^{-i phi_k}): a forward fft2 of the zero-padded
        # array of dvh over the kept modes.
        full = np.zeros((b, width, ny, nx), dtype=np.complex128)
        full[:, :, ky, :modes] = dvh
        dv = dv_in + np.real(np.fft.fft2(full))
    g["pb"] = dv.sum(axis=(0, 2, 3))
    g["P"] = np.einsum("bixy,boxy->io", x, dv)
    # pack, R gradient as (re, im) of the conjugate convention: for a real
    # loss, dL/dRe = Re(dR), dL/dIm = -Im(dR) with dL = Re(sum dR * dR_param)
    parts = [g["P"].ravel(), g["pb"]]
    for l in range(layers):
        r = g["R"][l]
        parts.append(np.stack([r.real, -r.imag], axis=-1).ravel())
        parts.append(g["W"][l].ravel())
        parts.append(g["b"][l])
    parts += [g["Q"], g["qb"]]
    return np.concatenate(parts), float(np.mean((y - t) ** 2))

