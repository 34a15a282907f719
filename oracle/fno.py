"""Float64 Fourier neural operator: forward and hand-written backward.

TEST INFRASTRUCTURE ONLY (the reference for the GPU kernels' gradient
checks).  Not part of the paper: the learned warm start of the PAGD solve
predicts a correction to the extrapolated initial guess.

Network (width W, retained modes M per axis, L spectral layers), input
x[b, 2, Ny, Nx] (2D) or x[b, 2, Nz, Ny, Nx] (3D):
    v0 = lift(x)            v0[b,o] = sum_i P[i,o] x[b,i] + pb[o]
    for l < L:
        s  = K_l(v)         spectral convolution: real FFT over the grid axes,
                            keep kx in {0..M-1} and, on every other axis, k in
                            {0..M-1} U {N-M..N-1}, multiply by R_l[i,o,k]
                            summed over i, zero every other mode, inverse FFT
        z  = s + sum_i W_l[i,o] v[b,i] + b_l[o]
        v  = gelu(z) for l < L-1, v = z for the last layer
    y[b] = sum_i Q[i] v[b,i] + qb                       (one output channel)
gelu(z) = z (1 + erf(z / sqrt 2)) / 2.  Loss: mean over all points of
(y - t)^2.

Flat parameter layout (float32 on the device, float64 here), in order:
P[2][W], pb[W], then per layer R[W][W][2M][M][2] (2D) or
R[W][W][2M][2M][M][2] (3D, kz then ky then kx) (re, im; on a full axis index
ki < M is k = ki, ki >= M is k = N - 2M + ki), Wl[W][W], bl[W]; then Q[W],
qb[1].
"""
import math

import numpy as np
from scipy.special import erf


def n_modes(modes, ndim=2):
    """Retained complex modes per channel pair: (2M)^(ndim-1) M."""
    return (2 * modes) ** (ndim - 1) * modes


def n_params(width, modes, layers, ndim=2):
    W = width
    return 2 * W + W + layers * (W * W * n_modes(modes, ndim) * 2 + W * W + W) + W + 1


def unpack(theta, width, modes, layers, ndim=2):
    W, M = width, modes
    rshape = (W, W) + (2 * M,) * (ndim - 1) + (M, 2)
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
        r = take(W * W * n_modes(M, ndim) * 2, rshape)
        p["R"].append(r[..., 0] + 1j * r[..., 1])
        p["W"].append(take(W * W, (W, W)))
        p["b"].append(take(W, (W,)))
    p["Q"] = take(W, (W,))
    p["qb"] = take(1, (1,))
    assert o == theta.size
    return p


def init_params(width, modes, layers, seed=0, ndim=2):
    """Deterministic initial weights (scaled uniform)."""
    rng = np.random.default_rng(seed)
    W, M = width, modes
    parts = [rng.uniform(-1, 1, 2 * W) / math.sqrt(2), np.zeros(W)]
    for _ in range(layers):
        parts.append(rng.uniform(0, 1, W * W * n_modes(M, ndim) * 2) / (W * W))
        parts.append(rng.uniform(-1, 1, W * W) / math.sqrt(W))
        parts.append(np.zeros(W))
    parts += [rng.uniform(-1, 1, W) / math.sqrt(W), np.zeros(1)]
    return np.concatenate(parts)


def _kept(n, modes):
    return np.concatenate([np.arange(modes), np.arange(n - modes, n)])


def _kept_index(shape, modes):
    """Index tuple selecting the retained modes of a real-FFT array whose
    last len(shape) axes are the grid axes (x last, half spectrum)."""
    full = [np.ix_(*([_kept(n, modes) for n in shape[:-1]] + [np.arange(modes)]))]
    return (Ellipsis,) + tuple(full[0])


def gelu(z):
    return 0.5 * z * (1.0 + erf(z / math.sqrt(2.0)))


def gelu_grad(z):
    return 0.5 * (1.0 + erf(z / math.sqrt(2.0))) + z * np.exp(-0.5 * z * z) / math.sqrt(2.0 * math.pi)


def spectral(v, R, modes):
    """K v for v[b, i, *grid] with weights R[i, o, *kept modes] (complex)."""
    grid = v.shape[2:]
    axes = tuple(range(2, v.ndim))
    sel = _kept_index(grid, modes)
    vh = np.fft.rfftn(v, axes=axes)[sel]
    yh = np.einsum("bi...,io...->bo...", vh, R)
    full = np.zeros((v.shape[0], R.shape[1]) + grid[:-1] + (grid[-1] // 2 + 1,), dtype=np.complex128)
    full[sel] = yh
    return np.fft.irfftn(full, s=grid, axes=axes)


def forward(theta, x, width, modes, layers):
    """Returns (y[b, *grid], cache); 2D or 3D from x's rank."""
    ndim = x.ndim - 2
    p = unpack(theta, width, modes, layers, ndim)
    lift = lambda a, w: np.einsum("bi...,io->bo...", a, w)
    chan = lambda c: c.reshape((1, -1) + (1,) * ndim)
    v = lift(x, p["P"]) + chan(p["pb"])
    cache = {"x": x, "v": [v], "z": []}
    for l in range(layers):
        s = spectral(v, p["R"][l], modes)
        z = s + lift(v, p["W"][l]) + chan(p["b"][l])
        cache["z"].append(z)
        v = gelu(z) if l < layers - 1 else z
        cache["v"].append(v)
    y = np.einsum("bi...,i->b...", v, p["Q"]) + p["qb"][0]
    return y, cache


def loss(theta, x, t, width, modes, layers):
    y, _ = forward(theta, x, width, modes, layers)
    return float(np.mean((y - t) ** 2))


def backward(theta, x, t, width, modes, layers):
    """Gradient of the loss with respect to the flat parameter vector."""
    ndim = x.ndim - 2
    p = unpack(theta, width, modes, layers, ndim)
    y, c = forward(theta, x, width, modes, layers)
    grid = x.shape[2:]
    axes = tuple(range(2, x.ndim))
    sum_axes = (0,) + axes
    npts = int(np.prod(grid))
    sel = _kept_index(grid, modes)
    dy = 2.0 * (y - t) / y.size
    g = {"R": [None] * layers, "W": [None] * layers, "b": [None] * layers}
    v_last = c["v"][-1]
    flat = lambda a: a.reshape(a.shape[:a.ndim - ndim] + (-1,))  # grid axes -> one
    g["Q"] = np.einsum("bip,bp->i", flat(v_last), flat(dy))
    g["qb"] = np.array([dy.sum()])
    dv = np.einsum("b...,i->bi...", dy, p["Q"])
    nxh = grid[-1] // 2 + 1
    wk = np.full(nxh, 2.0)
    wk[0] = 1.0
    if grid[-1] % 2 == 0:
        wk[-1] = 1.0
    for l in reversed(range(layers)):
        z = c["z"][l]
        dz = dv * gelu_grad(z) if l < layers - 1 else dv
        v_in = c["v"][l]
        g["b"][l] = dz.sum(axis=sum_axes)
        g["W"][l] = np.einsum("bip,bop->io", flat(v_in), flat(dz))
        dv_in = np.einsum("bo...,io->bi...", dz, p["W"][l])
        # spectral path: s = irfftn(place(vh_kept @ R)); the real loss
        # gradient through irfftn is rfftn with the Hermitian weights of the
        # half spectrum (1/P per mode, doubled for 0 < kx < Nx/2).
        dfull = np.fft.rfftn(dz, axes=axes) / npts
        dyh = np.conj(dfull[sel]) * wk[:modes]
        # dyh holds dL/d(yh) in the convention dL = Re(sum dyh * d yh)
        vh = np.fft.rfftn(v_in, axes=axes)[sel]
        # yh = sum_i vh R  ->  dR = sum_b vh * dyh  (same convention)
        g["R"][l] = np.einsum("bi...,bo...->io...", vh, dyh)
        dvh = np.einsum("bo...,io...->bi...", dyh, p["R"][l])
        # vh_k = sum_x v e^{-i phi_k}, so d(Re sum_k dvh_k vh_k)/dv(x) =
        # Re(sum_k dvh_k e^{-i phi_k}): a forward FFT of the zero-padded
        # array of dvh over the kept modes.
        full = np.zeros(x.shape[:1] + (width,) + grid, dtype=np.complex128)
        full[sel] = dvh
        dv = dv_in + np.real(np.fft.fftn(full, axes=axes))
    g["pb"] = dv.sum(axis=sum_axes)
    g["P"] = np.einsum("bip,bop->io", flat(x), flat(dv))
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


def band_resample(f, shape):
    """Band-limited resampling of a real periodic 2D field f [Ny, Nx] onto a
    grid of `shape` (same periods): the Fourier modes |ky| < Ny'/2 and
    |kx| < Nx'/2, with Ny', Nx' the smaller of the two grids' sizes per axis,
    are kept and every other mode is dropped (so the coarser grid's Nyquist
    mode is dropped too); the resulting trigonometric polynomial is then
    evaluated at the target grid's points.  Used as the reference of the
    learned guess's change of grid (a network that runs on a coarser grid
    than the solver's)."""
    f = np.asarray(f, dtype=np.float64)
    ny, nx = f.shape
    my, mx = shape
    by, bx = min(ny, my) // 2, min(nx, mx) // 2
    c = np.fft.fft2(f) / (ny * nx)  # f = sum_k c_k exp(2 pi i k.x / L)
    g = np.zeros((my, mx), dtype=np.complex128)
    for ky in range(-by + 1, by):
        for kx in range(-bx + 1, bx):
            g[ky % my, kx % mx] = c[ky % ny, kx % nx]
    return np.real(np.fft.ifft2(g)) * (my * mx)
