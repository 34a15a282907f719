"""Brute-force Fourier sums (paper Sec. 3.2), used only to pin ``spectral``.

Given a real grid function w, apply the symbol (2 pi |r| / L)^(2 alpha) of
eq. def:frac-Lap by explicit double (triple) sums

    w_hat(r) = sum_m w(x_m) exp(-i 2 pi r.x_m / L)
    [op w](x_m) = (1/P) sum_r sym(r) w_hat(r) exp(+i 2 pi r.x_m / L)

over r in [-N/2, N/2) per axis (even N; [-(N-1)/2, (N-1)/2] for odd N), with
no FFT involved.  O(P^2) work: tiny grids only.
"""
import itertools

import numpy as np


def _modes(n):
    if n % 2 == 0:
        return list(range(-n // 2, n // 2))
    return list(range(-(n - 1) // 2, (n - 1) // 2 + 1))


def apply_symbol(w, lengths, alpha, drop_zero=False):
    """(-Delta_N)^alpha w by direct summation; ``drop_zero`` excludes r = 0."""
    shape = w.shape
    nd = len(shape)
    coords = [np.arange(n) * (L / n) for n, L in zip(shape, lengths)]
    pts = list(itertools.product(*[range(n) for n in shape]))
    P = len(pts)
    out = np.zeros(P, dtype=np.complex128)
    wv = np.array([w[p] for p in pts])
    xs = np.array([[coords[a][p[a]] for a in range(nd)] for p in pts])
    for r in itertools.product(*[_modes(n) for n in shape]):
        kvec = np.array([2.0 * np.pi * r[a] / lengths[a] for a in range(nd)])
        k2 = float(np.dot(kvec, kvec))
        if k2 == 0.0:
            if drop_zero or alpha < 0:
                continue
            sym = 1.0 if alpha == 0 else 0.0
        else:
            sym = k2 ** alpha
        phase = xs @ kvec
        what = np.sum(wv * np.exp(-1j * phase))
        out += sym * what * np.exp(1j * phase)
    out /= P
    res = np.zeros(shape)
    for i, p in enumerate(pts):
        res[p] = out[i].real
    return res
