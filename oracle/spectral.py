"""Fourier-collocation grid and operators (paper Sec. 3.2).

Readings of the paper taken here (its text treats only odd N and L = 1):

* The domain is [0, L) per axis with N unique points, x_m = m L / N; the
  periodic duplicate of the end point is dropped.  The paper's PFC shift to
  [-L/2, L/2] is cosmetic and not applied.
* Even N is used throughout.  Mode indices are r in [-N/2, N/2) per axis and
  the Nyquist mode is kept, with symbol (2 pi r / L)^2 evaluated at
  r = -N/2.  Only even powers of the wavenumber are ever applied, so no odd
  derivative of the Nyquist mode is needed.
* The forward/inverse DFT pair is NumPy's (unnormalised forward, 1/P
  inverse).  The operators (-Delta_N)^alpha of eq. def:frac-Lap do not
  depend on how the normalisation is split between the two transforms.
* (-Delta_N)^{-1} drops the r = 0 mode (text after eq. def:frac-Lap).
* The discrete inner product is the composite trapezoid rule
  (u, v)_N = (prod_i h_i) sum u v with h_i = L_i / N_i; fields are real.
"""
import numpy as np


class Grid:
    """Periodic grid on prod_i [0, L_i) with C-order arrays, x fastest.

    ``shape`` is (Ny, Nx) in 2D or (Nz, Ny, Nx) in 3D; ``lengths`` matches.
    """

    def __init__(self, shape, lengths):
        shape = tuple(int(n) for n in shape)
        lengths = tuple(float(v) for v in lengths)
        if len(shape) != len(lengths) or len(shape) not in (1, 2, 3):
            raise ValueError("shape and lengths must both have 1, 2 or 3 entries")
        self.shape = shape
        self.lengths = lengths
        self.ndim = len(shape)
        self.npoints = int(np.prod(shape))
        self.cell = float(np.prod([L / n for L, n in zip(lengths, shape)]))
        self.area = float(np.prod(lengths))
        # Wavenumbers 2 pi r / L per axis.  The last axis uses the half
        # spectrum of a real transform (r = 0 .. N/2); the others use the
        # full index set r in [-N/2, N/2).
        ks = []
        for ax, (n, L) in enumerate(zip(shape, lengths)):
            if ax == self.ndim - 1:
                r = np.arange(n // 2 + 1, dtype=np.float64)
            else:
                r = np.fft.fftfreq(n, d=1.0 / n)
            ks.append(2.0 * np.pi * r / L)
        grids = np.meshgrid(*ks, indexing="ij")
        self.k2 = sum(g * g for g in grids)
        self.inv_k2 = np.zeros_like(self.k2)
        nz = self.k2 > 0
        self.inv_k2[nz] = 1.0 / self.k2[nz]

    def coords(self):
        """Grid coordinates x_m = m L / N, one array per axis (C order)."""
        axes = [np.arange(n) * (L / n) for n, L in zip(self.shape, self.lengths)]
        return np.meshgrid(*axes, indexing="ij")

    # -- transforms -------------------------------------------------------
    def fwd(self, w):
        return np.fft.rfftn(w)

    def inv(self, w_hat):
        return np.fft.irfftn(w_hat, s=self.shape, axes=tuple(range(self.ndim)))

    # -- operators of eq. def:frac-Lap ------------------------------------
    def lap(self, w):
        """Delta_N w: symbol -|k|^2."""
        return self.inv(-self.k2 * self.fwd(w))

    def bilap(self, w):
        """Delta_N^2 w: symbol |k|^4."""
        return self.inv(self.k2 * self.k2 * self.fwd(w))

    def inv_neg_lap(self, w):
        """(-Delta_N)^{-1} w with the r = 0 mode excluded."""
        return self.inv(self.inv_k2 * self.fwd(w))

    # -- means, projections, inner products -------------------------------
    def mean(self, w):
        return float(np.mean(w))

    def proj0(self, w):
        """Mean-zero projection Pi_0 (Remark rmk:meanzero)."""
        return w - np.mean(w)

    def inner(self, u, v):
        """(u, v)_N: trapezoid rule on the periodic grid (real fields)."""
        return self.cell * float(np.sum(u * v))

    def neg_norm_sq(self, w):
        """||w||_{-1,N}^2 = ((-Delta_N)^{-1} w, w)_N (eq. def:neg-norm)."""
        return self.inner(self.inv_neg_lap(w), w)
