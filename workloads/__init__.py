"""Seeded synthetic workloads shared by the tests, the smoke check and the bench.

This module holds the workload definitions (grid, model parameters, scheme,
step size) and the seeded initial-condition generators only.  It contains
none of the method's arithmetic and imports neither the CPU oracle nor the
HIP library; both sides receive the same arrays from here.

The paper's own benchmark initial conditions (FCH1-3, PFC1-2) are defined
in external references and are not reproduced; uniform-noise initial
conditions around a mean value of the same shapes and parameter ranges stand
in for them.  A field is ``mean + amp * U(-1, 1)`` drawn i.i.d. per grid point
from ``numpy.random.default_rng(seed)`` in C order (x fastest).
"""
import math
from dataclasses import dataclass, field, replace

import numpy as np

PAPER_ETAS = tuple(math.sqrt(v) for v in (0.1, 0.575, 1.05, 1.525, 2.0))


@dataclass(frozen=True)
class Workload:
    name: str
    model: str              # "pfc" | "fch"
    scheme: str             # "mp" | "bdf2"
    shape: tuple            # (Ny, Nx) or (Nz, Ny, Nx)
    lengths: tuple          # periods, same order as shape
    dt: float
    steps: int
    mean: float
    amp: float
    eps: float
    eta1: float = 0.0       # FCH coefficients as they multiply the energy terms
    eta2: float = 0.0
    tau: float = 0.0
    s: float = 0.9
    etas: tuple = PAPER_ETAS
    tol: float = 1e-10
    max_iter: int = 1000
    mobility: float = 1.0
    seeds: tuple = (0,)

    @property
    def npoints(self):
        return int(np.prod(self.shape))

    def params(self):
        return dict(eps=self.eps, eta1=self.eta1, eta2=self.eta2, tau=self.tau)


def initial_field(shape, mean, amp, seed):
    """mean + amp * U(-1, 1) i.i.d. per point, C order, float64."""
    rng = np.random.default_rng(seed)
    return mean + amp * rng.uniform(-1.0, 1.0, size=tuple(shape))


def initial_condition(w: Workload, seed=None):
    s = w.seeds[0] if seed is None else seed
    return initial_field(w.shape, w.mean, w.amp, s)


# PFC 2D, 64 x 64 on [0, 64)^2, eps = 0.25, phi0 = -0.25 + 0.05 U(-1, 1),
# implicit midpoint, dt = 0.1, 20 steps.  Small case: the oracle runs it in
# seconds.
PFC64_MP = Workload(
    name="pfc2d_64_mp", model="pfc", scheme="mp", shape=(64, 64),
    lengths=(64.0, 64.0), dt=0.1, steps=20, mean=-0.25, amp=0.05, eps=0.25,
    seeds=(0, 1, 2, 3, 4))

# FCH 2D, 256 x 256 on [0, 4 pi)^2, eps = 0.1, eta1 = 1.45 eps, eta2 = 2 eps,
# W = (u^2 - 1)^2 / 4 (tau = 0), u0 = -0.6 + 0.01 U(-1, 1), BDF2 (backward
# Euler first), dt = 1e-3, 100 steps.  Same L, N, eps, eta's as the paper's
# FCH3 (Table tab:setting-benchmark) except tau and the initial condition.
FCH256_BDF2 = Workload(
    name="fch2d_256_bdf2", model="fch", scheme="bdf2", shape=(256, 256),
    lengths=(4 * math.pi, 4 * math.pi), dt=1e-3, steps=100, mean=-0.6, amp=0.01,
    eps=0.1, eta1=0.145, eta2=0.2, tau=0.0, seeds=(0, 1, 2, 3, 4))


def pfc_ensemble(count=64, steps=200, base_seed=1000, sizes=(128, 256, 512)):
    """Batched PFC ensemble: Nx, Ny drawn independently from ``sizes``,
    L = N per axis (dx = 1), eps ~ U[0.2, 0.3], mean ~ U[-0.35, -0.15],
    noise amplitude 0.05, implicit midpoint, dt = 0.1.  Instance i draws its
    parameters from seed ``base_seed + i``."""
    out = []
    for i in range(count):
        rng = np.random.default_rng(base_seed + i)
        ny = int(rng.choice(sizes))
        nx = int(rng.choice(sizes))
        eps = float(rng.uniform(0.2, 0.3))
        mean = float(rng.uniform(-0.35, -0.15))
        out.append(Workload(
            name=f"pfc2d_ens{i}_{ny}x{nx}", model="pfc", scheme="mp", shape=(ny, nx),
            lengths=(float(ny), float(nx)), dt=0.1, steps=steps, mean=mean, amp=0.05,
            eps=eps, seeds=(base_seed + i,)))
    return out


def scaled(w: Workload, **changes):
    return replace(w, **changes)


# PFC 3D, 192^3 on [0, 192)^3, eps = 0.25, phi0 = -0.2 + 0.05 U(-1, 1),
# BDF2 (backward Euler first), dt = 0.1, 300 steps.
PFC192_3D = Workload(
    name="pfc3d_192_bdf2", model="pfc", scheme="bdf2", shape=(192, 192, 192),
    lengths=(192.0, 192.0, 192.0), dt=0.1, steps=300, mean=-0.2, amp=0.05, eps=0.25,
    seeds=(0,))


def fch_ensemble(count_per_size=8, sizes=(1024, 2048), steps=300, base_seed=2000):
    """Large FCH ensemble: ``count_per_size`` instances per grid size (square
    grids on [0, 4 pi)^2), e ~ U[0.08, 0.12] with eps = e, eta1 = 1.45 e,
    eta2 = 2 e, tau = 0, mean ~ U[-0.7, -0.5], noise amplitude 0.01, BDF2
    (backward Euler first), dt = 1e-3.  Instance i draws its parameters from
    seed ``base_seed + i``."""
    out = []
    i = 0
    for n in sizes:
        for _ in range(count_per_size):
            rng = np.random.default_rng(base_seed + i)
            e = float(rng.uniform(0.08, 0.12))
            mean = float(rng.uniform(-0.7, -0.5))
            out.append(Workload(
                name=f"fch2d_ens{i}_{n}", model="fch", scheme="bdf2", shape=(n, n),
                lengths=(4 * math.pi, 4 * math.pi), dt=1e-3, steps=steps, mean=mean, amp=0.01,
                eps=e, eta1=1.45 * e, eta2=2.0 * e, tau=0.0, seeds=(base_seed + i,)))
            i += 1
    return out
