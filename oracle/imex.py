"""Linear IMEX schemes LBDF2 and LMP (paper Sec. 3.1.1, eq.
eqn:FCH-semidis-simplicit).

TEST INFRASTRUCTURE ONLY (the reference the GPU path is checked against).

The chemical potential is split as mu = L(u) + N(u) with L linear and
positive semi-definite:
    PFC: L(u) = (1 + Delta)^2 u,            N(u) = u^3 - eps u
    FCH: L(u) = eps^4 Delta^2 u + kappa2 (-Delta) u + kappa0 u,
         N(u) = -kappa0 u - eps^2 Delta F'(u)
                - (eps^2 (F''(u) - eta1) - kappa2) Delta u + (F''(u) - eta2) F'(u),
         kappa0 = 1 - 2 tau^2 + eta2, kappa2 = 1.
L is taken implicitly at u_bar, N explicitly at the extrapolation u_breve:
    a u^{n+1} + b u^n + c u^{n-1} = M Delta (L(u_bar) + N(u_breve)),
    LBDF2: (a, b, c) of BDF2 (backward Euler first), u_bar = u^{n+1},
           u_breve = u^n + rho (u^n - u^{n-1});
    LMP:   (a, b, c) of MP, u_bar = (u^n + u^{n+1})/2,
           u_breve = ((2 + rho) u^n - rho u^{n-1}) / 2;
rho = dt_{n+1}/dt_n and u^{-1} := u^0 on the first step.  In Fourier
space, with q = |k|^2 and l(k) the symbol of L, theta = 1 (LBDF2) or 1/2
(LMP):
    (a + M q theta l) u^{n+1}^ = -b u^n^ - c u^{n-1}^ - M q (N^(u_breve) + (1 - theta) l u^n^).
"""
import numpy as np

from . import models as _models
from . import schemes as _schemes

LBDF2 = "lbdf2"
LMP = "lmp"


def kappas(model):
    """(kappa0, kappa2) of the FCH splitting."""
    return 1.0 - 2.0 * model.tau ** 2 + model.eta2, 1.0


def linear_symbol(model, grid):
    """Symbol l(k) of L on the grid's half spectrum."""
    q = grid.k2
    if model.name == "pfc":
        return (1.0 - q) ** 2
    k0, k2 = kappas(model)
    return model.eps ** 4 * q * q + k2 * q + k0


def linear_part(model, grid, u):
    return grid.inv(linear_symbol(model, grid) * grid.fwd(u))


def nonlinear_part(model, grid, u):
    """N(u) written term by term as in the splitting above."""
    if model.name == "pfc":
        return u ** 3 - model.eps * u
    e2 = model.eps ** 2
    k0, k2 = kappas(model)
    f1 = _models.dF(u, model.tau)
    f2 = _models.d2F(u, model.tau)
    return (-k0 * u - e2 * grid.lap(f1) - (e2 * (f2 - model.eta1) - k2) * grid.lap(u)
            + (f2 - model.eta2) * f1)


def step(model, grid, scheme, u_n, u_nm1, dt_new, dt_old, mobility=1.0):
    """u^{n+1} of one LBDF2 / LMP step; u_nm1 and dt_old are None on the first."""
    base = _schemes.BDF2 if scheme == LBDF2 else _schemes.MP
    a, b, c, _ = _schemes.coefficients(base, dt_new, dt_old)
    if u_nm1 is None:
        u_prev, rho = u_n, 0.0
    else:
        u_prev, rho = u_nm1, dt_new / dt_old
    if scheme == LBDF2:
        theta = 1.0
        u_breve = u_n + rho * (u_n - u_prev)
    elif scheme == LMP:
        theta = 0.5
        u_breve = ((2.0 + rho) * u_n - rho * u_prev) / 2.0
    else:
        raise ValueError(f"unknown IMEX scheme {scheme!r}")
    q = grid.k2
    lsym = linear_symbol(model, grid)
    un_h = grid.fwd(u_n)
    rhs = (-b * un_h - c * grid.fwd(u_prev)
           - mobility * q * (grid.fwd(nonlinear_part(model, grid, u_breve)) + (1.0 - theta) * lsym * un_h))
    return grid.inv(rhs / (a + mobility * q * theta * lsym))


def run(model, grid, scheme, u0, dt, nsteps, mobility=1.0):
    """Fixed-step march; returns the final state."""
    u_n, u_nm1, dt_old = np.array(u0, dtype=np.float64), None, None
    for _ in range(nsteps):
        u_np1 = step(model, grid, scheme, u_n, u_nm1, dt, dt_old, mobility)
        u_nm1, u_n, dt_old = u_n, u_np1, dt
    return u_n
