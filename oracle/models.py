"""PFC and FCH energies and chemical potentials (paper Sec. 2).

PFC (eq. obj:PFC-egy and eq. eqn:PFCsystem):
    E(u)  = int u^4/4 + (1-eps) u^2/2 - |grad u|^2 + (Delta u)^2/2
    mu(u) = u^3 + (1-eps) u + 2 Delta u + Delta^2 u

FCH (eq. obj:FCHegy) with the double well F of Sec. 2.2:
    E(u)  = int (eps^2 Delta u - F'(u))^2 / 2 - (eps^2 eta1 |grad u|^2 / 2 + eta2 F(u))

The printed FCH chemical potential (eqs. eqn:FCHPDE, eqn:FCHsystem) is
garbled: it writes F'' where the operator (eps^2 Delta - F''(u)) is meant and
defines omega with F'' instead of F'.  The reading used here is the exact
variational derivative of the energy above,
    omega = eps^2 Delta u - F'(u)
    mu    = eps^2 Delta omega - F''(u) omega + eps^2 eta1 Delta u - eta2 F'(u),
which equals (eps^2 Delta - F'' + eta1) omega + (eta1 - eta2) F' and the
linear + nonlinear split L + N of Sec. 3.1.1.

Discrete energies replace the gradient term by summation by parts,
-(|grad u|^2, 1) = (Delta_N u, u)_N, so that mu_N is exactly the gradient of
E_N in the (., .)_N inner product on any even grid.

Parameter convention for FCH: ``eta1`` and ``eta2`` are the coefficients as
they stand in the energy above (the paper's Table tab:setting-benchmark gives
e.g. eta1 = 1.45 eps, eta2 = 2 eps for FCH3; those products are passed in).
"""
import numpy as np


# -- double well, Sec. 2.2 ---------------------------------------------------
def F(z, tau):
    """F(z) = (z+1)^2 ((z-1)^2/2 + (2/3) tau (z-2)) / 2."""
    return 0.5 * (z + 1.0) ** 2 * (0.5 * (z - 1.0) ** 2 + (2.0 / 3.0) * tau * (z - 2.0))


def dF(z, tau):
    """F'(z) = (z^2 - 1)(z + tau)."""
    return (z * z - 1.0) * (z + tau)


def d2F(z, tau):
    """F''(z) = 3 z^2 - 1 + 2 tau z."""
    return 3.0 * z * z - 1.0 + 2.0 * tau * z


def d3F(z, tau):
    """F'''(z) = 6 z + 2 tau."""
    return 6.0 * z + 2.0 * tau


class PFC:
    """Phase field crystal model; parameter ``eps``."""

    name = "pfc"

    def __init__(self, eps):
        self.eps = float(eps)

    def mu(self, grid, u):
        lu = grid.lap(u)
        return u ** 3 + (1.0 - self.eps) * u + 2.0 * lu + grid.lap(lu)

    def energy(self, grid, u):
        lu = grid.lap(u)
        density = 0.25 * u ** 4 + 0.5 * (1.0 - self.eps) * u * u + 0.5 * lu * lu
        return grid.inner(density, np.ones_like(u)) + grid.inner(lu, u)


class FCH:
    """Functionalized Cahn-Hilliard model; parameters eps, eta1, eta2, tau."""

    name = "fch"

    def __init__(self, eps, eta1, eta2, tau=0.0):
        self.eps = float(eps)
        self.eta1 = float(eta1)
        self.eta2 = float(eta2)
        self.tau = float(tau)

    def omega(self, grid, u):
        return self.eps ** 2 * grid.lap(u) - dF(u, self.tau)

    def mu(self, grid, u):
        e2 = self.eps ** 2
        lu = grid.lap(u)
        om = e2 * lu - dF(u, self.tau)
        return (e2 * grid.lap(om) - d2F(u, self.tau) * om
                + e2 * self.eta1 * lu - self.eta2 * dF(u, self.tau))

    def energy(self, grid, u):
        e2 = self.eps ** 2
        lu = grid.lap(u)
        om = e2 * lu - dF(u, self.tau)
        density = 0.5 * om * om - self.eta2 * F(u, self.tau)
        return grid.inner(density, np.ones_like(u)) + 0.5 * e2 * self.eta1 * grid.inner(lu, u)


def make_model(kind, **params):
    if kind == "pfc":
        return PFC(params["eps"])
    if kind == "fch":
        return FCH(params["eps"], params["eta1"], params["eta2"], params.get("tau", 0.0))
    raise ValueError(f"unknown model {kind!r}")
