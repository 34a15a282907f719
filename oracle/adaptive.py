"""Adaptive time stepping (paper Sec. 3.1.2 and Alg. 3): the AM3 and
midAB2 error estimators and the step-size controller.

TEST INFRASTRUCTURE ONLY (the reference the GPU path is checked against).

Formulas, in the paper's notation (rho = dt~_{n+1} / dt_n):

* R(v) = M Delta mu(v), the right-hand side of the PDE.
* AM3 (eq. fml:AM3-high-sol): an explicit third-order Adams-Moulton value
      u^_{n+1} = u^n + dt~/6 [ (3 + 2 rho)/(1 + rho) R(u~^{n+1})
                              + (3 + rho) R(u^n) - rho^2/(1 + rho) R(u^{n-1}) ],
  ERR = ||u~^{n+1} - u^_{n+1}|| / ||u^_{n+1}|| (eq. fml:AM3-err).
* midAB2 (eq. fml:midAB2-high-sol): the quadratic through (t_n, u^n),
  (t_{n-1}, u^{n-1}), (t_{n-2}, u^{n-2}) evaluated at t_n + dt~, and
  ERR = ||u~ - u^|| / ||u^|| / (1 - 1/(24 R_n)) with
  R_n = 1/24 + (1 + dt_n/dt~)(1 + 2 dt_n/dt~ + dt_{n-1}/dt~) / 8
  (eq. fml:midAB2-err).
* Accept when ERR <= TOL or dt~ <= dt_min; the next tentative size is
  0.9 (TOL/ERR)^(1/3) dt~ clamped to [dt_min, dt_max] (eqs. fml:time-step,
  fml:time-step-med), computed after every attempt.

Readings where the paper is silent:

* First step (no u^{n-1}, no dt_n): rho = 0, so the R(u^{n-1}) term drops
  and AM3 reduces to the trapezoidal rule.
* midAB2 needs three solutions; with fewer (the first two steps) AM3 is
  used, as the paper does for n = 1, 2.  The "auto" estimator is midAB2 for
  the MP scheme and AM3 for BDF2, LBDF2 and LMP (the paper's default
  pairing; its one exception, LMP on PFC2, is a per-experiment choice).
* A tentative solve that fails counts as ERR = +inf: the attempt is
  rejected and the next tentative size is dt_min.  A failed solve at dt_min
  cannot be accepted and ends the march.
* ERR = 0 gives the next size dt_max.
* L2 norms are grid sums times the cell volume (the trapezoid rule of the
  collocation inner product); the volume cancels in every ratio.
"""
import math

import numpy as np

from . import driver as _driver
from . import imex as _imex
from . import pagd as _pagd

AM3 = "am3"
MIDAB2 = "midab2"
AUTO = "auto"


def rhs(model, grid, v, mobility=1.0):
    """R(v) = M Delta_N mu(v)."""
    return mobility * grid.lap(model.mu(grid, v))


def l2(grid, w):
    return math.sqrt(grid.cell * float(np.sum(w * w)))


def am3_weights(dt_t, dt_n):
    """Weights (w_t, w_n, w_m) of R(u~), R(u^n), R(u^{n-1}) in u^ - u^n;
    dt_n None on the first step (rho = 0)."""
    rho = 0.0 if dt_n is None else dt_t / dt_n
    return (dt_t / 6.0 * (3.0 + 2.0 * rho) / (1.0 + rho),
            dt_t / 6.0 * (3.0 + rho),
            -dt_t / 6.0 * rho * rho / (1.0 + rho))


def am3_value(u_n, R_t, R_n, R_m, dt_t, dt_n):
    w_t, w_n, w_m = am3_weights(dt_t, dt_n)
    out = u_n + w_t * R_t + w_n * R_n
    if w_m != 0.0:
        out = out + w_m * R_m
    return out


def midab2_weights(dt_t, dt_n, dt_m):
    """Weights of u^n, u^{n-1}, u^{n-2} in the midAB2 value."""
    c0 = (dt_t + dt_n) * (dt_t + dt_n + dt_m) / (dt_n * (dt_n + dt_m))
    c1 = -dt_t * (dt_t + dt_n + dt_m) / (dt_n * dt_m)
    c2 = dt_t * (dt_t + dt_n) / (dt_m * (dt_n + dt_m))
    return c0, c1, c2


def midab2_factor(dt_t, dt_n, dt_m):
    """1 / (1 - 1/(24 R_n))."""
    rn = 1.0 / 24.0 + 0.125 * (1.0 + dt_n / dt_t) * (1.0 + 2.0 * dt_n / dt_t + dt_m / dt_t)
    return 1.0 / (1.0 - 1.0 / (24.0 * rn))


def next_dt(err, tol, dt_tmp, dt_min, dt_max):
    """Eqs. fml:time-step and fml:time-step-med."""
    if err == 0.0:
        bar = math.inf
    elif math.isinf(err):
        bar = 0.0
    else:
        bar = 0.9 * (tol / err) ** (1.0 / 3.0) * dt_tmp
    return max(dt_min, min(bar, dt_max))


def uses_midab2(estimator, scheme, n_hist):
    """n_hist: number of stored solutions (u^n, u^{n-1}, ...) available."""
    want = estimator == MIDAB2 or (estimator == AUTO and scheme == "mp")
    return want and n_hist >= 3


class AdaptiveRun:
    """Alg. 3 with a PAGD (BDF2, MP) or linear IMEX (LBDF2, LMP) step.

    ``attempt()`` is one pass of the loop body: tentative solve at the current
    tentative size, error estimate, accept or reject, next tentative size.
    """

    def __init__(self, grid, model, scheme, u0, tol, dt_min, dt_max, estimator=AUTO,
                 mobility=1.0, solver=None):
        """``solver``: keyword arguments of the PAGD driver (s, etas, tol,
        max_iter, ...); ``tol`` here is the stepping tolerance TOL."""
        self.grid, self.model, self.scheme = grid, model, scheme
        self.tol, self.dt_min, self.dt_max = float(tol), float(dt_min), float(dt_max)
        self.estimator = estimator
        self.M = float(mobility)
        if scheme in ("bdf2", "mp"):
            self.sim = _driver.Simulation(grid, model, scheme, mobility=mobility, **(solver or {}))
        else:
            self.sim = None
        u0 = np.array(u0, dtype=np.float64)
        self.hist = [u0]            # u^n, u^{n-1}, u^{n-2}
        self.dts = []               # dt_n, dt_{n-1}
        self.R = [self.rhs(u0)]     # R(u^n), R(u^{n-1})
        self.t = 0.0
        self.n = 0
        self.dt_try = self.dt_min

    def rhs(self, v):
        return rhs(self.model, self.grid, v, self.M)

    def solve(self, dt):
        u_n = self.hist[0]
        u_nm1 = self.hist[1] if len(self.hist) > 1 else None
        dt_old = self.dts[0] if self.dts else None
        if self.sim is not None:
            out = self.sim.step(u_n, u_nm1, dt, dt_old)
            return out["x"], out["status"], out["iters"]
        x = _imex.step(self.model, self.grid, self.scheme, u_n, u_nm1, dt, dt_old, self.M)
        return x, _pagd.OK, 1

    def estimate(self, u_t, R_t, dt_t):
        """(ERR, u^) for the tentative solution u_t at size dt_t."""
        g = self.grid
        if uses_midab2(self.estimator, self.scheme, len(self.hist)):
            c0, c1, c2 = midab2_weights(dt_t, self.dts[0], self.dts[1])
            u_hat = c0 * self.hist[0] + c1 * self.hist[1] + c2 * self.hist[2]
            fac = midab2_factor(dt_t, self.dts[0], self.dts[1])
            return l2(g, u_t - u_hat) / l2(g, u_hat) * fac, u_hat
        dt_n = self.dts[0] if self.dts else None
        R_m = self.R[1] if len(self.R) > 1 else None
        u_hat = am3_value(self.hist[0], R_t, self.R[0], R_m, dt_t, dt_n)
        return l2(g, u_t - u_hat) / l2(g, u_hat), u_hat

    def attempt(self):
        """Returns a record of the attempt (dt, status, err, accepted, iters)."""
        dt = self.dt_try
        u_t, status, iters = self.solve(dt)
        if status == _pagd.OK:
            R_t = self.rhs(u_t)
            err, _ = self.estimate(u_t, R_t, dt)
        else:
            R_t, err = None, math.inf
        accepted = status == _pagd.OK and (err <= self.tol or dt <= self.dt_min)
        if accepted:
            self.hist = [u_t] + self.hist[:2]
            self.dts = [dt] + self.dts[:1]
            self.R = [R_t] + self.R[:1]
            self.t += dt
            self.n += 1
        self.dt_try = next_dt(err, self.tol, dt, self.dt_min, self.dt_max)
        return dict(dt=dt, status=status, err=err, accepted=accepted, iters=iters)

    def run(self, T, max_attempts=100000):
        """March until t >= T; returns the list of attempt records."""
        log = []
        while self.t < T and len(log) < max_attempts:
            rec = self.attempt()
            log.append(rec)
            if rec["status"] != _pagd.OK and rec["dt"] <= self.dt_min:
                break
        return log

    @property
    def u(self):
        return self.hist[0]
