"""Fixed-step time marching with a PAGD solve per step (Alg. 3, no adaptivity).

Each step: coefficients from ``schemes.coefficients`` (backward Euler on the
first BDF2 step), initial guess from ``schemes.extrapolate``, averaged-Newton
constants frozen at that guess, then PAGD to ||d||_inf < TOL.  A step that
fails (no convergence, non-finite values, non-positive preconditioner) does
not advance the history.
"""
import numpy as np

from . import pagd as _pagd
from . import schemes as _schemes

PAPER_ETAS = tuple(float(np.sqrt(v)) for v in (0.1, 0.575, 1.05, 1.525, 2.0))


class Simulation:
    def __init__(self, grid, model, scheme, s=0.9, etas=PAPER_ETAS, tol=1e-10,
                 max_iter=1000, theta_l=1.0, accelerated=True, mobility=1.0):
        self.grid = grid
        self.model = model
        self.scheme = scheme
        self.s = float(s)
        self.etas = tuple(float(e) for e in etas)
        self.tol = float(tol)
        self.max_iter = int(max_iter)
        self.theta_l = float(theta_l)
        self.accelerated = bool(accelerated)
        self.M = float(mobility)

    def step(self, u_n, u_nm1, dt_new, dt_old, history=None):
        """One step from (u^n, u^{n-1}); ``u_nm1``/``dt_old`` None on the first."""
        a, b, c, theta = _schemes.coefficients(self.scheme, dt_new, dt_old)
        x0 = _schemes.extrapolate(u_n, u_nm1, dt_new, dt_old)
        prob = _pagd.StepProblem(self.grid, self.model, a, b, c, theta, u_n,
                                 u_nm1, self.M)
        out = _pagd.solve_step(prob, x0, self.s, self.etas, self.tol, self.max_iter,
                               theta_l=self.theta_l, accelerated=self.accelerated,
                               history=history)
        out["abc"] = (a, b, c, theta)
        return out

    def run(self, u0, dt, nsteps, keep=False):
        """March ``nsteps`` constant steps; returns final state and stats."""
        u_n, u_nm1, dt_old = np.array(u0, dtype=np.float64), None, None
        iters, traj = [], []
        for _ in range(nsteps):
            out = self.step(u_n, u_nm1, dt, dt_old)
            if out["status"] != _pagd.OK:
                return dict(u=u_n, u_prev=u_nm1, iters=iters, status=out["status"],
                            traj=traj)
            u_nm1, u_n, dt_old = u_n, out["x"], dt
            iters.append(out["iters"])
            if keep:
                traj.append(u_n)
        return dict(u=u_n, u_prev=u_nm1, iters=iters, status=_pagd.OK, traj=traj)
