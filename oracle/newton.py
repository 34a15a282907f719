"""Dense Newton solve of one fully discrete step, used only to pin PAGD.

Solves F(u) = a u + b u^n + c u^{n-1} - M Delta_N mu(u_breve) = 0
(eq. eqn:FCH-fulldis-implicit) with the exact Jacobian
J = a I - M theta Delta_N Dmu(u_breve), assembled as dense matrices.  The
discrete Laplacian matrix is built column by column from unit vectors, so the
only ingredient shared with the PAGD path is the operator Delta_N itself.
Tiny grids only (P up to a few hundred).
"""
import numpy as np

from . import models as _models


def laplacian_matrix(grid):
    P = grid.npoints
    D = np.zeros((P, P))
    e = np.zeros(P)
    for i in range(P):
        e[:] = 0.0
        e[i] = 1.0
        D[:, i] = grid.lap(e.reshape(grid.shape)).ravel()
    return D


def mu_jacobian(model, grid, D, v):
    """Dense Jacobian of u -> mu_N(u) at v (C-order flattening)."""
    P = grid.npoints
    I = np.eye(P)
    vf = v.ravel()
    if isinstance(model, _models.PFC):
        return np.diag(3.0 * vf * vf) + (1.0 - model.eps) * I + 2.0 * D + D @ D
    if isinstance(model, _models.FCH):
        e2 = model.eps ** 2
        f1 = _models.dF(vf, model.tau)
        f2 = _models.d2F(vf, model.tau)
        f3 = _models.d3F(vf, model.tau)
        om = e2 * (D @ vf) - f1
        Dom = e2 * D - np.diag(f2)
        return (e2 * D @ Dom - np.diag(f3 * om) - np.diag(f2) @ Dom
                + e2 * model.eta1 * D - model.eta2 * np.diag(f2))
    raise TypeError("unknown model")


def solve(problem, x0, tol=1e-13, max_iter=50):
    """Newton iteration from x0; returns (u, iterations, ||F||_inf)."""
    g = problem.grid
    D = laplacian_matrix(g)
    u = np.array(x0, dtype=np.float64).ravel()
    un = problem.u_n.ravel()
    unm1 = problem.u_nm1.ravel()
    th, M = problem.theta, problem.M

    def residual(uf):
        ub = th * uf + (1.0 - th) * un
        mu = problem.model.mu(g, ub.reshape(g.shape)).ravel()
        return problem.a * uf + problem.b * un + problem.c * unm1 - M * (D @ mu)

    F = residual(u)
    for it in range(max_iter):
        if np.max(np.abs(F)) < tol:
            return u.reshape(g.shape), it, float(np.max(np.abs(F)))
        ub = th * u + (1.0 - th) * un
        J = problem.a * np.eye(g.npoints) - M * th * D @ mu_jacobian(problem.model, g, D, ub.reshape(g.shape))
        u = u - np.linalg.solve(J, F)
        F = residual(u)
    return u.reshape(g.shape), max_iter, float(np.max(np.abs(F)))
