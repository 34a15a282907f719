"""Step objective, projected gradient, averaged-Newton preconditioner, PGD/PAGD.

Paper Sec. 3.4.  Given u^n, u^{n-1} and (a, b, c), the step problem
(eq. eqn:FCH-fulldis-implicit) is the critical point of (Prop. minimization
problem, eq. obj:FCH-mini-objv)

    G_N(v) = ||a v + b u^n + c u^{n-1}||_{-1,N}^2 / (2 M a) + E~_N(v_breve),

with E~ = E (BDF2) or 2 E(v_breve) (MP).  The solvers use the mean-zero
projected gradient of eq. obj:G' as minus the residual,

    G'(v) = (1/M) (-Delta_N)^{-1} Pi_0 (a v + b u^n + c u^{n-1})
            + Pi_0 dE~/du(v_breve),

where dE~/du(v_breve) = mu(v_breve) for both schemes (for MP the factor 2 of
E~ cancels the 1/2 of the chain rule).

Averaged-Newton preconditioner (Sec. 3.4.1):
    L = beta_-2 (-Delta)^{-1} + beta_0 + beta_2 (-Delta) + beta_4 Delta^2
with beta_-2 = a / M and, evaluated at the step's initial guess,
    PFC: beta_0 = |mean(3 v^2 + 1 - eps)|, beta_2 = -2, beta_4 = 1
    FCH: beta_0 = |mean(F''^2 - eta2 F'' + F''' F')|,
         beta_2 = |mean(eps^2 F'' - eta1 eps^2)|, beta_4 = eps^4.
Readings: the averages are grid means taken at v_breve(x0); the constant PFC
coefficient beta_2 keeps its sign ("keep the value"); the FCH beta_0 drops the
two Laplacian terms the paper says it drops; the paper prints no scheme
factor, so by default the beta_0/beta_2/beta_4 part enters with weight
``theta_l`` = 1 (``theta_l`` = 1/2 is the exact MP Hessian scale, offered as
an option).  The r = 0 mode of L^{-1} r is set to zero; L must be positive on
every other grid mode or the step is rejected (PRECOND).

PAGD with sweeping friction is Alg. 2; PGD (Alg. 1) is the same loop with the
extrapolation coefficient lambda fixed at zero.  Both loops are read as
"repeat ... until ||d_i||_inf < TOL" (the printed while-condition is
inverted); the returned iterate is x_{i+1} and the iteration count is i + 1.
"""
import numpy as np

from . import models as _models

OK = 0
NOCONV = -4
NONFINITE = -5
PRECOND = -6


class StepProblem:
    """One fully discrete step: grid, model, coefficients and history."""

    def __init__(self, grid, model, a, b, c, theta, u_n, u_nm1=None, mobility=1.0):
        self.grid = grid
        self.model = model
        self.a, self.b, self.c = float(a), float(b), float(c)
        self.theta = float(theta)
        self.M = float(mobility)
        self.u_n = u_n
        self.u_nm1 = u_n if u_nm1 is None else u_nm1

    def breve(self, v):
        """v_breve = theta v + (1 - theta) u^n."""
        return self.theta * v + (1.0 - self.theta) * self.u_n

    def linear_part(self, v):
        """a v + b u^n + c u^{n-1}."""
        return self.a * v + self.b * self.u_n + self.c * self.u_nm1

    def objective(self, v):
        """G_N(v), eq. obj:FCH-mini-objv."""
        g = self.grid
        lin = self.linear_part(v)
        e = self.model.energy(g, self.breve(v))
        # E~ = E for BDF2 (theta = 1) and 2 E(v_breve) for MP (theta = 1/2).
        e_tilde = e if self.theta == 1.0 else 2.0 * e
        return g.neg_norm_sq(lin) / (2.0 * self.M * self.a) + e_tilde

    def gradient(self, v):
        """Projected gradient G'(v), eq. obj:G'."""
        g = self.grid
        first = g.inv_neg_lap(g.proj0(self.linear_part(v))) / self.M
        return first + g.proj0(self.model.mu(g, self.breve(v)))

    def residual(self, v):
        return -self.gradient(v)


def averaged_newton_betas(problem, x0):
    """(beta_-2, beta_0, beta_2, beta_4) evaluated at v_breve(x0)."""
    m = problem.model
    v = problem.breve(x0)
    bm2 = problem.a / problem.M
    if isinstance(m, _models.PFC):
        b0 = abs(float(np.mean(3.0 * v * v + 1.0 - m.eps)))
        return bm2, b0, -2.0, 1.0
    if isinstance(m, _models.FCH):
        f1 = _models.dF(v, m.tau)
        f2 = _models.d2F(v, m.tau)
        f3 = _models.d3F(v, m.tau)
        e2 = m.eps ** 2
        b0 = abs(float(np.mean(f2 * f2 - m.eta2 * f2 + f3 * f1)))
        b2 = abs(float(np.mean(e2 * f2 - m.eta1 * e2)))
        return bm2, b0, b2, e2 * e2
    raise TypeError("unknown model")


def precond_symbol(grid, betas, theta_l=1.0):
    """Symbol of L on the half spectrum; the r = 0 entry is left at 0."""
    bm2, b0, b2, b4 = betas
    k2 = grid.k2
    sym = np.zeros_like(k2)
    nz = k2 > 0
    sym[nz] = bm2 / k2[nz] + theta_l * (b0 + b2 * k2[nz] + b4 * k2[nz] ** 2)
    return sym


class Preconditioner:
    """d = L^{-1} r computed with one forward and one inverse transform."""

    def __init__(self, grid, betas, theta_l=1.0):
        self.grid = grid
        self.betas = tuple(float(b) for b in betas)
        self.symbol = precond_symbol(grid, self.betas, theta_l)
        nz = grid.k2 > 0
        self.positive = bool(np.all(self.symbol[nz] > 0.0))

    def apply(self, r):
        g = self.grid
        r_hat = g.fwd(r)
        d_hat = np.zeros_like(r_hat)
        nz = g.k2 > 0
        d_hat[nz] = r_hat[nz] / self.symbol[nz]
        return g.inv(d_hat)


def friction_lambdas(s, etas):
    """lambda_j = (1 - eta_j sqrt(s)) / (1 + eta_j sqrt(s)) of Alg. 2."""
    rs = np.sqrt(s)
    return [(1.0 - e * rs) / (1.0 + e * rs) for e in etas]


def pagd(residual, precond, x0, s, etas, tol, max_iter, accelerated=True, history=None):
    """PAGD with sweeping friction (Alg. 2); PGD (Alg. 1) if not accelerated.

    ``residual(y)`` returns r = -G'(y); ``precond(r)`` returns d = L^{-1} r.
    Returns (x, iterations, status, last ||d||_inf).  ``history``, if a
    list, receives ||d_i||_inf for every iteration.
    """
    lams = friction_lambdas(s, etas)
    x_prev = x0
    x = x0
    dnorm = float("nan")
    for i in range(max_iter):
        lam = lams[i % len(lams)] if accelerated else 0.0
        y = x + lam * (x - x_prev)
        r = residual(y)
        d = precond(r)
        x_prev, x = x, y + s * d
        dnorm = float(np.max(np.abs(d)))
        if history is not None:
            history.append(dnorm)
        if not np.isfinite(dnorm):
            return x, i + 1, NONFINITE, dnorm
        if dnorm < tol:
            return x, i + 1, OK, dnorm
    return x, max_iter, NOCONV, dnorm


def solve_step(problem, x0, s, etas, tol, max_iter, theta_l=1.0, accelerated=True,
               history=None):
    """Set up the averaged-Newton preconditioner at x0 and run PAGD / PGD.

    Returns a dict with the solution and the solver's statistics.
    """
    betas = averaged_newton_betas(problem, x0)
    pre = Preconditioner(problem.grid, betas, theta_l)
    if not pre.positive:
        return dict(x=x0, iters=0, status=PRECOND, dnorm=float("nan"), betas=betas)
    x, it, status, dnorm = pagd(problem.residual, pre.apply, x0, s, etas, tol, max_iter,
                                accelerated=accelerated, history=history)
    return dict(x=x, iters=it, status=status, dnorm=dnorm, betas=betas)
