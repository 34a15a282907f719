"""Fully implicit time discretisations (paper Sec. 3.1.1).

Each step solves a u^{n+1} + b u^n + c u^{n-1} = M Delta mu(u_breve)
(eq. eqn:FCH-semidis-implicit):

* BDF2 (eq. obj:BDF2), variable step, u_breve = u^{n+1}:
      a = 1/dt+ + 1/(dt+ + dt),  b = -1/dt+ - 1/dt,  c = 1/dt - 1/(dt+ + dt)
  with the first step taken by backward Euler, (a, b, c) = (1/dt, -1/dt, 0)
  (caption of Alg. 3).
* Implicit midpoint MP (eq. obj:MP): (a, b, c) = (1/dt, -1/dt, 0) and
  u_breve = (u^{n+1} + u^n) / 2, i.e. theta = 1/2.

``theta`` is the weight of the unknown in u_breve = theta v + (1-theta) u^n.
"""

BDF2 = "bdf2"
MP = "mp"


def coefficients(scheme, dt_new, dt_old=None):
    """Return (a, b, c, theta) for the step of size ``dt_new``.

    ``dt_old`` is the previous step size; ``None`` marks the first step.
    """
    if scheme == BDF2:
        if dt_old is None:
            return 1.0 / dt_new, -1.0 / dt_new, 0.0, 1.0
        a = 1.0 / dt_new + 1.0 / (dt_new + dt_old)
        b = -1.0 / dt_new - 1.0 / dt_old
        c = 1.0 / dt_old - 1.0 / (dt_new + dt_old)
        return a, b, c, 1.0
    if scheme == MP:
        return 1.0 / dt_new, -1.0 / dt_new, 0.0, 0.5
    raise ValueError(f"unknown scheme {scheme!r}")


def extrapolate(u_n, u_nm1, dt_new, dt_old):
    """Initial guess from the two previous solutions (last sentence before Alg. 2).

    The paper names the guess only as an extrapolation of the two previous
    histories; the reading used is its own second-order extrapolation
    u^n + rho (u^n - u^{n-1}), rho = dt_{n+1} / dt_n (Sec. 3.1.1, LBDF2).
    With no history (first step) the guess is u^0.
    """
    if u_nm1 is None or dt_old is None:
        return u_n.copy()
    rho = dt_new / dt_old
    return u_n + rho * (u_n - u_nm1)
