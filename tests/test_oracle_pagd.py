"""Pins of the oracle's step objective, preconditioner and PAGD (paper Sec. 3.4)."""
import json
import os

import numpy as np
import pytest

from oracle import driver, models, newton, pagd, schemes, spectral

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def smooth_field(g, mean, amp, seed, damp=0.05):
    rng = np.random.default_rng(seed)
    return mean + amp * g.inv(g.fwd(rng.uniform(-1, 1, g.shape)) * np.exp(-damp * g.k2))


PROBLEMS = [
    ("pfc", dict(eps=0.25), schemes.MP, (8, 8), (8.0, 8.0), -0.25, 0.3),
    ("pfc", dict(eps=0.25), schemes.BDF2, (8, 10), (8.0, 10.0), -0.25, 0.3),
    ("fch", dict(eps=0.3, eta1=0.45, eta2=0.6, tau=0.125), schemes.BDF2, (8, 8), (2.0, 2.0), -0.4, 0.2),
    ("fch", dict(eps=0.3, eta1=0.45, eta2=0.6, tau=0.0), schemes.MP, (10, 8), (2.5, 2.0), -0.4, 0.2),
]


def make_problem(kind, params, scheme, shape, lengths, mean, amp, dt=0.05, first=False):
    g = spectral.Grid(shape, lengths)
    m = models.make_model(kind, **params)
    un = smooth_field(g, mean, amp, 1)
    unm1 = smooth_field(g, mean, amp, 2)
    unm1 = unm1 - np.mean(unm1) + np.mean(un)
    a, b, c, th = schemes.coefficients(scheme, dt, None if first else 0.8 * dt)
    return pagd.StepProblem(g, m, a, b, c, th, un, unm1)


@pytest.mark.parametrize("prob", PROBLEMS)
def test_projected_gradient_is_gradient_of_objective(prob):
    """Proposition (eq. misc07 / obj:G'): (G'(v), w)_N = dG_N[w] for mean-zero w."""
    P = make_problem(*prob)
    g = P.grid
    v = smooth_field(g, np.mean(P.u_n), 0.3, 5)
    for seed in range(3):
        w = g.proj0(np.random.default_rng(10 + seed).standard_normal(g.shape))
        h = 1e-4
        f = P.objective
        fd = (-f(v + 2 * h * w) + 8 * f(v + h * w) - 8 * f(v - h * w) + f(v - 2 * h * w)) / (12 * h)
        an = g.inner(P.gradient(v), w)
        assert abs(fd - an) <= 1e-7 * max(1.0, abs(an))


def test_gradient_identity_with_step_residual():
    """G'(v) = (1/M)(-Delta)^{-1} Pi0 F(v) with F = a v + f - M Delta mu(v_breve)."""
    P = make_problem(*PROBLEMS[2])
    g = P.grid
    v = smooth_field(g, np.mean(P.u_n), 0.2, 9)
    F = P.linear_part(v) - P.M * g.lap(P.model.mu(g, P.breve(v)))
    assert np.allclose(P.gradient(v), g.inv_neg_lap(g.proj0(F)) / P.M, atol=1e-10)


def _sweep():
    with open(os.path.join(GOLDEN, "friction_sweep.json")) as fh:
        return json.load(fh)


def test_friction_sweep_from_printed_settings():
    """eta = sqrt of five equally spaced values in [0.1, 2], s = 0.9 (Table
    tab:setting-benchmark): lambda decreases through 0 where eta sqrt(s) = 1."""
    fx = _sweep()
    etas = [np.sqrt(v) for v in fx["eta_squared"]]
    lam = pagd.friction_lambdas(fx["s"], etas)
    assert np.allclose(fx["eta_squared"], np.linspace(0.1, 2.0, 5))
    assert all(l1 > l2 for l1, l2 in zip(lam, lam[1:]))
    assert all(-1 < l < 1 for l in lam)
    for e, l in zip(etas, lam):
        assert (l > 0) == (e * np.sqrt(fx["s"]) < 1)


def test_friction_lambdas_match_hand_worked_values():
    """lambda_j of Alg. 2 at the printed sweep and s = 0.9 against values
    worked out by hand (7/13 and (3 sqrt5 - 7)/2 exactly; the rest in decimal
    arithmetic), so that eta s in place of eta sqrt(s), a swapped sign or a
    dropped term fails."""
    fx = _sweep()
    lam = pagd.friction_lambdas(fx["s"], [np.sqrt(v) for v in fx["eta_squared"]])
    assert abs(fx["lambda"][0] - 7.0 / 13.0) <= 1e-16
    assert abs(fx["lambda"][4] - (3.0 * np.sqrt(5.0) - 7.0) / 2.0) <= 1e-15
    for got, want in zip(lam, fx["lambda"]):
        assert abs(got - want) <= 2e-16, (got, want)


@pytest.mark.parametrize("accelerated", [True, False])
def test_pagd_iterates_on_a_diagonal_quadratic(accelerated):
    """On G(x) = sum h_k x_k^2 / 2 - b_k x_k with diagonal L, each component's
    error obeys e_{i+1} = (1 - s h/l)((1 + lambda_i) e_i - lambda_i e_{i-1}),
    e_{-1} = e_0 (Alg. 2 with x_{-1} = x_0); lambda = 0 gives PGD (Alg. 1).
    The lambda_i come from the hand-worked table, not from the oracle."""
    rng = np.random.default_rng(0)
    h = rng.uniform(0.5, 3.0, 12)
    ell = rng.uniform(0.8, 2.5, 12)
    bvec = rng.standard_normal(12)
    xstar = bvec / h
    s = 0.9
    fx = _sweep()
    etas = [np.sqrt(v) for v in fx["eta_squared"]]
    x0 = rng.standard_normal(12)
    hist = []
    iters = 23
    pagd.pagd(lambda y: bvec - h * y, lambda r: r / ell, x0, s, etas, tol=0.0,
              max_iter=iters, accelerated=accelerated, history=hist)
    # closed-form recurrence for the error, including d_i = (b - h y_i)/l
    e_prev = e = x0 - xstar
    q = 1.0 - s * h / ell
    for i in range(iters):
        lam = fx["lambda"][i % 5] if accelerated else 0.0
        ey = (1 + lam) * e - lam * e_prev
        d = -h * ey / ell
        assert abs(np.max(np.abs(d)) - hist[i]) <= 1e-13 * max(1.0, hist[i])
        e_prev, e = e, q * ey


@pytest.mark.parametrize("prob", PROBLEMS)
def test_pagd_fixed_point_matches_dense_newton(prob):
    P = make_problem(*prob)
    x0 = schemes.extrapolate(P.u_n, P.u_nm1, 0.05, 0.04)
    tol = 1e-12
    out = pagd.solve_step(P, x0, 0.9, driver.PAPER_ETAS, tol, 5000)
    assert out["status"] == pagd.OK
    un, it, res = newton.solve(P, x0)
    assert res < 1e-11
    assert np.max(np.abs(out["x"] - un)) <= 10 * tol
    assert abs(np.mean(out["x"]) - np.mean(P.u_n)) < 1e-14


def linear_rate(kind, params, ubar, k2):
    """Linearised growth rate lambda_k of d_t u = M Delta mu about a constant."""
    if kind == "pfc":
        return k2 * (3 * ubar ** 2 + 1 - params["eps"] - 2 * k2 + k2 * k2)
    e2 = params["eps"] ** 2
    tau = params.get("tau", 0.0)
    f1, f2, f3 = models.dF(ubar, tau), models.d2F(ubar, tau), models.d3F(ubar, tau)
    return k2 * (e2 * e2 * k2 * k2 + e2 * k2 * (2 * f2 - params["eta1"]) + f2 * f2
                 - params["eta2"] * f2 + f3 * f1)


AMP_CASES = [
    ("pfc", dict(eps=0.25), (16, 16), (16.0, 16.0), (1, 2)),
    ("pfc", dict(eps=0.25), (16, 16), (16.0, 16.0), (3, 0)),
    ("fch", dict(eps=0.1, eta1=0.145, eta2=0.2, tau=0.0), (16, 16), (2.0, 2.0), (0, 1)),
    ("fch", dict(eps=0.1, eta1=0.145, eta2=0.2, tau=0.0), (16, 16), (2.0, 2.0), (2, 3)),
]


@pytest.mark.parametrize("kind,params,shape,lengths,mode", AMP_CASES)
@pytest.mark.parametrize("scheme,first", [(schemes.BDF2, True), (schemes.MP, False), (schemes.BDF2, False)])
def test_single_mode_amplification(kind, params, shape, lengths, mode, scheme, first):
    """A small Fourier mode about u = 0 evolves by the scheme's linear factor:
    BE 1/(1 + l dt), MP (1 - l dt/2)/(1 + l dt/2), BDF2 -(b d + c d-)/(a + l)."""
    g = spectral.Grid(shape, lengths)
    m = models.make_model(kind, **params)
    y, x = g.coords()
    ky, kx = 2 * np.pi * mode[0] / lengths[0], 2 * np.pi * mode[1] / lengths[1]
    phi = np.cos(ky * y + kx * x)
    k2 = kx * kx + ky * ky
    lam = linear_rate(kind, params, 0.0, k2)
    dt, dt_old = 0.05, 0.04
    d_n, d_nm1 = 1e-6, 1.3e-6
    un, unm1 = d_n * phi, d_nm1 * phi
    a, b, c, th = schemes.coefficients(scheme, dt, None if first else dt_old)
    P = pagd.StepProblem(g, m, a, b, c, th, un, unm1)
    x0 = un.copy()
    out = pagd.solve_step(P, x0, 0.9, driver.PAPER_ETAS, 1e-20, 5000)
    assert out["status"] == pagd.OK
    if scheme == schemes.MP:
        expect = d_n * (1 - lam * dt / 2) / (1 + lam * dt / 2)
    elif first:
        expect = d_n / (1 + lam * dt)
    else:
        expect = -(b * d_n + c * d_nm1) / (a + lam)
    assert np.max(np.abs(out["x"] - expect * phi)) <= 1e-9 * abs(expect) + 1e-18


@pytest.mark.parametrize("scheme", [schemes.MP, schemes.BDF2])
def test_second_order_in_time(scheme):
    """Self-convergence: halving dt reduces the step-to-step difference about
    four times (second order).  dx = 4 keeps every mode non-stiff at these dt."""
    g = spectral.Grid((16, 16), (64.0, 64.0))
    m = models.PFC(0.25)
    u0 = -0.25 + 0.5 * np.random.default_rng(4).uniform(-1, 1, g.shape)
    T = 2.0
    sols = []
    for n in (8, 16, 32, 64):
        sim = driver.Simulation(g, m, scheme, tol=1e-14, max_iter=5000)
        out = sim.run(u0, T / n, n)
        assert out["status"] == pagd.OK
        sols.append(out["u"])
    e = [np.max(np.abs(sols[i + 1] - sols[i])) for i in range(3)]
    ratios = [e[0] / e[1], e[1] / e[2]]
    assert all(3.6 <= r <= 4.4 for r in ratios), ratios


def test_mass_conserved_and_energy_decreases_pfc():
    g = spectral.Grid((32, 32), (32.0, 32.0))
    m = models.PFC(0.25)
    u0 = -0.25 + 0.05 * np.random.default_rng(0).uniform(-1, 1, g.shape)
    sim = driver.Simulation(g, m, schemes.MP)
    u, up, dto = u0, None, None
    e_prev = m.energy(g, u0)
    for _ in range(6):
        out = sim.step(u, up, 0.1, dto)
        assert out["status"] == pagd.OK
        up, u, dto = u, out["x"], 0.1
        assert abs(np.mean(u) - np.mean(u0)) < 1e-14
        e = m.energy(g, u)
        assert e <= e_prev + 1e-12 * abs(e_prev)
        e_prev = e


def test_mass_conserved_and_energy_decreases_fch():
    g = spectral.Grid((32, 32), (4 * np.pi / 4, 4 * np.pi / 4))
    m = models.FCH(0.1, 0.145, 0.2, 0.0)
    u0 = -0.6 + 0.01 * np.random.default_rng(0).uniform(-1, 1, g.shape)
    sim = driver.Simulation(g, m, schemes.BDF2)
    u, up, dto = u0, None, None
    e_prev = m.energy(g, u0)
    for _ in range(5):
        out = sim.step(u, up, 1e-3, dto)
        assert out["status"] == pagd.OK
        up, u, dto = u, out["x"], 1e-3
        assert abs(np.mean(u) - np.mean(u0)) < 1e-14
        e = m.energy(g, u)
        assert e <= e_prev + 1e-12 * abs(e_prev)
        e_prev = e


def test_backward_euler_step_lowers_the_objective():
    """G(u^1) = E(u^1) + ||u^1 - u^0||_{-1}^2 / (2 M dt) <= G(u^0) = E(u^0)."""
    g = spectral.Grid((16, 16), (16.0, 16.0))
    m = models.PFC(0.25)
    u0 = -0.25 + 0.1 * np.random.default_rng(3).uniform(-1, 1, g.shape)
    dt = 0.5
    a, b, c, th = schemes.coefficients(schemes.BDF2, dt, None)
    P = pagd.StepProblem(g, m, a, b, c, th, u0, None)
    out = pagd.solve_step(P, u0, 0.9, driver.PAPER_ETAS, 1e-10, 1000)
    u1 = out["x"]
    lhs = m.energy(g, u1) + g.neg_norm_sq(u1 - u0) / (2 * dt)
    assert abs(P.objective(u1) - lhs) < 1e-10 * abs(lhs)
    assert lhs <= m.energy(g, u0)


def test_failure_modes():
    g = spectral.Grid((8, 8), (2 * np.pi, 2 * np.pi))
    m = models.PFC(0.25)
    u0 = 0.01 * np.random.default_rng(0).uniform(-1, 1, g.shape)
    # iteration cap
    sim = driver.Simulation(g, m, schemes.MP, max_iter=1)
    assert sim.step(u0, None, 0.1, None)["status"] == pagd.NOCONV
    # averaged-Newton symbol a/k^2 + beta0 - 2 k^2 + k^4 negative at |k| = 1
    sim = driver.Simulation(g, m, schemes.BDF2)
    out = sim.step(u0, None, 100.0, None)
    assert out["status"] == pagd.PRECOND
    # non-finite data
    bad = u0.copy()
    bad[3, 4] = np.nan
    assert driver.Simulation(g, m, schemes.MP).step(bad, None, 0.1, None)["status"] in (
        pagd.NONFINITE, pagd.PRECOND)


@pytest.mark.parametrize("kind,params,ubar,shape,lengths", [
    ("pfc", dict(eps=0.25), -0.3, (8, 8), (8.0, 8.0)),
    ("fch", dict(eps=0.3, eta1=0.45, eta2=0.6, tau=0.125), -1.2, (8, 8), (2.0, 2.0)),
])
@pytest.mark.parametrize("scheme", [schemes.BDF2, schemes.MP])
def test_averaged_newton_symbol_is_exact_hessian_at_constant_state(kind, params, ubar, shape,
                                                                   lengths, scheme):
    """At a constant state the averaged coefficients are exact, so with the
    scheme's own Hessian scale (theta_l = theta) the preconditioner's symbol is
    the spectrum of the dense Hessian (a/M)(-Delta)^{-1} + theta Dmu(u) of G,
    up to the one term the printed FCH coefficient of (-Delta) leaves out:
    the exact coefficient is eps^2 (2 F'' - eta1), the printed one
    eps^2 (F'' - eta1)."""
    g = spectral.Grid(shape, lengths)
    m = models.make_model(kind, **params)
    un = np.full(shape, ubar)
    a, b, c, th = schemes.coefficients(scheme, 0.1, None)
    P = pagd.StepProblem(g, m, a, b, c, th, un, None)
    betas = pagd.averaged_newton_betas(P, un)
    sym = pagd.precond_symbol(g, betas, theta_l=th)
    D = newton.laplacian_matrix(g)
    Dinv = np.linalg.pinv(-D)
    H = a / P.M * Dinv + th * newton.mu_jacobian(m, g, D, un)
    y, x = g.coords()
    for r in ((0, 1), (1, 1), (2, 3), (4, 0), (3, 4)):
        ky, kx = 2 * np.pi * r[0] / lengths[0], 2 * np.pi * r[1] / lengths[1]
        phi = np.cos(ky * y + kx * x).ravel()
        k2 = kx * kx + ky * ky
        ev = float(phi @ H @ phi / (phi @ phi))
        iy = r[0] % shape[0]
        missing = 0.0
        if kind == "fch":
            missing = th * params["eps"] ** 2 * models.d2F(ubar, params["tau"]) * k2
        expect = sym[iy, abs(r[1])] + missing
        assert abs(ev - expect) <= 1e-9 * abs(ev), (r, ev, expect)
        assert abs(sym[iy, abs(r[1])] - (a / k2 + th * (betas[1] + betas[2] * k2 + betas[3] * k2 * k2))) < 1e-9 * abs(ev)


@pytest.mark.parametrize("kind,params", [("pfc", dict(eps=0.25)),
                                         ("fch", dict(eps=0.3, eta1=0.45, eta2=0.6, tau=0.125))])
def test_dense_mu_jacobian_matches_finite_differences(kind, params):
    g = spectral.Grid((6, 8), (3.0, 4.0))
    m = models.make_model(kind, **params)
    u = smooth_field(g, -0.3, 0.3, 8)
    D = newton.laplacian_matrix(g)
    J = newton.mu_jacobian(m, g, D, u)
    v = np.random.default_rng(4).standard_normal(g.shape)
    h = 1e-5
    fd = (m.mu(g, u + h * v) - m.mu(g, u - h * v)) / (2 * h)
    an = (J @ v.ravel()).reshape(g.shape)
    assert np.max(np.abs(fd - an)) <= 1e-6 * np.max(np.abs(an))


def _two_valued_cases():
    with open(os.path.join(GOLDEN, "averaged_newton_two_valued.json")) as fh:
        return json.load(fh)["cases"]


@pytest.mark.parametrize("case", _two_valued_cases(), ids=lambda c: c["name"])
def test_averaged_newton_betas_on_two_valued_fields(case):
    """Sec. 3.4.1's grid means on a field that takes u1 on one half of the grid
    and u2 on the other, against the hand-worked values: a square of the mean
    in place of the mean of squares, an absolute value moved inside the mean,
    or the wrong evaluation point (x0 instead of the midpoint) changes them."""
    shape = (8, 6)
    g = spectral.Grid(shape, (3.0, 2.0))
    if case["model"] == "pfc":
        m = models.make_model("pfc", eps=case["eps"])
    else:
        m = models.make_model("fch", eps=case["eps"], eta1=case["eta1"], eta2=case["eta2"],
                              tau=case["tau"])
    x0 = np.empty(shape)
    x0[: shape[0] // 2] = case["x0"][0]
    x0[shape[0] // 2:] = case["x0"][1]
    un = x0 if case["un"] is None else np.full(shape, case["un"])
    a = 7.5
    P = pagd.StepProblem(g, m, a, -a, 0.0, case["theta"], un, None)
    bm2, b0, b2, b4 = pagd.averaged_newton_betas(P, x0)
    assert bm2 == a
    assert abs(b0 - case["beta0"]) <= 1e-14 * abs(case["beta0"])
    assert abs(b2 - case["beta2"]) <= 1e-13 * abs(case["beta2"])
    assert abs(b4 - case["beta4"]) <= 1e-15
