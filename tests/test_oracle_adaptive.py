"""Pins of the adaptive-stepping oracle (Sec. 3.1.2, Alg. 3).

* AM3 weights integrate quadratics in t exactly (third order); with rho = 0
  (first step) they are the trapezoidal rule.
* midAB2 weights reproduce quadratics in t exactly (extrapolation).
* Both error estimates shrink like dt^3 on a smooth solution (second-order
  schemes against a higher-order value), which a wrong weight would break.
* R(v) = M Delta mu(v): closed form on a single PFC Fourier mode (with the
  cubic's third harmonic), the linearised FCH symbol, zero mean, and
  (R(v), mu(v)) = -M ||grad mu||^2 < 0.
* The controller: the step-size formula and its clamps; along a run, the
  time is the sum of accepted sizes, accepted attempts have ERR <= TOL (or
  dt = dt_min), rejected ones ERR > TOL, and mass is conserved; tighter TOL
  gives a more accurate end state.
"""
import math

import numpy as np
import pytest

from oracle import adaptive, driver, models, pagd, spectral


def _quad(c):
    return lambda t: c[0] + c[1] * t + c[2] * t * t


def _quad_int(c, a, b):
    F = lambda t: c[0] * t + c[1] * t * t / 2 + c[2] * t ** 3 / 3
    return F(b) - F(a)


@pytest.mark.parametrize("dt_t,dt_n", [(0.1, 0.1), (0.3, 0.1), (0.02, 0.07), (1.7, 0.4)])
def test_am3_integrates_quadratics(dt_t, dt_n):
    rng = np.random.default_rng(1)
    for _ in range(3):
        c = rng.uniform(-2, 2, 3)
        f = _quad(c)
        w_t, w_n, w_m = adaptive.am3_weights(dt_t, dt_n)
        approx = w_t * f(dt_t) + w_n * f(0.0) + w_m * f(-dt_n)
        exact = _quad_int(c, 0.0, dt_t)
        assert abs(approx - exact) <= 1e-13 * (1 + abs(exact))


def test_am3_uniform_is_adams_moulton_and_first_step_is_trapezoid():
    w = adaptive.am3_weights(0.5, 0.5)
    assert np.allclose(np.array(w) / 0.5, [5 / 12, 8 / 12, -1 / 12], rtol=0, atol=1e-15)
    w_t, w_n, w_m = adaptive.am3_weights(0.5, None)
    assert (w_t, w_n, w_m) == (0.25, 0.25, -0.0)
    # trapezoid: exact for linear, not for quadratic
    assert abs(w_t * 2.0 + w_n * 1.0 - _quad_int((1.0, 2.0, 0.0), 0.0, 0.5)) < 1e-15
    assert abs(w_t * 0.25 - _quad_int((0.0, 0.0, 1.0), 0.0, 0.5)) > 1e-3


@pytest.mark.parametrize("dts", [(0.1, 0.1, 0.1), (0.3, 0.1, 0.2), (0.05, 0.2, 0.13)])
def test_midab2_reproduces_quadratics(dts):
    dt_t, dt_n, dt_m = dts
    c0, c1, c2 = adaptive.midab2_weights(dt_t, dt_n, dt_m)
    assert abs(c0 + c1 + c2 - 1.0) < 1e-13
    rng = np.random.default_rng(2)
    for _ in range(3):
        f = _quad(rng.uniform(-2, 2, 3))
        t_n = 0.4
        val = c0 * f(t_n) + c1 * f(t_n - dt_n) + c2 * f(t_n - dt_n - dt_m)
        assert abs(val - f(t_n + dt_t)) < 1e-12 * (1 + abs(f(t_n + dt_t)))


def test_next_dt_formula_and_clamps():
    nd = adaptive.next_dt
    assert math.isclose(nd(1e-4, 1e-4, 0.1, 1e-6, 1.0), 0.09, rel_tol=1e-14)
    assert math.isclose(nd(1e-4 / 8, 1e-4, 0.1, 1e-6, 1.0), 0.18, rel_tol=1e-14)
    assert nd(1e-4 / 8, 1e-4, 0.1, 1e-6, 0.15) == 0.15
    assert nd(1e6, 1e-4, 0.1, 0.02, 1.0) == 0.02
    assert nd(0.0, 1e-4, 0.1, 1e-6, 0.7) == 0.7
    assert nd(math.inf, 1e-4, 0.1, 1e-6, 0.7) == 1e-6


def test_rhs_single_pfc_mode_closed_form():
    g = spectral.Grid((16, 32), (16.0, 32.0))
    m = models.PFC(0.25)
    y, x = g.coords()
    k = 2 * math.pi * 3 / 32.0          # 3 k stays below the Nyquist mode
    A, M = 0.4, 1.7
    th = k * x
    v = A * np.cos(th)
    q = k * k
    lin = 1 - m.eps - 2 * q + q * q
    exact = -M * (q * (lin * A + 0.75 * A ** 3) * np.cos(th) + 9 * q * 0.25 * A ** 3 * np.cos(3 * th))
    R = adaptive.rhs(m, g, v, M)
    assert np.max(np.abs(R - exact)) <= 1e-11 * np.max(np.abs(exact))


def test_rhs_fch_linearised_symbol():
    g = spectral.Grid((16, 16), (2.0, 2.0))
    m = models.FCH(0.1, 0.145, 0.2, 0.0)
    y, x = g.coords()
    kx, ky = 2 * math.pi * 2 / 2.0, 2 * math.pi * 1 / 2.0
    q = kx * kx + ky * ky
    A = 1e-7
    v = A * np.cos(kx * x + ky * y)
    e2 = m.eps ** 2
    mu1 = e2 * e2 * q * q + e2 * q * (-2.0 - m.eta1) + 1.0 + m.eta2  # F''(0) = -1
    R = adaptive.rhs(m, g, v, 1.0)
    lin = -q * mu1 * v
    assert np.max(np.abs(R - lin)) <= 1e-6 * np.max(np.abs(lin))


@pytest.mark.parametrize("kind", ["pfc", "fch"])
def test_rhs_mass_and_dissipation(kind):
    g = spectral.Grid((16, 16), (16.0, 16.0) if kind == "pfc" else (2.0, 2.0))
    m = models.PFC(0.25) if kind == "pfc" else models.FCH(0.1, 0.145, 0.2, 0.125)
    rng = np.random.default_rng(7)
    v = -0.3 + 0.3 * rng.uniform(-1, 1, g.shape)
    R = adaptive.rhs(m, g, v, 0.8)
    mu = m.mu(g, v)
    assert abs(np.mean(R)) <= 1e-13 * np.max(np.abs(R))
    # (M Delta mu, mu) = -M ||grad mu||^2, grad via its Fourier symbol
    mh = np.fft.rfftn(mu)
    grad2 = g.cell * float(np.sum(g.k2 * np.abs(mh) ** 2 * np.where(
        np.arange(mh.shape[-1]) % (g.shape[-1] // 2) == 0, 1.0, 2.0))) / g.npoints
    assert grad2 > 0
    assert math.isclose(g.inner(R, mu), -0.8 * grad2, rel_tol=1e-10)


def _smooth_pfc():
    g = spectral.Grid((16, 16), (16.0, 16.0))
    m = models.PFC(0.25)
    y, x = g.coords()
    u0 = -0.25 + 0.1 * np.cos(2 * math.pi * x / 16) + 0.05 * np.sin(2 * math.pi * 2 * y / 16)
    return g, m, u0


def _estimate_after(scheme, h, nsteps):
    g, m, u0 = _smooth_pfc()
    est = adaptive.MIDAB2 if scheme == "mp" else adaptive.AM3
    run = adaptive.AdaptiveRun(g, m, scheme, u0, 1.0, h, h, est)
    run.sim.tol = 1e-13
    for _ in range(nsteps):
        assert run.attempt()["accepted"]
    u_t, status, _ = run.solve(h)
    assert status == pagd.OK
    return run.estimate(u_t, run.rhs(u_t), h)[0]


@pytest.mark.parametrize("scheme", ["bdf2", "mp"])
def test_error_estimates_scale_as_dt_cubed(scheme):
    """Estimate of the step from t = 1.6 after a fixed-step history (long
    enough for BDF2's parasitic mode from the backward-Euler start to decay)."""
    e1 = _estimate_after(scheme, 0.1, 16)
    e2 = _estimate_after(scheme, 0.05, 32)
    assert 7.0 <= e1 / e2 <= 9.0, (e1, e2)


def _invariants(run, log, u0):
    acc = [r for r in log if r["accepted"]]
    assert math.isclose(run.t, sum(r["dt"] for r in acc), rel_tol=1e-14)
    assert run.n == len(acc)
    prev = run.dt_min
    for k, r in enumerate(log):
        if k == 0:
            assert r["dt"] == run.dt_min
        else:
            assert r["dt"] == adaptive.next_dt(log[k - 1]["err"], run.tol, log[k - 1]["dt"],
                                               run.dt_min, run.dt_max)
        if r["accepted"]:
            assert r["err"] <= run.tol or r["dt"] <= run.dt_min
        else:
            assert r["err"] > run.tol and r["dt"] > run.dt_min
        prev = r["dt"]
    assert abs(np.mean(run.u) - np.mean(u0)) <= 1e-13


@pytest.mark.parametrize("scheme", ["bdf2", "mp", "lbdf2", "lmp"])
def test_adaptive_run_invariants(scheme):
    g, m, u0 = _smooth_pfc()
    rng = np.random.default_rng(3)
    u0 = u0 + 0.02 * rng.uniform(-1, 1, g.shape)
    run = adaptive.AdaptiveRun(g, m, scheme, u0, 1e-4, 1e-3, 5.0)
    log = run.run(4.0)
    assert run.t >= 4.0
    _invariants(run, log, u0)


@pytest.mark.parametrize("scheme", ["bdf2", "mp"])
@pytest.mark.parametrize("dt_try,solved", [(0.5, True), (30.0, False)])
def test_rejected_attempt_keeps_history(scheme, dt_try, solved):
    """A converged attempt with ERR > TOL, and a failed solve (ERR = inf,
    next size dt_min), both leave the history untouched."""
    g, m, u0 = _smooth_pfc()
    u0 = u0 + 0.1 * np.random.default_rng(3).uniform(-1, 1, g.shape)
    run = adaptive.AdaptiveRun(g, m, scheme, u0, 1e-5, 1e-3, 50.0)
    for _ in range(4):
        run.attempt()
    t, n, hist, dts = run.t, run.n, [h.copy() for h in run.hist], list(run.dts)
    run.dt_try = dt_try
    with np.errstate(over="ignore", invalid="ignore"):
        rec = run.attempt()
    assert (rec["status"] == pagd.OK) == solved
    assert not rec["accepted"] and rec["err"] > run.tol
    assert (run.t, run.n, run.dts) == (t, n, dts)
    assert all(np.array_equal(a, b) for a, b in zip(run.hist, hist))
    assert run.dt_try == adaptive.next_dt(rec["err"], run.tol, dt_try, 1e-3, 50.0) < dt_try
    if not solved:
        assert run.dt_try == 1e-3


def test_tighter_tolerance_is_more_accurate():
    g, m, u0 = _smooth_pfc()
    errs = []
    for tol in (1e-3, 1e-5):
        run = adaptive.AdaptiveRun(g, m, "bdf2", u0, tol, 1e-3, 2.0)
        run.run(3.0)
        n = 400
        ref = driver.Simulation(g, m, "bdf2", tol=1e-12).run(u0, run.t / n, n)["u"]
        errs.append(np.linalg.norm(run.u - ref) / np.linalg.norm(ref))
    assert errs[1] < errs[0] / 10, errs
