"""Float32 FNO kernels against the float64 reference network, and the learned
initial guess inside pfch_step.

Forward and gradient are compared on tiny 2D and 3D networks at
float32-scaled tolerances; the learned guess must leave the converged step
within the PAGD tolerance of the extrapolated-guess step, with the same
mass, and fall back to the extrapolated guess when its own solve fails."""
import dataclasses

import numpy as np
import pytest

import workloads as W
from oracle import fno as ofno
from tests._common import desc_for, oracle_run, rel_l2

pytestmark = pytest.mark.gpu

NETS = [  # (width, modes, layers, ny, nx, batch)
    (4, 3, 2, 12, 12, 2),
    (5, 3, 3, 8, 12, 3),   # rectangular
    (4, 3, 2, 6, 10, 2),   # 2M == Ny: every ky kept
]


NETS3 = [  # (width, modes, layers, nz, ny, nx, batch)
    (3, 2, 2, 6, 8, 10, 2),
    (4, 2, 3, 4, 6, 8, 1),   # 2M == Nz: every kz kept
    (2, 3, 2, 8, 6, 12, 2),  # 2M == Ny
]


def _split(net):
    """(width, modes, layers, grid, batch) of a 2D or 3D net tuple."""
    return net[0], net[1], net[2], tuple(net[3:-1]), net[-1]


def _inputs(net, seed):
    w, m, l, grid, b = _split(net)
    rng = np.random.default_rng(seed)
    theta = ofno.init_params(w, m, l, seed=seed, ndim=len(grid))
    x = rng.normal(size=(b, 2) + grid)
    t = rng.normal(size=(b,) + grid) * 0.5
    # round to float32 first so both sides see the same numbers
    return theta.astype(np.float32), x.astype(np.float32), t.astype(np.float32)


def _groups(w, m, l, ndim=2):
    """(name, slice) of each parameter block in the flat layout."""
    out, o = [], 0
    for name, n in [("P", 2 * w), ("pb", w)]:
        out.append((name, slice(o, o + n)))
        o += n
    for k in range(l):
        for name, n in [(f"R{k}", w * w * ofno.n_modes(m, ndim) * 2), (f"W{k}", w * w), (f"b{k}", w)]:
            out.append((name, slice(o, o + n)))
            o += n
    for name, n in [("Q", w), ("qb", 1)]:
        out.append((name, slice(o, o + n)))
        o += n
    return out


def _net(net, theta):
    import torch
    from paper_2204_07247_amd import pfch
    w, m, l, grid, b = _split(net)
    f = pfch.Fno(w, m, l, *grid, max_batch=b)
    assert f.n_params == theta.size
    f.set_params(torch.from_numpy(theta).cuda())
    return f


def _rel(a, b):
    return float(np.linalg.norm(np.ravel(a - b)) / max(np.linalg.norm(np.ravel(b)), 1e-30))


@pytest.mark.parametrize("net", NETS + NETS3, ids=lambda n: "x".join(map(str, n)))
def test_forward_matches_reference(net):
    import torch
    w, m, l, grid, b = _split(net)
    theta, x, _ = _inputs(net, seed=11)
    print(f"fno forward {net}", flush=True)
    f = _net(net, theta)
    y = f.forward(torch.from_numpy(x).cuda()).cpu().numpy()
    ref, _ = ofno.forward(theta.astype(np.float64), x.astype(np.float64), w, m, l)
    assert y.shape == ref.shape
    assert _rel(y, ref) <= 1e-5, _rel(y, ref)
    f.close()


@pytest.mark.parametrize("net", NETS + NETS3, ids=lambda n: "x".join(map(str, n)))
def test_gradient_matches_reference(net):
    import torch
    w, m, l, grid, b = _split(net)
    theta, x, t = _inputs(net, seed=12)
    print(f"fno grad {net}", flush=True)
    f = _net(net, theta)
    loss, g = f.grad(torch.from_numpy(x).cuda(), torch.from_numpy(t).cuda())
    g = g.cpu().numpy().astype(np.float64)
    gref, lref = ofno.backward(theta.astype(np.float64), x.astype(np.float64), t.astype(np.float64),
                               w, m, l)
    assert abs(loss - lref) <= 1e-5 * abs(lref)
    assert _rel(g, gref) <= 1e-4, _rel(g, gref)
    for name, sl in _groups(w, m, l, len(grid)):
        assert _rel(g[sl], gref[sl]) <= 1e-3, (name, _rel(g[sl], gref[sl]))
    f.close()


def test_3d_network_rejects_mismatched_sizes():
    from paper_2204_07247_amd import pfch
    with pytest.raises(pfch.PfchError):
        pfch.Fno(4, 3, 1, 4, 8, 8)      # 2M > Nz
    with pytest.raises(pfch.PfchError):
        pfch.Fno(4, 2, 1, 8, 8, 3)      # M > Nx / 2
    assert pfch.fno_num_params(4, 2, 1, ndim=3) == ofno.n_params(4, 2, 1, ndim=3)


def test_adam_update_and_training_reduce_loss():
    """One Adam update equals the textbook formula on the returned gradient;
    a few dozen updates on a fixed batch cut the loss."""
    import torch
    net = (4, 3, 2, 12, 12, 4)
    theta, x, _ = _inputs(net, seed=13)
    t = (0.5 * x[:, 0] - 0.3 * x[:, 1]).astype(np.float32)  # a target the network can fit
    f = _net(net, theta)
    xd, td = torch.from_numpy(x).cuda(), torch.from_numpy(t).cuda()
    loss0, g = f.grad(xd, td)
    lr, b1, b2, eps = 1e-2, 0.9, 0.999, 1e-8
    f.adam_step(lr, 1, b1, b2, eps)
    th1 = f.get_params().cpu().numpy().astype(np.float64)
    g = g.cpu().numpy().astype(np.float64)
    mh = (1 - b1) * g / (1 - b1)
    vh = (1 - b2) * g * g / (1 - b2)
    expect = theta.astype(np.float64) - lr * mh / (np.sqrt(vh) + eps)
    assert np.max(np.abs(th1 - expect)) <= 1e-6
    for k in range(2, 41):
        f.grad(xd, td, want_grad=False, want_loss=False)
        f.adam_step(lr, k, b1, b2, eps)
    loss1, _ = f.grad(xd, td, want_grad=False)
    assert loss1 < 0.6 * loss0, (loss0, loss1)
    f.close()


def _history(w, nsteps):
    """State after `nsteps` plain steps (u^n, u^{n-1}, dt_prev) on the GPU."""
    import torch
    from paper_2204_07247_amd import pfch
    ctx = pfch.Context([desc_for(w)])
    u0 = torch.from_numpy(W.initial_condition(w)).cuda()
    ctx.set_state(0, u0)
    for _ in range(nsteps):
        rc, _ = ctx.step(w.dt)
        assert rc == pfch.PFCH_OK
    un, unm1 = torch.empty_like(u0), torch.empty_like(u0)
    _, dtp, k = ctx.get_state(0, un, unm1)
    ctx.close()
    return un, unm1, dtp, k


def _one_step(w, un, unm1, dtp, k, fno=None, norm=None, guess=0, max_iter=None):
    import torch
    from paper_2204_07247_amd import pfch
    d = desc_for(w)
    d.guess = guess
    if max_iter is not None:
        d.max_iter = max_iter
    ctx = pfch.Context([d])
    ctx.set_state(0, un, unm1, t=0.0, dt_prev=dtp, step_index=k)
    if fno is not None:
        ctx.set_fno(0, fno, norm)
    rc, st = ctx.step(w.dt)
    out = torch.empty_like(un)
    ctx.get_state(0, out)
    ctx.close()
    return rc, st[0], out.cpu().numpy()


@pytest.mark.parametrize("w", [
    dataclasses.replace(W.PFC64_MP, seeds=(0,)),
    dataclasses.replace(W.FCH256_BDF2, shape=(64, 64), seeds=(1,)),
    dataclasses.replace(W.PFC192_3D, shape=(16, 16, 32), lengths=(16.0, 16.0, 32.0), seeds=(2,)),
], ids=lambda w: f"{w.model}-{w.scheme}-{len(w.shape)}d")
def test_learned_guess_step_within_tolerance(w):
    """From the same state, the learned-guess step and the extrapolated-guess
    step both converge; the solutions differ within the PAGD tolerance and
    have the same mass."""
    from paper_2204_07247_amd import pfch
    print(f"learned guess {w.model} {w.scheme} {w.shape}", flush=True)
    un, unm1, dtp, k = _history(w, 3)
    fno = pfch.Fno(8, 4, 2, *w.shape)
    fno.init_params(seed=5)
    u = un.cpu().numpy()
    du = (un - unm1).cpu().numpy()
    norm = (float(u.mean()), float(u.std()), float(du.std()), 0.1 * float(du.std()))
    rc_p, st_p, plain = _one_step(w, un, unm1, dtp, k)
    rc_l, st_l, learned = _one_step(w, un, unm1, dtp, k, fno=fno, norm=norm, guess=1)
    assert rc_p == pfch.PFCH_OK and rc_l == pfch.PFCH_OK
    assert st_p["guess"] == 0 and st_l["guess"] == 1
    assert st_l["dnorm"] < w.tol and st_p["dnorm"] < w.tol
    assert np.max(np.abs(learned - plain)) <= 1e-9
    assert abs(learned.mean() - plain.mean()) <= 1e-14
    # without desc.guess = 1 the attached network is not used
    rc_n, st_n, same = _one_step(w, un, unm1, dtp, k, fno=fno, norm=norm, guess=0)
    assert rc_n == pfch.PFCH_OK and st_n["guess"] == 0 and np.array_equal(same, plain)
    fno.close()


def test_learned_gain_is_the_last_steps_least_squares_gain():
    """The first learned step after pfch_set_fno (or pfch_set_state) uses
    gain 1; the next one the least-squares gain of the first step's
    correction c = so (y - mean y) against the solution x it reached,
    sum c (x - e) / sum c^2 with e the extrapolation, clamped to [0, 1],
    recomputed here from the network's own forward pass on the same inputs.
    After pfch_set_state the gain is 1 again and the first learned step
    repeats bitwise; steps without the learned guess report no gain."""
    import math

    import torch
    from paper_2204_07247_amd import pfch
    w = dataclasses.replace(W.FCH256_BDF2, shape=(64, 64), seeds=(1,))
    un, unm1, dtp, k = _history(w, 3)
    fno = pfch.Fno(8, 4, 2, *w.shape)
    rng = np.random.default_rng(11)
    fno.set_params(torch.from_numpy(rng.normal(0.0, 0.3, fno.n_params).astype(np.float32)).cuda())
    u = un.cpu().numpy()
    du = (un - unm1).cpu().numpy()
    norm = [float(u.mean()), float(u.std()), float(du.std()), 1.0]
    # the network's output on the first step's inputs (dt equal to dt_prev:
    # extrapolation factor 1); the output scale so makes the correction five
    # times the largest |u^n - u^{n-1}|, far larger than the step's own
    # correction, so that its least-squares gain lies well inside (0, 1)
    X = torch.empty((1, 2) + tuple(w.shape), dtype=torch.float32, device="cuda")
    fno.prepare(unm1, un, None, 1.0, norm, X[0])
    y = fno.forward(X)[0].double().cpu().numpy()
    norm[3] = so = 5.0 * float(np.abs(du).max()) / float(np.abs(y - y.mean()).max())
    d = desc_for(w)
    d.guess = 1
    ctx = pfch.Context([d])
    ctx.set_state(0, un, unm1, t=0.0, dt_prev=dtp, step_index=k)
    ctx.set_fno(0, fno, norm)
    rc, st = ctx.step(w.dt)
    assert rc == pfch.PFCH_OK and st[0]["guess"] == 1 and st[0]["gain"] == 1.0
    x1 = torch.empty_like(un)
    ctx.get_state(0, x1)
    c = so * (y - y.mean())
    e = 2.0 * u - unm1.cpu().numpy()
    x0 = e + c
    cf = c.astype(np.float32).astype(np.float64)
    raw = 1.0 + float(np.sum(cf * (x1.cpu().numpy() - x0)) / np.sum(cf * cf))
    want = min(1.0, max(0.0, raw))
    rc, st = ctx.step(w.dt)
    assert rc == pfch.PFCH_OK and st[0]["guess"] == 1
    print(f"gain of the second step {st[0]['gain']:.9f}, recomputed {want:.9f} (unclamped {raw:.9f})",
          flush=True)
    assert abs(st[0]["gain"] - want) <= 1e-6
    assert 0.0 < st[0]["gain"] < 0.5
    # a new history: gain 1, the first step again bit for bit
    ctx.set_state(0, un, unm1, t=0.0, dt_prev=dtp, step_index=k)
    rc, st = ctx.step(w.dt)
    again = torch.empty_like(un)
    ctx.get_state(0, again)
    assert rc == pfch.PFCH_OK and st[0]["gain"] == 1.0 and torch.equal(again, x1)
    ctx.close()
    # the extrapolated guess reports no gain
    rc, st, _ = _one_step(w, un, unm1, dtp, k)
    assert rc == pfch.PFCH_OK and st["guess"] == 0 and math.isnan(st["gain"])
    fno.close()


def test_learned_gate_closes_below_the_gain_bound_and_probes():
    """A learned step whose fitted gain is below 0.98 leaves the correction
    out and closes the gate: the next 16 steps take the extrapolated guess
    (no gain reported), then two probe steps take the network again (the
    first adds its correction with gain 0, so that its solution is that of
    the extrapolated guess within the tolerance; the second reports the
    gain fitted to the first), and a probe gain below the bound closes the
    gate again for twice as long; pfch_set_state opens it."""
    import math

    import torch
    from paper_2204_07247_amd import pfch
    w = dataclasses.replace(W.FCH256_BDF2, shape=(64, 64), seeds=(1,))
    un, unm1, dtp, k = _history(w, 3)
    fno = pfch.Fno(8, 4, 2, *w.shape)
    rng = np.random.default_rng(11)
    fno.set_params(torch.from_numpy(rng.normal(0.0, 0.3, fno.n_params).astype(np.float32)).cuda())
    u = un.cpu().numpy()
    du = (un - unm1).cpu().numpy()
    norm = [float(u.mean()), float(u.std()), float(du.std()), 1.0]
    X = torch.empty((1, 2) + tuple(w.shape), dtype=torch.float32, device="cuda")
    fno.prepare(unm1, un, None, 1.0, norm, X[0])
    y = fno.forward(X)[0].double().cpu().numpy()
    # a correction five times the largest |u^n - u^{n-1}|: fitted gains far below 0.98
    norm[3] = 5.0 * float(np.abs(du).max()) / float(np.abs(y - y.mean()).max())
    d = desc_for(w)
    d.guess = 1
    ctx = pfch.Context([d])
    ctx.set_state(0, un, unm1, t=0.0, dt_prev=dtp, step_index=k)
    ctx.set_fno(0, fno, norm)
    kinds = []
    gains = []
    for _ in range(2 + 16 + 2 + 32 + 2 + 1):
        rc, st = ctx.step(w.dt)
        assert rc == pfch.PFCH_OK
        kinds.append(st[0]["guess"])
        gains.append(st[0]["gain"])
    print(f"guess kinds {kinds}, gains {[round(g, 4) for g in gains]}", flush=True)
    assert kinds == [1, 1] + [0] * 16 + [1, 1] + [0] * 32 + [1, 1] + [0]
    assert gains[0] == 1.0 and gains[1] < 0.98
    off = gains[2:18] + gains[20:52] + gains[54:]
    assert all(math.isnan(g) for g in off)
    assert gains[18] == 0.0 and gains[52] == 0.0  # first probe steps: the correction with gain 0
    assert gains[19] < 0.98 and gains[53] < 0.98
    # a new history opens the gate
    ctx.set_state(0, un, unm1, t=0.0, dt_prev=dtp, step_index=k)
    rc, st = ctx.step(w.dt)
    assert rc == pfch.PFCH_OK and st[0]["guess"] == 1 and st[0]["gain"] == 1.0
    ctx.close()
    fno.close()


def test_failed_learned_guess_falls_back_to_extrapolation():
    """A guess from which the solve fails (here: non-finite residual) is
    replaced by the extrapolated guess; the step then equals the plain step
    bitwise."""
    from paper_2204_07247_amd import pfch
    w = dataclasses.replace(W.PFC64_MP, seeds=(2,))
    un, unm1, dtp, k = _history(w, 2)
    fno = pfch.Fno(4, 3, 1, *w.shape)
    fno.init_params(seed=9)
    norm = (0.0, 1.0, 1.0, 1e150)  # correction of order 1e150: the cubic term overflows
    rc_p, st_p, plain = _one_step(w, un, unm1, dtp, k, max_iter=60)
    rc_l, st_l, learned = _one_step(w, un, unm1, dtp, k, fno=fno, norm=norm, guess=1, max_iter=60)
    assert rc_p == pfch.PFCH_OK and rc_l == pfch.PFCH_OK
    assert st_l["guess"] == 2
    assert st_l["iters"] == st_p["iters"]
    assert np.array_equal(learned, plain)
    fno.close()


def test_network_grid_must_match_instance():
    """A 2D network does not attach to a 3D instance and vice versa."""
    from paper_2204_07247_amd import pfch
    w3 = dataclasses.replace(W.PFC192_3D, shape=(16, 16, 32), lengths=(16.0, 16.0, 32.0))
    ctx = pfch.Context([desc_for(w3, guess=1)])
    norm = (0.0, 1.0, 1.0, 1.0)
    f2 = pfch.Fno(4, 2, 1, 16, 32)
    f3 = pfch.Fno(4, 2, 1, 16, 16, 32)
    f3b = pfch.Fno(4, 2, 1, 8, 16, 32)
    with pytest.raises(pfch.PfchError):
        ctx.set_fno(0, f2, norm)
    with pytest.raises(pfch.PfchError):
        ctx.set_fno(0, f3b, norm)
    ctx.set_fno(0, f3, norm)
    ctx.close()
    for f in (f2, f3, f3b):
        f.close()


def test_trained_network_gains_over_extrapolation():
    """Trained on solver trajectories (PFC 64^2, MP), the network's guess is
    closer to the converged u^{n+1} than the extrapolated guess on states it
    was not trained on, and the learned steps from those states converge to
    the plain steps' solutions within the tolerance in fewer PAGD iterations
    in total."""
    import torch
    from paper_2204_07247_amd import learned, pfch
    base = W.PFC64_MP
    ws = [dataclasses.replace(base, seeds=(s,)) for s in range(100, 104)]
    u0s = [torch.from_numpy(W.initial_condition(w)).cuda() for w in ws]
    cfg = learned.TrainConfig(width=8, modes=8, layers=2, batch=8, epochs=25, lr=3e-3, seed=1)
    print("train on 4 x 30 steps of pfc64", flush=True)
    tr = learned.train(ws, u0s, 30, cfg)
    assert tr.val_loss[-1] < tr.val_loss[0]
    # held-out trajectory: seed 7, states after 10 steps
    w = dataclasses.replace(base, seeds=(7,))
    states = learned.trajectories([w], [torch.from_numpy(W.initial_condition(w)).cuda()], 14)[0]
    mu, su, sd, so = tr.norm
    x = torch.empty((1, 2) + tuple(w.shape), dtype=torch.float32, device="cuda")
    gains = []
    for n in range(10, 13):
        unm1, un, unp1 = states[n - 1], states[n], states[n + 1]
        tr.fno.prepare(unm1, un, None, 1.0, tr.norm, x[0])
        y = tr.fno.forward(x)[0].double()
        extrap = 2.0 * un - unm1
        guess = extrap + so * (y - y.mean())
        e_plain = float((extrap - unp1).norm())
        e_learned = float((guess - unp1).norm())
        gains.append(e_plain / e_learned)
        assert abs(float(guess.mean() - extrap.mean())) <= 1e-14
    print(f"guess error, extrapolated / learned: {gains}", flush=True)
    assert min(gains) > 1.5, gains
    # the learned steps themselves: converged, within the tolerance of the
    # plain steps, and in fewer PAGD iterations over the held-out states
    its_p, its_l = [], []
    for n in range(10, 13):
        un, unm1, dtp = states[n].clone(), states[n - 1].clone(), w.dt
        rc_p, st_p, plain = _one_step(w, un, unm1, dtp, n)
        rc_l, st_l, got = _one_step(w, un, unm1, dtp, n, fno=tr.fno, norm=tr.norm, guess=1)
        assert rc_p == pfch.PFCH_OK and rc_l == pfch.PFCH_OK and st_l["guess"] == 1
        assert np.max(np.abs(got - plain)) <= 1e-9
        its_p.append(st_p["iters"])
        its_l.append(st_l["iters"])
    print(f"iterations plain {its_p}, learned {its_l}", flush=True)
    assert sum(its_l) < sum(its_p), (its_p, its_l)
    tr.fno.close()


def test_learned_trajectory_matches_oracle_within_tolerance():
    """A trained network's gated learned guess over steps 11-30 of a
    held-out PFC 64^2 trajectory (steps 1-10 with the extrapolated guess):
    every step converges, the network runs on most of them, the mass is the
    oracle's, and the trajectory stays within the accumulated PAGD tolerance
    of the oracle's (extrapolated-guess) trajectory.  Each step's solution, from either guess, lies within about
    kappa tol of the step problem's solution (kappa the conditioning of the
    preconditioned problem, a few units), and a stable scheme carries such
    differences on without growth beyond 1 + O(dt) per step: after n = 20
    learned steps they stay below 2 kappa tol n = 2e-8 for kappa = 5.  The
    learned steps take fewer PAGD iterations in total than the oracle's
    steps 11-30."""
    import torch
    from paper_2204_07247_amd import learned, pfch
    base = W.PFC64_MP
    ws = [dataclasses.replace(base, seeds=(s,)) for s in range(100, 104)]
    u0s = [torch.from_numpy(W.initial_condition(w)).cuda() for w in ws]
    cfg = learned.TrainConfig(width=8, modes=8, layers=2, batch=8, epochs=25, lr=3e-3, seed=1)
    print("train on 4 x 30 steps of pfc64", flush=True)
    tr = learned.train(ws, u0s, 30, cfg)
    w = dataclasses.replace(base, seeds=(7,))
    u0 = W.initial_condition(w)
    n0, n = 10, 20
    ref, ref_iters = oracle_run(w, u0, n0 + n)
    ref_iters = ref_iters[n0:]
    ctx = pfch.Context([desc_for(w, guess=1)])
    ctx.set_state(0, torch.from_numpy(u0).cuda())
    for _ in range(n0):  # no network attached yet: the extrapolated guess
        rc, st = ctx.step(w.dt)
        assert rc == pfch.PFCH_OK and st[0]["guess"] == 0
    ctx.set_fno(0, tr.fno, tr.norm)
    kinds, iters = [], []
    for _ in range(n):
        rc, st = ctx.step(w.dt)
        assert rc == pfch.PFCH_OK
        kinds.append(st[0]["guess"])
        iters.append(st[0]["iters"])
    got = torch.empty(w.shape, dtype=torch.float64, device="cuda")
    ctx.get_state(0, got)
    ctx.close()
    tr.fno.close()
    got = got.cpu().numpy()
    diff = float(np.max(np.abs(got - ref)))
    print(f"guess kinds {kinds}; iterations learned {sum(iters)}, oracle {sum(ref_iters)}; "
          f"max |u - u_oracle| {diff:.3e}, rel L2 {rel_l2(got, ref):.3e}", flush=True)
    assert kinds.count(1) >= n // 2
    assert diff <= 2.0 * 5.0 * w.tol * n
    assert abs(float(got.mean()) - float(ref.mean())) <= 1e-13
    assert sum(iters) < sum(ref_iters)


def test_coarse_learned_trajectory_matches_oracle_within_tolerance():
    """FCH 128^2 BDF2 with the network on a coarser 32^2 grid (band-limited
    resampling in and out, the combined set's path), trained on 4 x 40
    steps: steps 11-30 of a held-out trajectory with the gated learned
    guess converge, keep the oracle's mass and stay within the accumulated
    PAGD tolerance (the bound of the PFC trajectory test) of the oracle's
    trajectory."""
    import torch
    from paper_2204_07247_amd import learned, pfch
    base = dataclasses.replace(W.FCH256_BDF2, shape=(128, 128))
    ws = [dataclasses.replace(base, seeds=(s,)) for s in range(200, 204)]
    u0s = [torch.from_numpy(W.initial_condition(w)).cuda() for w in ws]
    cfg = learned.TrainConfig(width=8, modes=8, layers=2, batch=8, epochs=10, lr=3e-3, seed=2,
                              grid=(32, 32))
    print("train on 4 x 40 steps of fch128, network on 32^2", flush=True)
    tr = learned.train(ws, u0s, 40, cfg)
    w = dataclasses.replace(base, seeds=(9,))
    u0 = W.initial_condition(w)
    n0, n = 10, 20
    ref, ref_iters = oracle_run(w, u0, n0 + n)
    ctx = pfch.Context([desc_for(w, guess=1)])
    ctx.set_state(0, torch.from_numpy(u0).cuda())
    for _ in range(n0):
        rc, st = ctx.step(w.dt)
        assert rc == pfch.PFCH_OK and st[0]["guess"] == 0
    ctx.set_fno(0, tr.fno, tr.norm)
    kinds, iters = [], []
    for _ in range(n):
        rc, st = ctx.step(w.dt)
        assert rc == pfch.PFCH_OK
        kinds.append(st[0]["guess"])
        iters.append(st[0]["iters"])
    got = torch.empty(w.shape, dtype=torch.float64, device="cuda")
    ctx.get_state(0, got)
    ctx.close()
    tr.fno.close()
    got = got.cpu().numpy()
    diff = float(np.max(np.abs(got - ref)))
    print(f"guess kinds {kinds}; iterations learned {sum(iters)}, oracle {sum(ref_iters[n0:])}; "
          f"max |u - u_oracle| {diff:.3e}, rel L2 {rel_l2(got, ref):.3e}", flush=True)
    assert kinds[:2] == [1, 1]
    assert diff <= 2.0 * 5.0 * w.tol * n
    assert abs(float(got.mean()) - float(ref.mean())) <= 1e-13


def test_3d_learned_trajectory_matches_oracle_within_tolerance():
    """PFC 3D (16 x 16 x 32, BDF2) with a 3D network trained on 4 x 20
    steps: steps 6-15 of a held-out trajectory with the gated learned guess
    converge, keep the oracle's mass and stay within the accumulated PAGD
    tolerance (2 kappa tol n, kappa = 5) of the oracle's trajectory."""
    import torch
    from paper_2204_07247_amd import learned, pfch
    base = dataclasses.replace(W.PFC192_3D, shape=(16, 16, 32), lengths=(16.0, 16.0, 32.0))
    ws = [dataclasses.replace(base, seeds=(s,)) for s in range(300, 304)]
    u0s = [torch.from_numpy(W.initial_condition(w)).cuda() for w in ws]
    cfg = learned.TrainConfig(width=8, modes=4, layers=2, batch=4, epochs=10, lr=3e-3, seed=3)
    print("train on 4 x 20 steps of pfc 16x16x32", flush=True)
    tr = learned.train(ws, u0s, 20, cfg)
    w = dataclasses.replace(base, seeds=(11,))
    u0 = W.initial_condition(w)
    n0, n = 5, 10
    ref, ref_iters = oracle_run(w, u0, n0 + n)
    ctx = pfch.Context([desc_for(w, guess=1)])
    ctx.set_state(0, torch.from_numpy(u0).cuda())
    for _ in range(n0):
        rc, st = ctx.step(w.dt)
        assert rc == pfch.PFCH_OK and st[0]["guess"] == 0
    ctx.set_fno(0, tr.fno, tr.norm)
    kinds, iters = [], []
    for _ in range(n):
        rc, st = ctx.step(w.dt)
        assert rc == pfch.PFCH_OK
        kinds.append(st[0]["guess"])
        iters.append(st[0]["iters"])
    got = torch.empty(w.shape, dtype=torch.float64, device="cuda")
    ctx.get_state(0, got)
    ctx.close()
    tr.fno.close()
    got = got.cpu().numpy()
    diff = float(np.max(np.abs(got - ref)))
    print(f"guess kinds {kinds}; iterations learned {sum(iters)}, oracle {sum(ref_iters[n0:])}; "
          f"max |u - u_oracle| {diff:.3e}, rel L2 {rel_l2(got, ref):.3e}", flush=True)
    assert kinds[:2] == [1, 1]
    assert diff <= 2.0 * 5.0 * w.tol * n
    assert abs(float(got.mean()) - float(ref.mean())) <= 1e-13


def _smooth(shape, seed, mean, amp):
    rng = np.random.default_rng(seed)
    f = rng.uniform(-1, 1, shape)
    k = np.fft.fft2(f)
    ky = np.fft.fftfreq(shape[0])[:, None]
    kx = np.fft.fftfreq(shape[1])[None, :]
    return mean + amp * np.real(np.fft.ifft2(k * np.exp(-40.0 * (kx * kx + ky * ky)))) + 0.1 * amp * f


@pytest.mark.parametrize("fine,coarse", [((128, 64), (32, 32)), ((256, 256), (64, 64)), ((64, 64), (64, 16))])
def test_prepare_resampled_matches_oracle(fine, coarse):
    """Network inputs and target of a sample whose fields live on a finer grid
    than the network's: the band-limited resampling of the normalised fields
    (reference: modes |k| < Nc/2 kept, evaluated at the network's points),
    at float32 accuracy."""
    import torch
    from paper_2204_07247_amd import pfch
    print(f"prepare resampled {fine} -> {coarse}", flush=True)
    unm1 = _smooth(fine, 1, -0.4, 0.3)
    un = unm1 + _smooth(fine, 2, 0.0, 0.01)
    unp1 = un + _smooth(fine, 3, 0.0, 0.01)
    rho, norm = 0.8, (-0.4, 0.3, 0.01, 0.002)
    f = pfch.Fno(4, 4, 1, *coarse)
    x = torch.empty((2,) + coarse, dtype=torch.float32, device="cuda")
    t = torch.empty(coarse, dtype=torch.float32, device="cuda")
    d = [torch.from_numpy(a).cuda() for a in (unm1, un, unp1)]
    f.prepare(d[0], d[1], d[2], rho, norm, x, t)
    mu, su, sd, so = norm
    ref = [ofno.band_resample((un - mu) / su, coarse), ofno.band_resample((un - unm1) / sd, coarse),
           ofno.band_resample((unp1 - (un + rho * (un - unm1))) / so, coarse)]
    got = [x[0].cpu().numpy(), x[1].cpu().numpy(), t.cpu().numpy()]
    fine_max = [np.max(np.abs((un - mu) / su)), np.max(np.abs((un - unm1) / sd)),
                np.max(np.abs((unp1 - (un + rho * (un - unm1))) / so))]
    for g, r, m in zip(got, ref, fine_max):
        assert np.max(np.abs(g - r)) <= 1e-5 * m, (np.max(np.abs(g - r)), m)
    f.close()


@pytest.mark.parametrize("w,coarse", [
    (dataclasses.replace(W.FCH256_BDF2, shape=(128, 128), lengths=(2 * np.pi, 2 * np.pi), seeds=(1,)), (32, 32)),
    (dataclasses.replace(W.PFC64_MP, shape=(128, 64), lengths=(128.0, 64.0), seeds=(3,)), (32, 16)),
], ids=["fch128-on32", "pfc128x64-on32x16"])
def test_coarse_network_learned_step_within_tolerance(w, coarse):
    """A network on a coarser grid than the instance's: the learned-guess step
    and the plain step both converge, differ within the PAGD tolerance and
    keep the same mass."""
    from paper_2204_07247_amd import pfch
    print(f"coarse network {coarse} on {w.model} {w.shape}", flush=True)
    un, unm1, dtp, k = _history(w, 3)
    fno = pfch.Fno(8, 4, 2, *coarse)
    fno.init_params(seed=5)
    u = un.cpu().numpy()
    du = (un - unm1).cpu().numpy()
    norm = (float(u.mean()), float(u.std()), float(du.std()), 0.1 * float(du.std()))
    rc_p, st_p, plain = _one_step(w, un, unm1, dtp, k)
    rc_l, st_l, learned = _one_step(w, un, unm1, dtp, k, fno=fno, norm=norm, guess=1)
    assert rc_p == pfch.PFCH_OK and rc_l == pfch.PFCH_OK
    assert st_l["guess"] == 1
    assert st_l["dnorm"] < w.tol and st_p["dnorm"] < w.tol
    assert np.max(np.abs(learned - plain)) <= 1e-9
    assert abs(learned.mean() - plain.mean()) <= 1e-14
    fno.close()


def test_coarse_network_must_fit_the_instance_grid():
    from paper_2204_07247_amd import pfch
    w = dataclasses.replace(W.PFC64_MP, shape=(64, 32), lengths=(64.0, 32.0))
    ctx = pfch.Context([desc_for(w, guess=1)])
    norm = (0.0, 1.0, 1.0, 1.0)
    too_big = pfch.Fno(4, 2, 1, 64, 64)   # finer than the instance on x
    ok = pfch.Fno(4, 2, 1, 16, 16)
    with pytest.raises(pfch.PfchError):
        ctx.set_fno(0, too_big, norm)
    ctx.set_fno(0, ok, norm)
    ctx.close()
    too_big.close()
    ok.close()


def test_batched_learned_guesses_match_solo():
    """Instances that share a network get their learned guesses from one
    batched forward pass: each equals its run alone (the network's products
    do not depend on the batch size), bit for bit, with the same iteration
    counts and guess kinds step by step."""
    import torch
    from paper_2204_07247_amd import pfch
    w = dataclasses.replace(W.FCH256_BDF2, shape=(64, 64), lengths=(np.pi, np.pi))
    print("batched learned guesses", flush=True)
    fno = pfch.Fno(8, 4, 2, 32, 32, max_batch=2)   # three instances: batches of 2 and 1
    fno.init_params(seed=11)
    seeds = (21, 22, 23)
    u0 = [torch.from_numpy(W.initial_condition(w, seed=s)).cuda() for s in seeds]

    def run(idx):
        ctx = pfch.Context([desc_for(w, guess=1) for _ in idx])
        for k, i in enumerate(idx):
            ctx.set_state(k, u0[i])
        assert ctx.step(w.dt)[0] == pfch.PFCH_OK
        for k, i in enumerate(idx):
            un, unm1 = torch.empty_like(u0[i]), torch.empty_like(u0[i])
            ctx.get_state(k, un, unm1)
            d = un - unm1
            ctx.set_fno(k, fno, (float(un.mean()), float(un.std()), float(d.std()), 0.1 * float(d.std())))
        its = []
        for step in range(3):
            rc, st = ctx.step(w.dt)
            assert rc == pfch.PFCH_OK
            if step < 2:  # (an untrained network may close the gate after its fitted gain)
                assert all(s["guess"] == 1 for s in st)
            its.append([(s["iters"], s["guess"]) for s in st])
        out = []
        for k in range(len(idx)):
            o = torch.empty_like(u0[0])
            ctx.get_state(k, o)
            out.append(o)
        ctx.close()
        return out, its

    batch, bits = run([0, 1, 2])
    for i in range(3):
        solo, sits = run([i])
        assert [x[i] for x in bits] == [x[0] for x in sits]
        assert torch.equal(batch[i], solo[0])
    fno.close()
