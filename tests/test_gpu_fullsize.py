"""Parity at the bench sizes, in the launch configuration the bench uses
(autotuned plans, the same context set-up): the first step of PFC 1024^2
(implicit midpoint) and of FCH 1024^2 (backward Euler), and the first two
steps of FCH 2048^2, PFC 1024^2 and PFC 192^3, against the oracle,
field by field; then properties that hold at any size over further steps
(convergence to the tolerance, exact mass; energy decrease for BDF2);
and the combined set batched against solo runs, with and without the
learned guess."""
import numpy as np
import pytest

import bench
import workloads as W
from oracle import models as omodels
from oracle import spectral as ospectral
from tests._common import oracle_run, rel_l2

pytestmark = pytest.mark.gpu


def _ctx(w):
    import torch
    from paper_2204_07247_amd import pfch
    ctx = pfch.Context([bench._desc(w)])
    u0 = W.initial_condition(w)
    ctx.set_state(0, torch.from_numpy(u0).cuda())
    return ctx, u0


@pytest.mark.parametrize("name", ["pfc1024", "fch1024"])
def test_first_step_matches_oracle_at_full_size(name):
    import torch
    from paper_2204_07247_amd import pfch
    w = bench.WORKLOADS[name]
    print(f"full size {w.name}", flush=True)
    ctx, u0 = _ctx(w)
    rc, st = ctx.step(w.dt)
    assert rc == pfch.PFCH_OK
    out = torch.empty(w.shape, dtype=torch.float64, device="cuda")
    ctx.get_state(0, out)
    ctx.close()
    ref, ref_iters = oracle_run(w, u0, 1)
    assert st[0]["iters"] == ref_iters[0]
    assert rel_l2(out.cpu().numpy(), ref) <= 1e-9


@pytest.mark.parametrize("name", ["fch2048", "pfc1024"])
def test_two_steps_match_oracle_at_full_size(name):
    """FCH 2048^2: the backward Euler first step (set-up from transforms of
    x0) and the BDF2 second step (set-up from the kept Laplacians); PFC
    1024^2: two implicit midpoint steps, the second from the extrapolated
    guess; against the oracle: iteration counts equal, relative L2 within
    the parity bar."""
    import torch
    from paper_2204_07247_amd import pfch
    w = bench.WORKLOADS[name]
    print(f"full size {w.name}, 2 steps", flush=True)
    ctx, u0 = _ctx(w)
    iters = []
    for _ in range(2):
        rc, st = ctx.step(w.dt)
        assert rc == pfch.PFCH_OK
        iters.append(st[0]["iters"])
    out = torch.empty(w.shape, dtype=torch.float64, device="cuda")
    ctx.get_state(0, out)
    ctx.close()
    ref, ref_iters = oracle_run(w, u0, 2)
    assert iters == ref_iters
    assert rel_l2(out.cpu().numpy(), ref) <= 1e-9


@pytest.mark.parametrize("name", ["pfc1024", "fch1024", "fch2048"])
def test_properties_over_steps_at_full_size(name):
    import torch
    from paper_2204_07247_amd import pfch
    w = bench.WORKLOADS[name]
    ctx, u0 = _ctx(w)
    g = ospectral.Grid(w.shape, w.lengths)
    m = omodels.make_model(w.model, **w.params())
    e_prev = m.energy(g, u0)
    out = torch.empty(w.shape, dtype=torch.float64, device="cuda")
    for _ in range(5):
        rc, st = ctx.step(w.dt)
        assert rc == pfch.PFCH_OK
        assert st[0]["dnorm"] < w.tol
        assert abs(st[0]["mass"] - u0.mean()) <= 1e-14
        ctx.get_state(0, out)
        u = out.cpu().numpy()
        e = m.energy(g, u)
        if w.scheme == "bdf2":  # energy decay is pinned for the BDF2 family only
            assert e <= e_prev + 1e-12 * abs(e_prev)
        e_prev = e
    ctx.close()


# --- the batched and 3D configurations at their real sizes -----------------

def _tuned():
    """The plan choices bench.py runs with (recorded autotuner output)."""
    import os
    os.environ.setdefault("PFCH_TUNE_FILE", os.path.join(
        os.path.dirname(bench.__file__), "paper_2204_07247_amd", "tune_mi355x.txt"))


def _run_set(ws, nsteps):
    """All of ws in one context, nsteps steps: final states and iteration counts."""
    import torch
    from paper_2204_07247_amd import pfch
    ctx = pfch.Context([bench._desc(w) for w in ws])
    ctx.set_stats_detail(0)
    us = [torch.from_numpy(W.initial_condition(w)).cuda() for w in ws]
    for i, u in enumerate(us):
        ctx.set_state(i, u)
    iters = [[] for _ in ws]
    for _ in range(nsteps):
        rc, st = ctx.step([w.dt for w in ws])
        assert rc == pfch.PFCH_OK, pfch.strerror(rc)
        for i, s in enumerate(st):
            iters[i].append(s["iters"])
    outs = []
    for i, u in enumerate(us):
        ctx.get_state(i, u)
        outs.append(u)
    ctx.close()
    return outs, iters


def test_3d_first_steps_match_oracle_at_full_size():
    """PFC 192^3 (the 3D instance of the combined set): the first two steps
    (backward Euler, then BDF2) field by field against the oracle."""
    _tuned()
    w = W.PFC192_3D
    print(f"full size {w.name}, 2 steps", flush=True)
    (got,), (iters,) = _run_set([w], 2)
    ref, ref_iters = oracle_run(w, W.initial_condition(w), 2)
    assert iters == ref_iters
    assert rel_l2(got.cpu().numpy(), ref) <= 1e-9


def test_combined_set_batched_equals_solo_and_oracle():
    """The combined set (8 FCH 1024^2 + 8 FCH 2048^2 with drawn eps and mean,
    PFC 192^3) in one context for two steps (backward Euler, then BDF2):
    every instance bitwise equal to its own solo run; the first FCH 1024^2
    instance against the oracle."""
    import torch
    _tuned()
    ws = W.fch_ensemble() + [W.PFC192_3D]
    print(f"combined set: {len(ws)} instances, 2 steps", flush=True)
    batch, biters = _run_set(ws, 2)
    for w, got, it in zip(ws, batch, biters):
        print(f"solo {w.name}", flush=True)
        (solo,), (siters,) = _run_set([w], 2)
        assert it == siters, w.name
        assert torch.equal(got, solo), w.name
    w0 = ws[0]
    ref, ref_iters = oracle_run(w0, W.initial_condition(w0), 2)
    assert biters[0] == ref_iters
    assert rel_l2(batch[0].cpu().numpy(), ref) <= 1e-9


def test_pfc_ensemble_at_real_sizes():
    """The 64-instance PFC ensemble (Nx, Ny in {128, 256, 512}, drawn eps and
    mean, MP) in one context for two steps: every instance bitwise equal to
    its solo run; a sample (the 512 x 512 instances' first, the rectangles
    512 x 128 and 128 x 512, a 256 x 256 one) against the oracle."""
    import torch
    _tuned()
    ens = W.pfc_ensemble(count=64, steps=2)
    print(f"pfc ensemble: {len(ens)} instances, 2 steps", flush=True)
    batch, biters = _run_set(ens, 2)
    for w, got, it in zip(ens, batch, biters):
        (solo,), (siters,) = _run_set([w], 2)
        assert it == siters, w.name
        assert torch.equal(got, solo), w.name
    picks = []
    for shape in ((512, 512), (512, 128), (128, 512), (256, 256)):
        idx = [i for i, w in enumerate(ens) if tuple(w.shape) == shape]
        if idx:
            picks.append(idx[0])
    assert len(picks) >= 3
    for i in picks:
        w = ens[i]
        print(f"oracle {w.name}", flush=True)
        ref, ref_iters = oracle_run(w, W.initial_condition(w), 2)
        assert biters[i] == ref_iters, w.name
        assert rel_l2(batch[i].cpu().numpy(), ref) <= 1e-9, w.name


def _run_set_learned(ws, fno, nsteps):
    """All of ws in one context with the learned guess: the first step
    (backward Euler, no history) with the extrapolated guess, then the
    network attached to every instance (normalisation from its own state)
    for nsteps - 1 more steps.  Final states, iteration counts and guess
    kinds."""
    import torch
    from paper_2204_07247_amd import learned, pfch
    ctx = pfch.Context([learned.desc_of(w, 1) for w in ws])
    ctx.set_stats_detail(0)
    us = [torch.from_numpy(W.initial_condition(w)).cuda() for w in ws]
    for i, u in enumerate(us):
        ctx.set_state(i, u)
    iters = [[] for _ in ws]
    kinds = [[] for _ in ws]
    for n in range(nsteps):
        if n == 1:
            for i, u in enumerate(us):
                un, unm1 = torch.empty_like(u), torch.empty_like(u)
                ctx.get_state(i, un, unm1)
                d = un - unm1
                ctx.set_fno(i, fno, (float(un.mean()), float(un.std()), float(d.std()), 0.1 * float(d.std())))
        rc, st = ctx.step([w.dt for w in ws])
        assert rc == pfch.PFCH_OK, pfch.strerror(rc)
        for i, s in enumerate(st):
            iters[i].append(s["iters"])
            kinds[i].append(s["guess"])
    outs = []
    for i, u in enumerate(us):
        ctx.get_state(i, u)
        outs.append(u)
    ctx.close()
    return outs, iters, kinds


def test_combined_set_learned_batched_equals_solo():
    """The 16 FCH instances of the combined set (1024^2 and 2048^2) with a
    network on a 64^2 grid (band-limited resampling in and out, one batched
    forward pass for all 16) in one context for three steps: every instance
    bitwise equal to its own solo run, with the same iteration counts and
    guess kinds (the extrapolated first step, then two learned steps)."""
    import torch
    from paper_2204_07247_amd import pfch
    _tuned()
    ws = W.fch_ensemble()
    fno = pfch.Fno(8, 4, 2, 64, 64, max_batch=len(ws))
    fno.init_params(seed=13)
    print(f"combined FCH set, learned: {len(ws)} instances, 3 steps", flush=True)
    batch, biters, bkinds = _run_set_learned(ws, fno, 3)
    for w, got, it, kd in zip(ws, batch, biters, bkinds):
        assert kd == [0, 1, 1], (w.name, kd)
        print(f"solo {w.name}", flush=True)
        (solo,), (siters,), (skinds,) = _run_set_learned([w], fno, 3)
        assert (it, kd) == (siters, skinds), w.name
        assert torch.equal(got, solo), w.name
    fno.close()
