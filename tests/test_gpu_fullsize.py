"""Parity at the bench sizes, in the launch configuration the bench uses
(autotuned plans, the same context set-up): the first step of PFC 1024^2
(implicit midpoint) and of FCH 1024^2 and 2048^2 (backward Euler) against
the oracle,
field by field; then properties that hold at any size over further steps
(convergence to the tolerance, exact mass; energy decrease for BDF2)."""
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


@pytest.mark.parametrize("name", ["pfc1024", "fch1024", "fch2048"])
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
