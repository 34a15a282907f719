"""The kernel-timing entry points the measurement uses (pfch_time_kernels,
pfch_time_group): per-launch averages of the iteration kernels and the time
per iteration of the chain of launches, from a solve that leaves the
instances' states alone."""
import dataclasses

import pytest

import workloads as W
from tests._common import desc_for

pytestmark = pytest.mark.gpu


def test_group_timing_and_state_untouched():
    import torch
    from paper_2204_07247_amd import pfch
    w = dataclasses.replace(W.FCH256_BDF2, shape=(128, 128))
    print("time_group fch 2 x 128^2", flush=True)
    ctx = pfch.Context([desc_for(w), desc_for(w)])
    us = [torch.from_numpy(W.initial_condition(w, seed=s)).cuda() for s in (1, 2)]
    for i, u in enumerate(us):
        ctx.set_state(i, u)
    for _ in range(2):
        assert ctx.step(w.dt)[0] == pfch.PFCH_OK
    before = [torch.empty_like(us[0]) for _ in range(4)]
    ctx.get_state(0, before[0], before[1])
    ctx.get_state(1, before[2], before[3])
    t = ctx.time_group(0, w.dt, 3)
    print(t, flush=True)
    assert set(t) == {"col_us", "row_us", "iteration_us"}
    assert t["col_us"] > 0 and t["row_us"] > 0
    # the chain without per-launch events: no slower than the launches with
    # them plus the gaps between launches, and not implausibly faster
    assert 0.5 * (t["col_us"] + t["row_us"]) < t["iteration_us"] < 2.0 * (t["col_us"] + t["row_us"])
    after = [torch.empty_like(us[0]) for _ in range(4)]
    ctx.get_state(0, after[0], after[1])
    ctx.get_state(1, after[2], after[3])
    assert all(torch.equal(a, b) for a, b in zip(before, after))
    # the next step after the timing equals the step of a context that was not timed
    rc, st = ctx.step(w.dt)
    assert rc == pfch.PFCH_OK
    ref = pfch.Context([desc_for(w), desc_for(w)])
    for i, u in enumerate(us):
        ref.set_state(i, u)
    for _ in range(3):
        assert ref.step(w.dt)[0] == pfch.PFCH_OK
    for i in range(2):
        a, b = torch.empty_like(us[0]), torch.empty_like(us[0])
        ctx.get_state(i, a)
        ref.get_state(i, b)
        assert torch.equal(a, b)
    tk = ctx.time_kernels(w.dt, 2)
    assert tk["iteration_us"] > 0 and tk["col_us"] > 0
    ctx.close()
    ref.close()
