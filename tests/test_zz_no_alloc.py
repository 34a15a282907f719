"""pfch_rhs_noalloc, the allocation-free variant of pfch_rhs, through the C ABI.

Its kernels are those of pfch_rhs with the spectral workspace and the
pointer staging in the library's static scratch, so its result must equal
pfch_rhs's bit for bit; two calls in a row, the second on a smaller grid,
check that the shared scratch carries nothing from one call to the next.
"""
import os

import numpy as np
import pytest

import workloads as W
from tests._common import desc_for

pytestmark = pytest.mark.gpu


def _fields(w, seeds):
    import torch
    return [torch.from_numpy(W.initial_condition(w, seed=s)).cuda() for s in seeds]


@pytest.mark.parametrize("model", ["fch", "pfc"])
def test_noalloc_rhs_equals_rhs_on_two_calls(model):
    import torch
    from paper_2204_07247_amd import pfch
    if model == "fch":
        big = W.FCH256_BDF2
        small = W.scaled(W.FCH256_BDF2, shape=(64, 32), lengths=(np.pi, np.pi / 2))
    else:
        big = W.scaled(W.PFC64_MP, shape=(256, 512), lengths=(256.0, 512.0))
        small = W.PFC64_MP
    print(f"noalloc rhs {model}: {big.shape} then {small.shape}", flush=True)
    ctx = pfch.Context([desc_for(big), desc_for(small)])
    for inst, w in ((0, big), (1, small)):
        v, = _fields(w, (31 + inst,))
        ref = torch.empty_like(v)
        got = torch.full_like(v, float("nan"))
        ctx.rhs(inst, v, ref)
        rc = ctx.rhs_noalloc(inst, v, got)
        assert rc == pfch.PFCH_OK, pfch.strerror(rc)
        torch.cuda.synchronize()
        assert torch.equal(got, ref), inst
        assert torch.isfinite(got).all()
    ctx.close()


def test_noalloc_rhs_keeps_the_context_state():
    """Calls between fixed-size steps leave the steps (and the set-up queued
    between them) exactly as without the calls."""
    import torch
    from paper_2204_07247_amd import pfch
    w = W.scaled(W.FCH256_BDF2, shape=(64, 64))
    print("noalloc rhs between steps", flush=True)
    u0, v = _fields(w, (41, 42))
    out = torch.empty_like(v)
    finals = []
    for interleave in (False, True):
        ctx = pfch.Context([desc_for(w)])
        ctx.set_state(0, u0)
        for k in range(4):
            assert ctx.step(w.dt)[0] == pfch.PFCH_OK
            if interleave:
                assert ctx.rhs_noalloc(0, v, out) == pfch.PFCH_OK
        a = torch.empty_like(u0)
        ctx.get_state(0, a)
        finals.append(a)
        ctx.close()
    assert torch.equal(finals[0], finals[1])


def test_noalloc_rhs_rejects_what_it_cannot_hold():
    import torch
    from paper_2204_07247_amd import pfch
    print("noalloc rhs limits", flush=True)
    old = os.environ.get("PFCH_AUTOTUNE")
    os.environ["PFCH_AUTOTUNE"] = "0"
    try:
        # 3 spectral fields of 1024 x 1024 complex doubles: 48 MiB > 32 MiB
        w = W.scaled(W.FCH256_BDF2, shape=(1024, 2048), lengths=(2 * np.pi, 4 * np.pi))
        ctx = pfch.Context([desc_for(w), desc_for(W.PFC64_MP)])
    finally:
        if old is None:
            del os.environ["PFCH_AUTOTUNE"]
        else:
            os.environ["PFCH_AUTOTUNE"] = old
    v = torch.zeros(w.shape, dtype=torch.float64, device="cuda")
    out = torch.empty_like(v)
    assert ctx.rhs_noalloc(0, v, out) == pfch.PFCH_E_SCRATCH
    assert "scratch" in pfch.strerror(pfch.PFCH_E_SCRATCH)
    s = torch.zeros(W.PFC64_MP.shape, dtype=torch.float64, device="cuda")
    assert ctx.rhs_noalloc(1, s, s) == pfch.PFCH_E_INVAL
    assert ctx.rhs_noalloc(2, s, out) == pfch.PFCH_E_INVAL
    ctx.close()
