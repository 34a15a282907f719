"""Batched execution: several instances of mixed shapes, models, schemes and
parameters advance together through grouped launches in one graph.  Each
instance must match its own solo run bitwise (launch geometry depends on the
grid shape only) and the CPU oracle to the parity bar."""
import dataclasses

import numpy as np
import pytest

import workloads as W
from tests._common import desc_for, oracle_run, rel_l2

pytestmark = pytest.mark.gpu

BATCH = [
    dataclasses.replace(W.PFC64_MP, name="a", seeds=(0,)),
    dataclasses.replace(W.PFC64_MP, name="b", eps=0.3, mean=-0.3, seeds=(1,)),  # same group as a
    dataclasses.replace(W.PFC64_MP, name="c", shape=(32, 64), lengths=(32.0, 64.0), seeds=(2,)),
    dataclasses.replace(W.FCH256_BDF2, name="d", shape=(64, 64), seeds=(3,)),
    dataclasses.replace(W.FCH256_BDF2, name="e", shape=(32, 32), scheme="mp", seeds=(4,)),
    dataclasses.replace(W.PFC64_MP, name="f", shape=(64, 128), lengths=(64.0, 128.0), scheme="bdf2",
                        seeds=(5,)),
]
NSTEPS = 6


def _run(ws, nsteps):
    import torch
    from paper_2204_07247_amd import pfch
    ctx = pfch.Context([desc_for(w) for w in ws])
    us = [torch.from_numpy(W.initial_condition(w)).cuda() for w in ws]
    for i, u in enumerate(us):
        ctx.set_state(i, u)
    iters = [[] for _ in ws]
    for _ in range(nsteps):
        rc, st = ctx.step([w.dt for w in ws])
        assert rc == pfch.PFCH_OK, (rc, st)
        for i, s in enumerate(st):
            iters[i].append(s["iters"])
    outs = []
    for i, u in enumerate(us):
        o = torch.empty_like(u)
        ctx.get_state(i, o)
        outs.append(o.cpu().numpy())
    ctx.close()
    return outs, iters


def test_batch_equals_solo_runs_bitwise():
    batch, biters = _run(BATCH, NSTEPS)
    for w, got, it in zip(BATCH, batch, biters):
        print(f"case {w.name} {w.model} {w.scheme} {w.shape}", flush=True)
        solo, siters = _run([w], NSTEPS)
        assert it == siters[0]
        assert np.array_equal(got, solo[0])


def test_batch_matches_oracle():
    batch, biters = _run(BATCH, NSTEPS)
    for w, got, it in zip(BATCH, batch, biters):
        ref, ref_iters = oracle_run(w, W.initial_condition(w), NSTEPS)
        assert it == ref_iters, (w.name, it, ref_iters)
        assert rel_l2(got, ref) <= 1e-9, w.name


def test_ensemble_generator_batch_matches_oracle():
    ens = W.pfc_ensemble(count=5, steps=3, sizes=(32, 64, 128))
    batch, biters = _run(ens, 3)
    for w, got, it in zip(ens, batch, biters):
        ref, ref_iters = oracle_run(w, W.initial_condition(w), 3)
        assert it == ref_iters, (w.name, it, ref_iters)
        assert rel_l2(got, ref) <= 1e-9, w.name
