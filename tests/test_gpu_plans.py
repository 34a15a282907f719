"""Every radix schedule and launch geometry the autotuner may pick for the
iteration kernels gives the oracle's step: same iteration count, relative
L2 difference within the parity bar.

Elongated grids (16 x N and N x 16) put each transform length N = 64..2048
on the row (x) or column (y) kernel while keeping the oracle cheap."""
import dataclasses
import math

import numpy as np
import pytest

import workloads as W
from tests._common import desc_for, oracle_run, rel_l2

pytestmark = pytest.mark.gpu

LENGTHS = (64, 128, 192, 256, 512, 1024, 2048)
H_FCH = 4 * math.pi / 256  # FCH grid spacing of the 256^2 workload


def _workload(model, scheme, shape):
    ny, nx = shape
    if model == "pfc":
        return dataclasses.replace(W.PFC64_MP, scheme=scheme, shape=shape,
                                   lengths=(float(ny), float(nx)), seeds=(3,))
    return dataclasses.replace(W.FCH256_BDF2, scheme=scheme, shape=shape,
                               lengths=(ny * H_FCH, nx * H_FCH), seeds=(3,))


def _candidates(ctx, axis):
    """(row_alt, teams, col_alt, cb) choices that vary one kernel's plan and
    geometry while the other keeps its default."""
    p = ctx.plan(0)
    out = []
    if axis == "row":
        for alt in range(-1, p["n_row_alts"]):
            for teams in (1, 2, 4, 8, 16, 32, 64):
                out.append(dict(row_alt=alt, teams=teams, col_alt=-1, cb=p["col_cb"]))
    else:
        for alt in range(-1, p["n_col_alts"]):
            for cb in (1, 2, 4):
                out.append(dict(row_alt=-1, teams=p["row_teams"], col_alt=alt, cb=cb))
    return out


CASES = [(m, s, axis, n) for m in ("pfc", "fch") for s in ("mp", "bdf2")
         for axis in ("row", "col") for n in LENGTHS]


@pytest.mark.parametrize("case", CASES, ids=lambda c: "-".join(map(str, c)))
def test_every_plan_matches_oracle(case):
    import torch
    from paper_2204_07247_amd import pfch
    model, scheme, axis, n = case
    shape = (16, n) if axis == "row" else (n, 16)
    w = _workload(model, scheme, shape)
    u0 = W.initial_condition(w)
    ref, ref_iters = oracle_run(w, u0, 1)
    ctx = pfch.Context([desc_for(w)])
    ud = torch.from_numpy(u0).cuda()
    out = torch.empty_like(ud)
    tried = 0
    for ch in _candidates(ctx, axis):
        try:
            ctx.set_plan(0, **ch)
        except pfch.PfchError as e:
            assert e.code == pfch.PFCH_E_INVAL
            continue
        plan = ctx.plan(0)
        print(f"{model} {scheme} {shape} plan {ch} rows {plan['row_radices']} "
              f"cols {plan['col_radices']}", flush=True)
        ctx.set_state(0, ud)
        rc, st = ctx.step(w.dt)
        assert rc == pfch.PFCH_OK, (ch, rc)
        ctx.get_state(0, out)
        assert st[0]["iters"] == ref_iters[0], (ch, st[0]["iters"], ref_iters)
        assert rel_l2(out.cpu().numpy(), ref) <= 1e-9, ch
        tried += 1
    assert tried >= 2
    ctx.close()


@pytest.mark.parametrize("scheme", ["bdf2", "mp"])
@pytest.mark.parametrize("axis", ["x", "y", "z"])
def test_every_3d_plan_matches_oracle(axis, scheme):
    """3D: every x-, y- and z-pass plan and geometry for the length 192 on
    one axis (16 on the others) against the oracle."""
    import torch
    from paper_2204_07247_amd import pfch
    shape = {"x": (16, 16, 192), "y": (16, 192, 16), "z": (192, 16, 16)}[axis]
    w = dataclasses.replace(W.PFC64_MP, scheme=scheme, shape=shape,
                            lengths=tuple(float(n) for n in shape), seeds=(4,))
    u0 = W.initial_condition(w)
    ref, ref_iters = oracle_run(w, u0, 1)
    ctx = pfch.Context([desc_for(w)])
    p = ctx.plan(0)
    base = [p["row_alt"], p["row_teams"], -1, 1, p["y_alt"], p["y_cb"], p["z_alt"], p["z_kyb"]]
    choices = []
    if axis == "x":
        for alt in range(-1, p["n_row_alts"]):
            for teams in (1, 2, 4, 8, 16):
                choices.append([alt, teams] + base[2:])
    elif axis == "y":
        for alt in range(-1, p["n_y_alts"]):
            for cy in (1, 2, 4):
                choices.append(base[:4] + [alt, cy] + base[6:])
    else:
        for alt in range(-1, p["n_z_alts"]):
            for kyb in (1, 2, 4, 8):
                choices.append(base[:6] + [alt, kyb])
    ud = torch.from_numpy(u0).cuda()
    out = torch.empty_like(ud)
    tried = 0
    for ch in choices:
        try:
            ctx.set_plan(0, *ch)
        except pfch.PfchError as e:
            assert e.code == pfch.PFCH_E_INVAL
            continue
        print(f"3d {shape} {scheme} plan {ch} {ctx.plan(0)}", flush=True)
        ctx.set_state(0, ud)
        rc, st = ctx.step(w.dt)
        assert rc == pfch.PFCH_OK, (ch, rc)
        ctx.get_state(0, out)
        assert st[0]["iters"] == ref_iters[0], (ch, st[0]["iters"], ref_iters)
        assert rel_l2(out.cpu().numpy(), ref) <= 1e-9, ch
        tried += 1
    assert tried >= 2
    ctx.close()
