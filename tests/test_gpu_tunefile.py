"""Plan choices read from and written to the tuning file (PFCH_TUNE_FILE):
a valid recorded choice is used as is, an invalid one is ignored (the group
is timed and the new choice appended), and either way the step matches the
oracle."""
import dataclasses

import pytest

import workloads as W
from tests._common import desc_for, oracle_run, rel_l2

pytestmark = pytest.mark.gpu


def _w(shape):
    return dataclasses.replace(W.PFC64_MP, shape=shape, lengths=tuple(float(n) for n in shape), seeds=(6,))


def _step_matches(ctx, w):
    import torch
    from paper_2204_07247_amd import pfch
    u0 = W.initial_condition(w)
    ref, ref_iters = oracle_run(w, u0, 1)
    ctx.set_state(0, torch.from_numpy(u0).cuda())
    rc, st = ctx.step(w.dt)
    assert rc == pfch.PFCH_OK
    out = torch.empty(w.shape, dtype=torch.float64, device="cuda")
    ctx.get_state(0, out)
    assert st[0]["iters"] == ref_iters[0]
    assert rel_l2(out.cpu().numpy(), ref) <= 1e-9


def test_tune_file_choice_is_used_and_new_choices_appended(tmp_path, monkeypatch):
    from paper_2204_07247_amd import pfch
    path = tmp_path / "tune.txt"
    wa, wb = _w((64, 128)), _w((128, 64))
    # model scheme nx ny nz  row_alt teams col_alt cb persist cy kyb y3_alt z3_alt
    path.write_text(f"# comment lines are skipped\n"
                    f"{pfch.PFC} {pfch.MP} 128 64 1  -1 4 0 2 0 0 0 -1 -1\n"
                    f"{pfch.PFC} {pfch.MP} 64 128 1  -1 3 -1 1 0 0 0 -1 -1\n")  # 3 row pairs per block: invalid
    monkeypatch.setenv("PFCH_TUNE_FILE", str(path))
    print("tune file (64, 128)", flush=True)
    ctx = pfch.Context([desc_for(wa)])
    p = ctx.plan(0)
    assert (p["row_alt"], p["row_teams"], p["col_alt"], p["col_cb"]) == (-1, 4, 0, 2)
    _step_matches(ctx, wa)
    ctx.close()
    print("tune file (128, 64)", flush=True)
    ctx = pfch.Context([desc_for(wb)])
    p = ctx.plan(0)
    assert p["row_teams"] != 3
    _step_matches(ctx, wb)
    ctx.close()
    lines = path.read_text().splitlines()
    assert len(lines) == 4
    last = [int(v) for v in lines[-1].split()]
    assert last[:5] == [pfch.PFC, pfch.MP, 64, 128, 1]
    assert (last[5], last[6], last[7], last[8]) == (p["row_alt"], p["row_teams"], p["col_alt"], p["col_cb"])
