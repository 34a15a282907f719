"""Plan choices read from and written to the tuning file (PFCH_TUNE_FILE):
a valid recorded choice is used as is, an invalid one is ignored (the group
is timed and the new choice appended), and either way the step matches the
oracle.  Runs in a child process: the process-wide choice cache of the
parent may already hold these grids."""
import json
import os
import subprocess
import sys

import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

CHILD = r'''
import dataclasses, json, sys
import torch
import workloads as W
from paper_2204_07247_amd import pfch
from tests._common import desc_for, oracle_run, rel_l2

def run(shape):
    w = dataclasses.replace(W.PFC64_MP, shape=shape, lengths=tuple(float(n) for n in shape), seeds=(6,))
    u0 = W.initial_condition(w)
    ref, ref_iters = oracle_run(w, u0, 1)
    ctx = pfch.Context([desc_for(w)])
    p = ctx.plan(0)
    ctx.set_state(0, torch.from_numpy(u0).cuda())
    rc, st = ctx.step(w.dt)
    out = torch.empty(w.shape, dtype=torch.float64, device="cuda")
    ctx.get_state(0, out)
    ctx.close()
    return dict(plan=[p["row_alt"], p["row_teams"], p["col_alt"], p["col_cb"]], rc=rc,
                iters=st[0]["iters"], ref_iters=ref_iters[0], err=rel_l2(out.cpu().numpy(), ref))

print(json.dumps([run((64, 128)), run((128, 64))]), flush=True)
'''


def test_tune_file_choice_is_used_and_new_choices_appended(tmp_path):
    from paper_2204_07247_amd import pfch
    path = tmp_path / "tune.txt"
    # model scheme nx ny nz  row_alt teams col_alt cb 0 cy kyb y3_alt z3_alt
    path.write_text(f"# comment lines are skipped\n"
                    f"{pfch.PFC} {pfch.MP} 128 64 1  -1 4 0 2 0 0 0 -1 -1\n"
                    f"{pfch.PFC} {pfch.MP} 64 128 1  -1 3 -1 1 0 0 0 -1 -1\n")  # 3 row pairs per block: invalid
    env = dict(os.environ, PFCH_TUNE_FILE=str(path), PYTHONPATH=ROOT)
    print("tune file child process", flush=True)
    r = subprocess.run([sys.executable, "-c", CHILD], cwd=ROOT, env=env, capture_output=True, text=True,
                       timeout=240)
    assert r.returncode == 0, r.stderr[-3000:]
    a, b = json.loads(r.stdout.strip().splitlines()[-1])
    for res in (a, b):
        assert res["rc"] == pfch.PFCH_OK
        assert res["iters"] == res["ref_iters"]
        assert res["err"] <= 1e-9
    assert a["plan"] == [-1, 4, 0, 2]          # the recorded choice
    assert b["plan"][1] != 3                   # the invalid one was not used
    lines = path.read_text().splitlines()
    assert len(lines) == 4                     # the timed choice was appended
    last = [int(v) for v in lines[-1].split()]
    assert last[:5] == [pfch.PFC, pfch.MP, 64, 128, 1]
    assert last[5:9] == b["plan"]
