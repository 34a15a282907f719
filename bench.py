"""Throughput of the PAGD-solved fully implicit steps on one MI355X.

Default workload: FCH 2D 256 x 256 on [0, 4 pi)^2, eps = 0.1, eta1 = 0.145,
eta2 = 0.2, tau = 0, u0 = -0.6 + 0.01 U(-1, 1) (seed 0), BDF2 (backward Euler
first step), dt = 1e-3, PAGD to ||d||_inf < 1e-10; one bench step = one time
step.  The timed region runs `--steps` consecutive time steps from u0 with all
data resident on the GPU, bracketed by torch.cuda.synchronize().

Prints one JSON line (metric, value in time-steps/s, iterations per step,
roofline of the dominant kernel from HIP-event timings, CPU-oracle baseline).
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import workloads as W  # noqa: E402

METRIC = "time-steps/sec & PAGD iters/step at 1e-10 residual: plain vs batched+learned"
HBM_PEAK_GBS = 8000.0

WORKLOADS = {
    "fch256": W.FCH256_BDF2,
    "pfc64": W.PFC64_MP,
    "pfc1024": W.Workload(
        name="pfc2d_1024_mp", model="pfc", scheme="mp", shape=(1024, 1024),
        lengths=(1024.0, 1024.0), dt=0.2, steps=500, mean=-0.25, amp=0.05, eps=0.25),
    "fch2048": W.scaled(W.FCH256_BDF2, name="fch2d_2048_bdf2", shape=(2048, 2048), steps=300),
    "fch1024": W.scaled(W.FCH256_BDF2, name="fch2d_1024_bdf2", shape=(1024, 1024), steps=300),
    "pfc192_3d": W.PFC192_3D,
}


def log(msg):
    print(msg, file=sys.stderr, flush=True)


KERNEL_NAMES = {"row": "k_row_iter", "col": "k_col_iter", "yfwd": "k_y3_iter<fwd>",
                "z": "k_z3_iter", "yinv": "k_y3_iter<inv>"}


def algorithmic_bytes(w):
    """Compulsory HBM bytes per launch of each iteration kernel.

    Real field: Ny*Nx (*Nz) doubles.  Spectral field: half as many complex
    doubles (the half spectrum's two real columns kx = 0 and kx = Nx/2 share
    one).  PFC row kernel: read 1 spectral + x_j, x_{j-1} (+ u^n for MP),
    write x_{j+1} + 2 spectral.  PFC column kernel: read 2 spectral + g^,
    write 1.  FCH row kernel: read 2 spectral + x_j, x_{j-1}, Lx_j, Lx_{j-1}
    (+ u^n, Lu^n for MP), write x_{j+1}, Lx_{j+1} + 3 spectral.  FCH column
    kernel: read 3 spectral + g^, write 2 spectral.  3D PFC: the row kernel
    as in 2D; y forward: read and write 2 spectral; z: read 2 spectral + g^,
    write 1; y inverse: read and write 1 spectral.
    """
    npts = int(np.prod(w.shape))
    real = 8 * npts
    spec = 16 * (npts // 2)
    mp = w.scheme == "mp"
    if w.model == "pfc":
        row = spec + 2 * real + (real if mp else 0) + real + 2 * spec
        if len(w.shape) == 3:
            return dict(yfwd=4 * spec, z=4 * spec, yinv=2 * spec, row=row)
        col = 2 * spec + spec + spec
    else:
        row = 2 * spec + 4 * real + (2 * real if mp else 0) + 2 * real + 3 * spec
        col = 3 * spec + spec + 2 * spec
    return dict(row=row, col=col)


def measured_traffic(w, kernel):
    """HBM bytes per launch from the committed PMC summary, if it was taken on
    the current kernel sources; otherwise None."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        rec = json.load(fh)
    ent = rec.get(w.name, {}).get(KERNEL_NAMES[kernel])
    if not ent or ent.get("source_sha256") != kernel_source_hash():
        return None
    return ent["traffic_bytes"]


def kernel_source_hash():
    """Hash of the sources that define the iteration kernels (transform
    passes, fused k-space and real-space bodies, plan table) and their
    compile flags: counter totals are reused only while this is unchanged."""
    import hashlib
    h = hashlib.sha256()
    pkg = os.path.join(ROOT, "paper_2204_07247_amd")
    for rel in ("csrc/fft.hpp", "csrc/kernels2d.hpp", "csrc/kernels3d.hpp", "csrc/pfch_dev.hpp",
                "csrc/plans.hpp", "build.py"):
        with open(os.path.join(pkg, rel), "rb") as fh:
            h.update(rel.encode() + b"\0" + fh.read())
    return h.hexdigest()


def gpu_run(w, steps, warmup, kernel_timing):
    import torch
    from paper_2204_07247_amd import pfch

    d = pfch.make_desc(w.model, w.scheme, w.shape, w.lengths, eps=w.eps, eta1=w.eta1,
                       eta2=w.eta2, tau=w.tau, mobility=w.mobility, s=w.s, etas=w.etas,
                       tol=w.tol, max_iter=w.max_iter)
    ctx = pfch.Context([d])
    ctx.set_stats_detail(0)
    u0 = torch.from_numpy(W.initial_condition(w)).cuda()

    def run(n):
        ctx.set_state(0, u0)
        iters = []
        for _ in range(n):
            rc, st = ctx.step(w.dt)
            if rc != pfch.PFCH_OK:
                raise RuntimeError(f"step failed: {pfch.strerror(rc)}")
            iters.append(st[0]["iters"])
        return iters

    log(f"[bench] warmup {warmup} steps")
    run(warmup)
    torch.cuda.synchronize()
    log(f"[bench] timed region: {steps} steps")
    t0 = time.perf_counter()
    iters = run(steps)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    log(f"[bench] timed region done: {elapsed:.4f} s")
    timing = None
    if kernel_timing:
        solves, reps = 20, 50
        log(f"[bench] kernel timing: HIP start/stop events on every iteration-kernel launch of "
            f"{solves} solves; HIP events around {reps} back-to-back launches per kernel")
        timing = ctx.time_kernels(w.dt, solves)
        timing["solves"] = solves
        timing["back_to_back"] = ctx.time_kernels(w.dt, reps, events=True)
        timing["back_to_back_reps"] = reps
    cfg = ctx.launch_config()
    cfg["plan"] = ctx.plan(0)
    ctx.close()
    return elapsed, iters, timing, cfg


def _desc(w):
    from paper_2204_07247_amd import pfch
    return pfch.make_desc(w.model, w.scheme, w.shape, w.lengths, eps=w.eps, eta1=w.eta1,
                          eta2=w.eta2, tau=w.tau, mobility=w.mobility, s=w.s, etas=w.etas,
                          tol=w.tol, max_iter=w.max_iter)


def batched_comparison(count, steps, solo_steps):
    """The PFC ensemble (Nx, Ny from {128, 256, 512}, eps, mean drawn per
    instance) advanced in one context (grouped launches, one iteration graph)
    against the same instances advanced one context at a time."""
    import torch
    from paper_2204_07247_amd import pfch
    ens = W.pfc_ensemble(count=count)
    u0 = [torch.from_numpy(W.initial_condition(w)).cuda() for w in ens]
    ctx = pfch.Context([_desc(w) for w in ens])
    ctx.set_stats_detail(0)

    def run(n):
        for i, u in enumerate(u0):
            ctx.set_state(i, u)
        its = []
        for _ in range(n):
            rc, st = ctx.step([w.dt for w in ens])
            if rc != pfch.PFCH_OK:
                raise RuntimeError(f"batched step failed: {pfch.strerror(rc)}")
            its.append(np.mean([x["iters"] for x in st]))
        return its

    log(f"[bench] batched ensemble: {count} instances, {steps} steps")
    run(2)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    its = run(steps)
    torch.cuda.synchronize()
    tb = time.perf_counter() - t0
    ctx.close()
    log(f"[bench] the same instances one context at a time, {solo_steps} steps each")
    ts = 0.0
    for w, u in zip(ens, u0):
        c = pfch.Context([_desc(w)])
        c.set_stats_detail(0)
        c.set_state(0, u)
        c.step(w.dt)
        c.set_state(0, u)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(solo_steps):
            rc, _ = c.step(w.dt)
            if rc != pfch.PFCH_OK:
                raise RuntimeError(f"solo step failed: {pfch.strerror(rc)}")
        torch.cuda.synchronize()
        ts += time.perf_counter() - t0
        c.close()
    npts = int(sum(w.npoints for w in ens))
    batched = count * steps / tb
    plain = count * solo_steps / ts
    return dict(workload=f"pfc2d_ensemble{count}", instances=count, points=npts,
                batched_instance_steps_per_s=round(batched, 2),
                plain_instance_steps_per_s=round(plain, 2),
                batched_over_plain=round(batched / plain, 3),
                batched_steps=steps, plain_steps_per_instance=solo_steps,
                iters_per_step_mean=round(float(np.mean(its)), 3))


def solver_variants(w, steps):
    """The same steps of w solved by PAGD with the paper's friction sweep,
    PAGD with each constant friction of the sweep, plain preconditioned
    gradient descent (Alg. 1), and the linear IMEX scheme of the same
    family (one linear solve per step): iterations and FFT pairs per step,
    time-steps/s."""
    import dataclasses

    import torch
    from paper_2204_07247_amd import pfch
    u0 = torch.from_numpy(W.initial_condition(w)).cuda()
    fft_pairs = {"pfc": 1.5, "fch": 2.5}[w.model]
    variants = [("pagd_sweep", {}), ("pgd", dict(etas=()))]
    variants += [(f"pagd_eta{e * e:g}", dict(etas=(e,))) for e in w.etas]
    imex = "lbdf2" if w.scheme == "bdf2" else "lmp"
    variants.append((imex, dict(scheme=imex)))
    out = {}
    for name, kw in variants:
        wv = dataclasses.replace(w, **{k: v for k, v in kw.items() if k in ("etas", "scheme")})
        ctx = pfch.Context([_desc(wv)])
        ctx.set_stats_detail(0)
        ctx.set_state(0, u0)
        its = []
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            rc, st = ctx.step(w.dt)
            if rc != pfch.PFCH_OK:
                its = None
                break
            its.append(st[0]["iters"])
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        ctx.close()
        if its is None:
            out[name] = dict(status=pfch.strerror(rc))
            continue
        out[name] = dict(iters_per_step=round(float(np.mean(its)), 3),
                         fft_pairs_per_step=round(float(np.mean(its)) * fft_pairs, 2),
                         steps_per_s=round(steps / el, 1))
    return dict(workload=w.name, steps=steps, variants=out)


def adaptive_run(w, tol, dt_min, dt_max, attempts):
    """Adaptive stepping (Alg. 3) of w from its initial condition:
    ``attempts`` passes of the loop body (tentative PAGD solve, R(u~), AM3 or
    midAB2 estimate, accept / reject, next size) with the paper's stepping
    tolerance and size bounds; counts, reached time and rates."""
    import torch
    from paper_2204_07247_amd import pfch
    ctx = pfch.Context([_desc(w)])
    ctx.set_stats_detail(0)
    ctx.set_state(0, torch.from_numpy(W.initial_condition(w)).cuda())
    dt = dt_min
    acc = rej = 0
    its, dts, ests = [], [], set()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(attempts):
        rc, res = ctx.step_adaptive(dt, tol, dt_min, dt_max)
        if rc != pfch.PFCH_OK:
            break
        r = res[0]
        its.append(r["solve"]["iters"])
        ests.add(r["estimator"])
        if r["accepted"]:
            acc += 1
            dts.append(r["dt"])
        else:
            rej += 1
        dt = r["dt_next"]
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    t, _, _ = ctx.get_state(0)
    ctx.close()
    return dict(workload=w.name, scheme=w.scheme, estimators=sorted(e for e in ests if e),
                tol=tol, dt_min=dt_min, dt_max=dt_max, attempts=acc + rej, accepted=acc,
                rejected=rej, t_reached=round(t, 6),
                dt_accepted=[round(min(dts), 8), round(max(dts), 8)] if dts else None,
                iters_per_attempt=round(float(np.mean(its)), 2) if its else None,
                attempts_per_s=round((acc + rej) / el, 1), wall_s=round(el, 3))


def ensemble_bandwidth(ws, steps, warmup, label):
    """All instances in one context (grouped launches): time-steps/s of the
    whole set and the effective bandwidth algorithmic bytes x iterations /
    wall time (setup, accept and host polls included)."""
    import torch
    from paper_2204_07247_amd import pfch
    ctx = pfch.Context([_desc(w) for w in ws])
    ctx.set_stats_detail(0)
    u0 = [torch.from_numpy(W.initial_condition(w)).cuda() for w in ws]
    per_iter = [sum(algorithmic_bytes(w).values()) for w in ws]

    def run(n):
        for i, u in enumerate(u0):
            ctx.set_state(i, u)
        its = np.zeros(len(ws))
        for _ in range(n):
            rc, st = ctx.step([w.dt for w in ws])
            if rc != pfch.PFCH_OK:
                raise RuntimeError(f"{label} step failed: {pfch.strerror(rc)}")
            its += [x["iters"] for x in st]
        return its

    log(f"[bench] {label}: {len(ws)} instances, {steps} steps")
    run(warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    its = run(steps)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    ctx.close()
    moved = float(np.dot(per_iter, its))
    return dict(workload=label, instances=len(ws), points=int(sum(w.npoints for w in ws)),
                steps=steps, instance_steps_per_s=round(len(ws) * steps / el, 2),
                ms_per_step=round(1e3 * el / steps, 3),
                iters_per_step_mean=round(float(its.sum() / (len(ws) * steps)), 3),
                effective_gbs=round(moved / el / 1e9, 1),
                effective_frac=round(moved / el / 1e9 / HBM_PEAK_GBS, 4))


def _learned_vs_plain(w, fno, norm_fn, steps):
    """Plain and learned-guess runs of `steps` steps of w from the same
    initial condition (after 2 untimed steps that build the history)."""
    import torch
    from paper_2204_07247_amd import learned, pfch
    u0 = torch.from_numpy(W.initial_condition(w)).cuda()
    res, finals = {}, {}
    for mode in ("plain", "learned"):
        ctx = pfch.Context([learned.desc_of(w, guess=1 if mode == "learned" else 0)])
        ctx.set_stats_detail(0)
        ctx.set_state(0, u0)
        for _ in range(2):
            ctx.step(w.dt)
        if mode == "learned":
            un, unm1 = torch.empty_like(u0), torch.empty_like(u0)
            ctx.get_state(0, un, unm1)
            ctx.set_fno(0, fno, norm_fn(un, unm1))
        its, kinds = [], []
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            rc, st = ctx.step(w.dt)
            if rc != pfch.PFCH_OK:
                raise RuntimeError(f"{mode} step failed: {pfch.strerror(rc)}")
            its.append(st[0]["iters"])
            kinds.append(st[0]["guess"])
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        out = torch.empty_like(u0)
        ctx.get_state(0, out)
        finals[mode] = out
        ctx.close()
        res[mode] = dict(steps_per_s=round(steps / el, 2), iters_per_step=round(float(np.mean(its)), 3))
        if mode == "learned":
            res[mode]["fallbacks"] = int(sum(k == 2 for k in kinds))
    x = torch.zeros((1, 2) + tuple(w.shape), dtype=torch.float32, device="cuda")
    fno.forward(x)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(10):
        fno.forward(x)
    torch.cuda.synchronize()
    res["fno_forward_ms"] = round(1e3 * (time.perf_counter() - t0) / 10, 3)
    res["steps"] = steps
    res["learned_over_plain_steps_per_s"] = round(res["learned"]["steps_per_s"] / res["plain"]["steps_per_s"], 3)
    res["final_max_abs_diff"] = float((finals["learned"] - finals["plain"]).abs().max().item())
    return res


def learned_comparison(epochs, eval_steps, deploy_steps):
    """FNO warm start trained on solver trajectories of the FCH 256^2
    generator (seeds 100-119, 100 steps each, 10% of the triples held out),
    then plain vs learned guess on FCH 256^2 (seed 0) and, with the same
    weights, on PFC 1024^2."""
    import dataclasses

    import torch
    from paper_2204_07247_amd import learned
    base = W.FCH256_BDF2
    ws = [dataclasses.replace(base, seeds=(s,)) for s in range(100, 120)]
    u0s = [torch.from_numpy(W.initial_condition(w)).cuda() for w in ws]
    cfg = learned.TrainConfig(epochs=epochs)
    log(f"[bench] learned guess: trajectories and training ({epochs} epochs)")
    t0 = time.perf_counter()
    tr = learned.train(ws, u0s, base.steps, cfg, log=log)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    res = dict(network=dict(width=cfg.width, modes=cfg.modes, layers=cfg.layers, dtype="f32"),
               training=dict(data=f"{len(ws)} x {base.steps} steps of {base.name} (seeds 100-119)",
                             triples=tr.n_train + tr.n_val, held_out=tr.n_val, epochs=epochs,
                             batch=cfg.batch, lr=cfg.lr, seconds=round(t_train, 1),
                             train_loss=[round(v, 5) for v in tr.train_loss],
                             held_out_loss=[round(v, 5) for v in tr.val_loss]))
    log("[bench] learned guess: FCH 256^2 plain vs learned")
    res[base.name] = _learned_vs_plain(base, tr.fno, lambda un, unm1: tr.norm, eval_steps)
    pfc = WORKLOADS["pfc1024"]
    f = learned.deploy(tr, *pfc.shape, cfg=cfg)
    ratio = tr.norm[3] / tr.norm[2]

    def pfc_norm(un, unm1):
        d = (un - unm1)
        sd = float(d.std().item()) or 1.0
        return (float(un.mean().item()), float(un.std().item()) or 1.0, sd, ratio * sd)

    log("[bench] learned guess: PFC 1024^2 with the FCH-trained weights")
    res[pfc.name + "_fch_trained"] = _learned_vs_plain(pfc, f, pfc_norm, deploy_steps)
    f.close()
    return res, tr, cfg


def learned_pfc_trained(epochs, eval_steps, deploy_steps):
    """The PFC-trained variant: the same network trained on trajectories of
    PFC 256^2 (L = 256, the grid spacing of PFC 1024^2; MP, dt = 0.2; seeds
    100-119, 100 steps each), then plain vs learned guess on PFC 256^2
    (seed 0) and, with the same weights, on PFC 1024^2."""
    import dataclasses

    import torch
    from paper_2204_07247_amd import learned
    big = WORKLOADS["pfc1024"]
    base = dataclasses.replace(big, name="pfc2d_256_mp", shape=(256, 256), lengths=(256.0, 256.0),
                               steps=100)
    ws = [dataclasses.replace(base, seeds=(s,)) for s in range(100, 120)]
    u0s = [torch.from_numpy(W.initial_condition(w)).cuda() for w in ws]
    cfg = learned.TrainConfig(epochs=epochs)
    log(f"[bench] learned guess, PFC-trained: trajectories and training ({epochs} epochs)")
    t0 = time.perf_counter()
    tr = learned.train(ws, u0s, base.steps, cfg, log=log)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    del u0s
    res = dict(training=dict(data=f"{len(ws)} x {base.steps} steps of {base.name} (seeds 100-119)",
                             triples=tr.n_train + tr.n_val, held_out=tr.n_val, epochs=epochs,
                             seconds=round(t_train, 1),
                             held_out_loss=[round(v, 5) for v in tr.val_loss]))
    log("[bench] learned guess, PFC-trained: PFC 256^2 and PFC 1024^2 plain vs learned")
    res[base.name] = _learned_vs_plain(base, tr.fno, lambda un, unm1: tr.norm, eval_steps)
    f = learned.deploy(tr, *big.shape, cfg=cfg)
    res[big.name] = _learned_vs_plain(big, f, lambda un, unm1: tr.norm, deploy_steps)
    f.close()
    tr.fno.close()
    return res


def learned3d_comparison(epochs, traj_steps, eval_steps):
    """FNO warm start (width 16, 8 modes per axis, 4 layers) trained on
    solver trajectories of the PFC 192^3 generator (seeds 100-103,
    `traj_steps` steps each, 10% of the triples held out), then plain vs
    learned guess on PFC 192^3 (seed 0)."""
    import dataclasses

    import torch
    from paper_2204_07247_amd import learned
    base = W.PFC192_3D
    ws = [dataclasses.replace(base, seeds=(s,)) for s in range(100, 104)]
    u0s = [torch.from_numpy(W.initial_condition(w)).cuda() for w in ws]
    cfg = learned.TrainConfig(width=16, modes=8, layers=4, batch=4, epochs=epochs)
    log(f"[bench] learned guess 3D: trajectories and training ({epochs} epochs)")
    t0 = time.perf_counter()
    tr = learned.train(ws, u0s, traj_steps, cfg, log=log)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    del u0s
    res = dict(network=dict(width=cfg.width, modes=cfg.modes, layers=cfg.layers, dtype="f32",
                            params=tr.fno.n_params),
               training=dict(data=f"{len(ws)} x {traj_steps} steps of {base.name} (seeds 100-103)",
                             triples=tr.n_train + tr.n_val, held_out=tr.n_val, epochs=epochs,
                             batch=cfg.batch, lr=cfg.lr, seconds=round(t_train, 1),
                             train_loss=[round(v, 5) for v in tr.train_loss],
                             held_out_loss=[round(v, 5) for v in tr.val_loss]))
    log("[bench] learned guess 3D: PFC 192^3 plain vs learned")
    res[base.name] = _learned_vs_plain(base, tr.fno, lambda un, unm1: tr.norm, eval_steps)
    return res, tr, cfg


def batched_learned(tr2, cfg2, tr3, steps, warmup):
    """The combined set (8 FCH 1024^2 + 8 FCH 2048^2 + PFC 192^3) in one
    context, plain and with the learned guess on every instance: the FCH
    instances share the FCH 256^2-trained weights (one network object per
    grid), the 3D instance uses the PFC 192^3 network.  Each instance's
    input normalisation comes from its own state after the warm-up steps,
    with the training set's ratio of correction to increment spread."""
    import torch
    from paper_2204_07247_amd import learned, pfch
    ws = W.fch_ensemble() + [W.PFC192_3D]
    u0 = [torch.from_numpy(W.initial_condition(w)).cuda() for w in ws]
    nets = {}
    for w in ws:
        if len(w.shape) == 2 and tuple(w.shape) not in nets:
            nets[tuple(w.shape)] = learned.deploy(tr2, *w.shape, cfg=cfg2)
    res = {}
    for mode in ("plain", "learned"):
        ctx = pfch.Context([learned.desc_of(w, guess=1 if mode == "learned" else 0) for w in ws])
        ctx.set_stats_detail(0)
        for i, u in enumerate(u0):
            ctx.set_state(i, u)
        for _ in range(warmup):
            ctx.step([w.dt for w in ws])
        if mode == "learned":
            for i, w in enumerate(ws):
                un, unm1 = torch.empty_like(u0[i]), torch.empty_like(u0[i])
                ctx.get_state(i, un, unm1)
                tr = tr3 if len(w.shape) == 3 else tr2
                d = un - unm1
                sd = float(d.std().item()) or 1.0
                norm = (float(un.mean().item()), float(un.std().item()) or 1.0, sd,
                        tr.norm[3] / tr.norm[2] * sd)
                ctx.set_fno(i, tr3.fno if len(w.shape) == 3 else nets[tuple(w.shape)], norm)
        its = np.zeros(len(ws))
        kinds = []
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            rc, st = ctx.step([w.dt for w in ws])
            if rc != pfch.PFCH_OK:
                raise RuntimeError(f"batched {mode} step failed: {pfch.strerror(rc)}")
            its += [x["iters"] for x in st]
            kinds += [x["guess"] for x in st]
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        ctx.close()
        res[mode] = dict(instance_steps_per_s=round(len(ws) * steps / el, 2),
                         ms_per_step=round(1e3 * el / steps, 3),
                         iters_per_step_mean=round(float(its.sum() / (len(ws) * steps)), 3))
        if mode == "learned":
            res[mode]["learned_guesses"] = int(sum(k == 1 for k in kinds))
            res[mode]["fallbacks"] = int(sum(k == 2 for k in kinds))
    for f in nets.values():
        f.close()
    res.update(workload="fch2d_8x1024_8x2048_bdf2 + pfc3d_192_bdf2", instances=len(ws), steps=steps,
               learned_over_plain=round(res["learned"]["instance_steps_per_s"] /
                                        res["plain"]["instance_steps_per_s"], 3))
    return res


def cpu_baseline(w, max_steps, budget_s):
    """The CPU oracle on the same workload, first steps of the same trajectory."""
    from oracle import driver, models, spectral
    g = spectral.Grid(w.shape, w.lengths)
    m = models.make_model(w.model, **w.params())
    sim = driver.Simulation(g, m, w.scheme, s=w.s, etas=w.etas, tol=w.tol, max_iter=w.max_iter)
    u, up, dto = W.initial_condition(w), None, None
    t0 = time.perf_counter()
    n = 0
    while n < max_steps and time.perf_counter() - t0 < budget_s:
        out = sim.step(u, up, w.dt, dto)
        up, u, dto = u, out["x"], w.dt
        n += 1
    el = time.perf_counter() - t0
    return dict(value=n / el, unit="time-steps/s", cores=1, kind="oracle",
                sample=f"first {n} of {max_steps} steps of {w.name} (seed {w.seeds[0]}), "
                       f"{el:.1f} s, NumPy float64 pocketfft, single thread",
                host_cpus=os.cpu_count(), host_cpus_usable=len(os.sched_getaffinity(0)))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="fch256", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU-oracle baseline")
    ap.add_argument("--cpu-budget", type=float, default=20.0, help="seconds of oracle work")
    ap.add_argument("--no-kernel-timing", action="store_true")
    ap.add_argument("--no-compare", action="store_true",
                    help="skip the batched-ensemble comparison")
    ap.add_argument("--ensemble", type=int, default=64, help="instances in the batched comparison")
    ap.add_argument("--no-learned", action="store_true", help="skip the learned-guess comparison")
    ap.add_argument("--learned-epochs", type=int, default=8)
    ap.add_argument("--learned3d-epochs", type=int, default=6,
                    help="epochs of the PFC 192^3 learned-guess comparison (0 skips it)")
    ap.add_argument("--tune-file", default=os.path.join(ROOT, "paper_2204_07247_amd", "tune_mi355x.txt"),
                    help="plan choices of the autotuner to reuse (PFCH_TUNE_FILE; an already set "
                         "environment variable wins; '' times every plan afresh)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="before the run, copy a MIB-sized float64 buffer three times "
                         "(a plain copy kernel of known traffic for counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for {args.gpus}): the library runs on one "
              "device; independent instances would shard across GPUs with no communication, "
              "which is not implemented", file=sys.stderr)
        sys.exit(2)
    if args.tune_file and "PFCH_TUNE_FILE" not in os.environ:
        os.environ["PFCH_TUNE_FILE"] = args.tune_file
    w = WORKLOADS[args.workload]
    if args.copy_calibration:
        import torch
        n = args.copy_calibration * (1 << 20) // 8
        src = torch.rand(n, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        log(f"[bench] calibration copy: 3 x {args.copy_calibration} MiB read + write")
        del src, dst
    elapsed, iters, timing, cfg = gpu_run(w, args.steps, args.warmup, not args.no_kernel_timing)
    if os.environ.get("PFCH_TUNE_FILE"):
        cfg["tune_file"] = os.path.relpath(os.environ["PFCH_TUNE_FILE"], ROOT)
    value = args.steps / elapsed
    ab = algorithmic_bytes(w)
    roof = None
    kernels = {}
    if timing:
        for k in ab:
            avg = timing[f"{k}_us"] * 1e-6
            kernels[k] = dict(avg_us=round(avg * 1e6, 3), solves=timing["solves"], alg_bytes=ab[k],
                              achieved_gbs=round(ab[k] / avg / 1e9, 2),
                              back_to_back_us=round(timing["back_to_back"][f"{k}_us"], 3))
        dom = max(kernels, key=lambda k: kernels[k]["avg_us"])
        kd = kernels[dom]
        roof = dict(bound="hbm", kernel=KERNEL_NAMES[dom], achieved=kd["achieved_gbs"],
                    peak=HBM_PEAK_GBS, unit="GB/s",
                    frac=round(kd["achieved_gbs"] / HBM_PEAK_GBS, 4),
                    traffic=measured_traffic(w, dom))
    batched = None
    if not args.no_compare:
        batched = batched_comparison(args.ensemble, steps=10, solo_steps=4)
    ensembles = None
    if not args.no_compare:
        ensembles = [
            ensemble_bandwidth(W.pfc_ensemble(count=64), steps=10, warmup=2,
                               label="pfc2d_ensemble64 (128..512, MP)"),
            ensemble_bandwidth(W.fch_ensemble() + [W.PFC192_3D], steps=5, warmup=2,
                               label="fch2d_8x1024_8x2048_bdf2 + pfc3d_192_bdf2"),
        ]
    variants = None
    if not args.no_compare:
        variants = [solver_variants(w, steps=min(w.steps, 50)),
                    solver_variants(W.PFC64_MP, steps=W.PFC64_MP.steps)]
    adaptive = None
    if not args.no_compare:
        log("[bench] adaptive stepping (AM3 / midAB2)")
        adaptive = [adaptive_run(W.FCH256_BDF2, 1e-4, 1e-5, 0.5, attempts=200),
                    adaptive_run(W.PFC64_MP, 1e-4, 1e-4, 0.5, attempts=200)]
    learned_res = None
    if not args.no_learned and not args.no_compare:
        learned_res, tr2, cfg2 = learned_comparison(args.learned_epochs, eval_steps=100, deploy_steps=20)
        learned_res["pfc_trained"] = learned_pfc_trained(args.learned_epochs, eval_steps=100,
                                                         deploy_steps=20)
        if args.learned3d_epochs > 0:
            learned_res["pfc3d"], tr3, _ = learned3d_comparison(args.learned3d_epochs, traj_steps=40,
                                                                eval_steps=40)
            log("[bench] batched + learned: FCH 8x1024^2 + 8x2048^2 + PFC 192^3")
            learned_res["batched"] = batched_learned(tr2, cfg2, tr3, steps=5, warmup=2)
            tr3.fno.close()
        tr2.fno.close()
    cpu = None
    if not args.no_cpu:
        log("[bench] CPU oracle baseline")
        cpu = cpu_baseline(w, w.steps, args.cpu_budget)
    it = np.array(iters)
    fft_pairs = {"pfc": 1.5, "fch": 2.5}[w.model]
    out = dict(
        metric=METRIC, value=round(value, 3), unit="time-steps/s", n_gpus=1, steps=args.steps,
        warmup=args.warmup, ms_per_step=round(1e3 * elapsed / args.steps, 4),
        higher_is_better=True, scaling="weak", vs_baseline=None, dtype="f64", data="synthetic",
        config=dict(workload=w.name, grid=list(w.shape), lengths=list(w.lengths),
                    scheme=w.scheme, dt=w.dt, tol=w.tol, s=w.s, seed=w.seeds[0]),
        iters_per_step=dict(mean=round(float(it.mean()), 3), min=int(it.min()), max=int(it.max())),
        fft_pairs_per_iter=fft_pairs,
        roofline=roof, kernels=kernels, launch=cfg, cpu_baseline=cpu, batched=batched,
        learned=learned_res, ensembles=ensembles, solver_variants=variants, adaptive=adaptive,
    )
    if cpu:
        out["gpu_over_cpu"] = round(value / cpu["value"], 2)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
