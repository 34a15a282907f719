"""Throughput of the PAGD-solved fully implicit steps on one MI355X.

Default workload, the combined set: 8 FCH 2D instances at 1024 x 1024 and 8
at 2048 x 2048 on [0, 4 pi)^2 (e ~ U[0.08, 0.12], eps = e, eta1 = 1.45 e,
eta2 = 2 e, tau = 0, mean ~ U[-0.7, -0.5], noise amplitude 0.01; seeds
2000-2015) and one PFC 3D instance at 192^3 on [0, 192)^3 (eps = 0.25, mean
-0.2, noise 0.05, seed 0); BDF2 with a backward Euler first step, dt = 1e-3
(FCH) and 0.1 (PFC); PAGD to ||d||_inf < 1e-10; 300 steps.  One bench step is
one time step of every instance.  All inputs are seeded synthetic fields (workloads/),
resident on the GPU before the timed region.

The same steps run four ways:
  plain            one context per instance, extrapolated initial guess;
  batched          all instances in one context (grouped launches);
  learned          one context per instance, learned guess on the FCH
                   instances (a float32 FNO: 4 spectral layers, 16 modes,
                   width 32, GELU, run on its own 64 x 64 grid of the
                   band-limited state, trained on 300-step FCH 256^2
                   trajectories with the set's parameter spread and the
                   same periods, and fed with the training set's
                   normalisation); the 3D instance keeps the extrapolated
                   guess;
  batched_learned  both: the headline `value`.
Each times `--steps` bench steps (default: the configuration's 300) from the
initial conditions, bracketed by torch.cuda.synchronize(), after `--warmup`
untimed steps whose states are discarded.  Also reported: PAGD iterations per step, the HBM
roofline of the FCH 2048^2 iteration (HIP events on the grouped launches),
the CPU oracle on the host's cores, and the paper's own timings as context
(its hardware is not stated).

Prints one JSON line.  --workload names a single-instance workload instead;
--extras adds the other comparisons (PFC ensemble, learned guess on PFC,
solver variants, adaptive stepping, 3D network).
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
COMBINED = "fch2d_8x1024_8x2048_bdf2+pfc3d_192_bdf2"
COMBINED_STEPS = 300

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


def combined_set():
    return W.fch_ensemble() + [W.PFC192_3D]


def log(msg):
    print(msg, file=sys.stderr, flush=True)


KERNEL_NAMES = {"row": "k_row_iter", "col": "k_col_iter", "yfwd": "k_y3_iter<fwd>",
                "z": "k_z3_iter", "yinv": "k_y3_iter<inv>"}

# Compulsory HBM bytes per grid point and PAGD iteration of the reference
# three-pass fused schedule (one out-of-LDS round trip per transform
# direction; the state x_j, x_{j-1}, their transforms and the step constant
# read once, the new iterate and its transform written once).  The kernels
# here carry the iterate in real space only and move fewer bytes (see
# algorithmic_bytes); the roofline is quoted against these figures.
SCHEDULE_BYTES = {("fch", "bdf2", 2): 160, ("fch", "mp", 2): 176, ("pfc", "bdf2", 2): 104,
                  ("pfc", "mp", 2): 120, ("pfc", "bdf2", 3): 136}


# Transform pairs per PAGD iteration (one forward and one inverse transform
# of a real field count as one pair): PFC 2 forward + 1 inverse, FCH 3 + 2.
PAIRS_PER_ITER = {"pfc": 1.5, "fch": 2.5}

# The paper's own timings, as context only: its benchmark table of the PAGD
# solved MP and BDF2 runs (Table tab:expbenchmark_csv) gives FFT pairs and
# wall-clock seconds per adaptive run; its hardware, FFT library and thread
# count are not stated (CPU time is 5-10 times the wall time: a multicore
# CPU).  Rates below are pairs / wall second, and grid points x pairs /
# wall second.
PAPER_RUNS = [  # (problem, scheme, N per axis, FFT pairs, wall s)
    ("FCH1", "MP", 128, 43769, 14), ("FCH1", "BDF2", 128, 77385, 23),
    ("FCH2", "MP", 256, 122049, 116), ("FCH2", "BDF2", 256, 106425, 90),
    ("FCH3", "MP", 256, 113089, 112), ("FCH3", "BDF2", 256, 142293, 120),
    ("PFC1", "MP", 512, 78289, 595), ("PFC1", "BDF2", 512, 82485, 437),
    ("PFC2", "MP", 512, 25551, 77), ("PFC2", "BDF2", 512, 237792, 747),
]


def paper_context(point_pairs_per_s):
    rates = [(p, sch, n, pairs / wall, n * n * pairs / wall) for p, sch, n, pairs, wall in PAPER_RUNS]
    lo = min(r[4] for r in rates)
    hi = max(r[4] for r in rates)
    return dict(
        source="the paper's benchmark table of PAGD-solved MP / BDF2 runs (Table tab:expbenchmark_csv)",
        hardware="not stated (CPU time 5-10 x wall time: a multicore CPU)",
        runs=[dict(problem=p, scheme=sch, grid=f"{n}^2", fft_pairs_per_s=round(r, 1),
                   mpoint_pairs_per_s=round(q / 1e6, 1)) for p, sch, n, r, q in rates],
        paper_mpoint_pairs_per_s=[round(lo / 1e6, 1), round(hi / 1e6, 1)],
        unit_mpoint_pairs="10^6 grid points x transform pairs per wall second",
        this_run_mpoint_pairs_per_s=round(point_pairs_per_s / 1e6, 1),
        note="context, not a like-for-like comparison: other grids, problems and an adaptive step size there; "
             "here the transform pairs of the PAGD iterations only")


def algorithmic_bytes(w):
    """Bytes the iteration kernels themselves must move per launch (one
    instance): real field = Ny*Nx (*Nz) doubles; spectral field = half as
    many complex doubles (the half spectrum's two real columns kx = 0 and
    kx = Nx/2 share one).  PFC row kernel: read 1 spectral + x_j, x_{j-1}
    (+ u^n for MP), write x_{j+1} + 2 spectral.  PFC column kernel: read 2
    spectral + g^, write 1.  FCH row kernel: read 2 spectral + x_j, x_{j-1},
    Lx_j, Lx_{j-1} (+ u^n, Lu^n for MP), write x_{j+1}, Lx_{j+1} + 3
    spectral.  FCH column kernel: read 3 spectral + g^, write 2 spectral.
    3D PFC: the row kernel as in 2D; y forward: read and write 2 spectral;
    z: read 2 spectral + g^, write 1; y inverse: read and write 1 spectral.
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


def measured_traffic(name, kernel):
    """HBM bytes per launch from the committed PMC summary, if it was taken on
    the current kernel sources; otherwise None."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        rec = json.load(fh)
    ent = rec.get(name, {}).get(kernel)
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


# ---------------------------------------------------------------------------
# CPU oracle baseline (runs before the GPU is touched: the worker processes
# are forked from this one)
# ---------------------------------------------------------------------------
def _oracle_first_step(w):
    from oracle import driver, models, spectral
    g = spectral.Grid(w.shape, w.lengths)
    m = models.make_model(w.model, **w.params())
    sim = driver.Simulation(g, m, w.scheme, s=w.s, etas=w.etas, tol=w.tol, max_iter=w.max_iter)
    u0 = W.initial_condition(w)
    t0 = time.perf_counter()
    out = sim.step(u0, None, w.dt, None)
    return w.name, time.perf_counter() - t0, int(out["iters"])


def cpu_baseline_set(ws):
    """The oracle's first time step (backward Euler, the same iterations as
    the GPU's first step) of every instance of the set, one single-threaded
    process per instance on the host's usable cores: the wall time of the
    whole set-step (all cores) and the sum of the per-instance times (one
    core)."""
    import multiprocessing as mp
    usable = len(os.sched_getaffinity(0))
    procs = max(1, min(len(ws), usable))
    order = sorted(ws, key=lambda w: -w.npoints)  # largest first
    t0 = time.perf_counter()
    with mp.get_context("fork").Pool(procs) as pool:
        res = pool.map(_oracle_first_step, order, chunksize=1)
    wall = time.perf_counter() - t0
    one = sum(r[1] for r in res)
    return dict(value=round(1.0 / wall, 5), unit="time-steps/s", cores=procs, kind="oracle",
                sample=f"first time step (backward Euler) of all {len(ws)} instances of {COMBINED}, "
                       f"one single-threaded NumPy float64 process per instance on {procs} cores: "
                       f"{wall:.1f} s wall",
                single_core=dict(value=round(1.0 / one, 6), unit="time-steps/s", cores=1,
                                 sample=f"sum of the {len(ws)} per-instance times measured in those "
                                        f"processes: {one:.1f} s"),
                iters=[r[2] for r in res],
                host_cpus=os.cpu_count(), host_cpus_usable=usable)


def cpu_baseline(w, max_steps, budget_s):
    """The CPU oracle on a single-instance workload: the first steps of the
    same trajectory, one thread."""
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


# ---------------------------------------------------------------------------
# The combined set: plain / batched / learned / batched + learned
# ---------------------------------------------------------------------------
def train_fch_network(epochs):
    """The FCH warm-start network: FNO (4 spectral layers, 16 modes, width 32,
    GELU, float32) on its own 64 x 64 grid, trained on 16 trajectories of
    300 steps of FCH 256^2 instances on the combined set's period with the
    set's parameter spread (e ~ U[0.08, 0.12], mean ~ U[-0.7, -0.5]; seeds
    100-115), resampled to that grid, 10% of the triples held out.  The
    trajectories cover the horizon the network is deployed on, and the
    deployed guesses use the training set's normalisation."""
    import torch
    from paper_2204_07247_amd import learned
    ws = W.fch_ensemble(count_per_size=16, sizes=(256,), steps=COMBINED_STEPS, base_seed=100)
    u0s = [torch.from_numpy(W.initial_condition(w)).cuda() for w in ws]
    cfg = learned.TrainConfig(width=32, modes=16, layers=4, epochs=epochs, grid=(64, 64))
    log(f"[bench] FCH network: trajectories and training ({epochs} epochs)")
    t0 = time.perf_counter()
    tr = learned.train(ws, u0s, COMBINED_STEPS, cfg, log=log)
    del u0s
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    info = dict(network=dict(width=cfg.width, modes=cfg.modes, layers=cfg.layers, grid=list(cfg.grid),
                             dtype="f32", params=tr.fno.n_params),
                training=dict(data=f"{len(ws)} x {COMBINED_STEPS} steps of FCH 256^2 on [0, 4 pi)^2 with "
                                   f"e ~ U[0.08, 0.12], mean ~ U[-0.7, -0.5] (seeds 100-{100 + len(ws) - 1}), "
                                   f"resampled to the network's grid",
                              triples=tr.n_train + tr.n_val, held_out=tr.n_val, epochs=epochs, batch=cfg.batch,
                              lr=cfg.lr, seconds=round(time.perf_counter() - t0, 1),
                              held_out_loss=[round(v, 5) for v in tr.val_loss],
                              normalisation=[float(v) for v in tr.norm]))
    return tr, info


def run_set(ws, mode, steps, warmup, tr=None, time_groups=None):
    """`steps` bench steps of the instances ws from their initial conditions
    (the configuration's steps 1 .. steps), after `warmup` untimed ones
    that are then discarded.  mode: plain | batched | learned |
    batched_learned."""
    import torch
    from paper_2204_07247_amd import learned, pfch
    batched = mode.startswith("batched")
    use_net = mode.endswith("learned")
    guess = [1 if use_net and w.model == "fch" and len(w.shape) == 2 else 0 for w in ws]
    if batched:
        ctxs = [(pfch.Context([learned.desc_of(w, g) for w, g in zip(ws, guess)]), list(range(len(ws))))]
    else:
        ctxs = [(pfch.Context([learned.desc_of(w, g)]), [i]) for i, (w, g) in enumerate(zip(ws, guess))]
    u = [torch.from_numpy(W.initial_condition(w)).cuda() for w in ws]
    for c, idx in ctxs:
        c.set_stats_detail(0)
        for k, i in enumerate(idx):
            c.set_state(k, u[i])
    dts = [[ws[i].dt for i in idx] for _, idx in ctxs]

    def one_step(its):
        for (c, idx), dt in zip(ctxs, dts):
            rc, st = c.step(dt)
            if rc != pfch.PFCH_OK:
                raise RuntimeError(f"{mode} step failed: {pfch.strerror(rc)}")
            for k, i in enumerate(idx):
                its[i].append(st[k]["iters"])
                if st[k]["guess"] == 2:
                    its["fallbacks"] += 1

    warm = {i: [] for i in range(len(ws))}
    warm["fallbacks"] = 0
    for _ in range(max(1, warmup)):
        one_step(warm)
    if use_net:  # the network with the training set's normalisation
        for c, idx in ctxs:
            for k, i in enumerate(idx):
                if guess[i]:
                    c.set_fno(k, tr.fno, tr.norm)
        one_step(warm)  # the first learned step, untimed
    # back to the initial conditions: the timed steps are the configuration's
    # first `steps` steps (a step without history is backward Euler with the
    # extrapolated guess; the network is used from the second step on)
    for c, idx in ctxs:
        for k, i in enumerate(idx):
            c.set_state(k, u[i])
    its = {i: [] for i in range(len(ws))}
    its["fallbacks"] = 0
    log(f"[bench] {mode}: {len(ws)} instances, {len(ctxs)} context(s), {steps} timed steps")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        one_step(its)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    log(f"[bench] {mode}: timed region done: {el:.4f} s")
    timing = None
    if time_groups and batched:
        c = ctxs[0][0]
        timing = {name: c.time_group(inst, ws[inst].dt, 5) for name, inst in time_groups.items()}
    for c, _ in ctxs:
        c.close()
    per = [np.mean(its[i]) for i in range(len(ws))]
    # whole-solve bandwidth: the schedule's bytes of every iteration run,
    # over the wall time (set-ups, accepts and host round trips included)
    moved = sum(SCHEDULE_BYTES[(w.model, w.scheme, len(w.shape))] * w.npoints * sum(its[i])
                for i, w in enumerate(ws))
    pairs = sum(PAIRS_PER_ITER[w.model] * w.npoints * sum(its[i]) for i, w in enumerate(ws))
    groups = {}
    for w, p in zip(ws, per):
        key = f"{w.model}{'x'.join(map(str, w.shape))}"
        groups.setdefault(key, []).append(p)
    out = dict(time_steps_per_s=round(steps / el, 3), instance_steps_per_s=round(len(ws) * steps / el, 2),
               ms_per_step=round(1e3 * el / steps, 3), iters_per_step=round(float(np.mean(per)), 3),
               iters_per_step_by_grid={k: round(float(np.mean(v)), 3) for k, v in groups.items()},
               contexts=len(ctxs), elapsed_s=round(el, 4),
               effective_gbs=round(moved / el / 1e9, 1), effective_frac=round(moved / el / 1e9 / HBM_PEAK_GBS, 4),
               point_pairs_per_s=round(pairs / el, 1))
    if use_net:
        out["learned_guess_instances"] = int(sum(guess))
        out["fallbacks"] = its["fallbacks"]
    return out, timing


def combined_bench(args):
    import torch
    ws = combined_set()
    tr, net_info = (None, None) if args.no_learned else train_fch_network(args.learned_epochs)
    first8 = next(i for i, w in enumerate(ws) if w.shape == (2048, 2048))
    i3 = next(i for i, w in enumerate(ws) if len(w.shape) == 3)
    groups = {"fch2048": first8, "fch1024": 0, "pfc192_3d": i3}
    variants = {}
    headline = "batched" if tr is None else "batched_learned"
    for mode in ("plain", "batched", "learned"):
        if (args.only and args.only != mode) or (tr is None and mode == "learned") or mode == headline:
            continue
        variants[mode], _ = run_set(ws, mode, args.steps, args.warmup, tr)
        torch.cuda.empty_cache()
    # the headline configuration last, with the kernel timing of its grouped
    # launches (without a network: the batched run)
    head, timing = run_set(ws, headline, args.steps, args.warmup, tr,
                           time_groups=None if args.no_kernel_timing else groups)
    variants[headline] = head
    if tr is not None:
        tr.fno.close()
    if "plain" in variants:
        plain = variants["plain"]["time_steps_per_s"]
        for k in variants:
            variants[k]["over_plain"] = round(variants[k]["time_steps_per_s"] / plain, 3)
    roof, kernels = None, {}
    if timing:
        for name, inst in groups.items():
            w = ws[inst]
            nm = sum(1 for v in ws if v.shape == w.shape and v.model == w.model)
            ab = algorithmic_bytes(w)
            t = dict(timing[name])
            # time per iteration of the chain of grouped launches (events
            # around the chain); the per-launch event pairs add a few
            # microseconds to each launch and give the split between kernels
            per_iter_us = t.pop("iteration_us")
            sched = SCHEDULE_BYTES[(w.model, w.scheme, len(w.shape))] * w.npoints * nm
            kernels[name] = dict(
                instances_per_launch=nm,
                launches_us={k: round(v, 2) for k, v in t.items()},
                launches_sum_us=round(sum(t.values()), 2),
                iteration_us=round(per_iter_us, 2),
                schedule_bytes_per_iter=sched,
                schedule_gbs=round(sched / (per_iter_us * 1e-6) / 1e9, 1),
                kernel_bytes_per_iter=nm * sum(ab.values()),
                kernel_gbs={k: round(nm * ab[k.replace("_us", "")] / (v * 1e-6) / 1e9, 1)
                            for k, v in t.items()})
        k8 = kernels["fch2048"]
        w8 = ws[first8]
        roof = dict(bound="hbm",
                    kernel="PAGD iteration of the FCH 2048^2 group: k_col_iter + k_row_iter, "
                           "8 instances per launch",
                    achieved=k8["schedule_gbs"], peak=HBM_PEAK_GBS, unit="GB/s",
                    frac=round(k8["schedule_gbs"] / HBM_PEAK_GBS, 4),
                    traffic=measured_traffic(COMBINED, "fch2048_iteration"),
                    bytes_per_point_per_iter=SCHEDULE_BYTES[("fch", "bdf2", 2)],
                    points_per_launch=8 * w8.npoints, launch_us=k8["iteration_us"])
    cfg = dict(workload=COMBINED, instances=len(ws), points=int(sum(w.npoints for w in ws)),
               grids={"fch2d_1024": 8, "fch2d_2048": 8, "pfc3d_192": 1}, scheme="bdf2",
               dt={"fch": 1e-3, "pfc": 0.1}, tol=1e-10, s=0.9, seeds="2000-2015 (FCH), 0 (PFC 3D)",
               headline=headline,
               guess="extrapolated" if tr is None else
               "learned on the FCH instances, extrapolated on the 3D instance")
    return dict(value=head["time_steps_per_s"], ms_per_step=head["ms_per_step"], config=cfg,
                iters_per_step=head["iters_per_step"], variants=variants, roofline=roof, kernels=kernels,
                learned_network=net_info, paper_context=paper_context(head["point_pairs_per_s"]))


# ---------------------------------------------------------------------------
# A single-instance workload (--workload)
# ---------------------------------------------------------------------------
def gpu_run(w, steps, warmup, kernel_timing):
    import torch
    from paper_2204_07247_amd import pfch

    ctx = pfch.Context([_desc(w)])
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


def single_bench(args, w):
    elapsed, iters, timing, cfg = gpu_run(w, args.steps, args.warmup, not args.no_kernel_timing)
    ab = algorithmic_bytes(w)
    roof, kernels = None, {}
    if timing:
        for k in ab:
            avg = timing[f"{k}_us"] * 1e-6
            kernels[k] = dict(avg_us=round(avg * 1e6, 3), solves=timing["solves"], alg_bytes=ab[k],
                              achieved_gbs=round(ab[k] / avg / 1e9, 2),
                              back_to_back_us=round(timing["back_to_back"][f"{k}_us"], 3))
        # per iteration of the chain of launches, without per-launch events
        iter_us = timing["iteration_us"]
        sched = SCHEDULE_BYTES[(w.model, w.scheme, len(w.shape))] * w.npoints
        roof = dict(bound="hbm", kernel=f"PAGD iteration ({' + '.join(KERNEL_NAMES[k] for k in kernels)})",
                    achieved=round(sched / (iter_us * 1e-6) / 1e9, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                    frac=round(sched / (iter_us * 1e-6) / 1e9 / HBM_PEAK_GBS, 4),
                    traffic=measured_traffic(w.name, "iteration"),
                    bytes_per_point_per_iter=SCHEDULE_BYTES[(w.model, w.scheme, len(w.shape))],
                    points_per_launch=w.npoints, launch_us=round(iter_us, 3))
    it = np.array(iters)
    cfg.update(workload=w.name, grid=list(w.shape), lengths=list(w.lengths), scheme=w.scheme, dt=w.dt,
               tol=w.tol, s=w.s, seed=w.seeds[0])
    return dict(value=round(args.steps / elapsed, 3), ms_per_step=round(1e3 * elapsed / args.steps, 4),
                config=cfg,
                iters_per_step=dict(mean=round(float(it.mean()), 3), min=int(it.min()), max=int(it.max())),
                roofline=roof, kernels=kernels,
                paper_context=paper_context(PAIRS_PER_ITER[w.model] * w.npoints * float(it.sum()) / elapsed))


# ---------------------------------------------------------------------------
# Extra comparisons (--extras)
# ---------------------------------------------------------------------------
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
    fft_pairs = PAIRS_PER_ITER[w.model]
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
    whole set and the effective bandwidth bytes x iterations / wall time
    (setup, accept and host polls included), on the schedule's bytes per
    point and iteration (as the combined set's variants report it) and on
    the bytes the iteration kernels themselves move."""
    import torch
    from paper_2204_07247_amd import pfch
    ctx = pfch.Context([_desc(w) for w in ws])
    ctx.set_stats_detail(0)
    u0 = [torch.from_numpy(W.initial_condition(w)).cuda() for w in ws]
    per_iter = [sum(algorithmic_bytes(w).values()) for w in ws]
    per_iter_sched = [SCHEDULE_BYTES[(w.model, w.scheme, len(w.shape))] * w.npoints for w in ws]

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
    sched = float(np.dot(per_iter_sched, its))
    return dict(workload=label, instances=len(ws), points=int(sum(w.npoints for w in ws)),
                steps=steps, instance_steps_per_s=round(len(ws) * steps / el, 2),
                ms_per_step=round(1e3 * el / steps, 3),
                iters_per_step_mean=round(float(its.sum() / (len(ws) * steps)), 3),
                effective_gbs=round(sched / el / 1e9, 1),
                effective_frac=round(sched / el / 1e9 / HBM_PEAK_GBS, 4),
                kernel_bytes_gbs=round(moved / el / 1e9, 1),
                kernel_bytes_frac=round(moved / el / 1e9 / HBM_PEAK_GBS, 4))


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


def extras(args):
    out = {}
    # the PFC ensemble over its full 200 steps (one context per instance:
    # the first 20)
    out["pfc_ensemble"] = batched_comparison(64, steps=200, solo_steps=20)
    out["ensembles"] = [ensemble_bandwidth(W.pfc_ensemble(count=64), steps=200, warmup=2,
                                           label="pfc2d_ensemble64 (128..512, MP)")]
    out["solver_variants"] = [solver_variants(W.FCH256_BDF2, steps=50),
                              solver_variants(W.PFC64_MP, steps=W.PFC64_MP.steps)]
    log("[bench] adaptive stepping (AM3 / midAB2)")
    out["adaptive"] = [adaptive_run(W.FCH256_BDF2, 1e-4, 1e-5, 0.5, attempts=200),
                       adaptive_run(W.PFC64_MP, 1e-4, 1e-4, 0.5, attempts=200),
                       adaptive_run(W.PFC192_3D, 1e-4, 1e-4, 0.5, attempts=100)]
    # PFC 1024^2 deployments over the learned-guess workload's 500 steps
    lr, tr2, _ = learned_comparison(args.learned_epochs, eval_steps=100, deploy_steps=500)
    tr2.fno.close()
    lr["pfc_trained"] = learned_pfc_trained(args.learned_epochs, eval_steps=100, deploy_steps=500)
    if args.learned3d_epochs > 0:
        lr["pfc3d"], tr3, _ = learned3d_comparison(args.learned3d_epochs, traj_steps=40, eval_steps=40)
        tr3.fno.close()
    out["learned"] = lr
    return out


def per_step_comparison(args):
    """The 16 FCH instances of the combined set in one context, extrapolated
    against learned guess (the bench's network, with its gain and gate), over
    the configuration's steps: per block of 20 steps the mean PAGD iterations
    of the 1024^2 and 2048^2 instances both ways, the mean fitted gain of the
    steps that ran the network, and the share of instance-steps that ran it."""
    import torch
    from paper_2204_07247_amd import learned, pfch
    ws = [w for w in combined_set() if len(w.shape) == 2]
    steps = args.steps or COMBINED_STEPS
    tr, _ = train_fch_network(args.learned_epochs)
    u = [torch.from_numpy(W.initial_condition(w)).cuda() for w in ws]
    its, gains = {}, None
    for mode in ("plain", "learned"):
        g = 1 if mode == "learned" else 0
        ctx = pfch.Context([learned.desc_of(w, g) for w in ws])
        ctx.set_stats_detail(0)
        for k in range(len(ws)):
            ctx.set_state(k, u[k])
            if g:
                ctx.set_fno(k, tr.fno, tr.norm)
        it = np.zeros((len(ws), steps))
        gn = np.full((len(ws), steps), np.nan)
        log(f"[bench] per-step {mode}: {len(ws)} instances, {steps} steps")
        for n in range(steps):
            rc, st = ctx.step([w.dt for w in ws])
            if rc != pfch.PFCH_OK:
                raise RuntimeError(f"per-step {mode}: {pfch.strerror(rc)}")
            for k in range(len(ws)):
                it[k, n] = st[k]["iters"]
                if st[k]["guess"] == 1:
                    gn[k, n] = st[k]["gain"]
        ctx.close()
        its[mode] = it
        if g:
            gains = gn
    tr.fno.close()
    by = {s: [i for i, w in enumerate(ws) if w.shape == (s, s)] for s in (1024, 2048)}
    blocks = []
    for a in range(0, steps, 20):
        sl = slice(a, min(a + 20, steps))
        blk = dict(steps=f"{a + 1}-{min(a + 20, steps)}")
        for s, idx in by.items():
            blk[f"fch{s}"] = [round(float(its["plain"][idx, sl].mean()), 2),
                              round(float(its["learned"][idx, sl].mean()), 2)]
        used = ~np.isnan(gains[:, sl])
        blk["network_share"] = round(float(used.mean()), 3)
        blk["mean_fitted_gain"] = round(float(np.nanmean(gains[:, sl])), 3) if used.any() else None
        blocks.append(blk)
    return dict(workload=COMBINED + " (its 16 FCH instances, one context)", steps=steps,
                iters_per_step=dict(plain=round(float(its["plain"].mean()), 3),
                                    learned=round(float(its["learned"].mean()), 3)),
                network_share=round(float((~np.isnan(gains)).mean()), 3),
                blocks_plain_vs_learned=blocks)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None,
                    help="timed steps from the initial conditions (default: the workload's "
                         "configured length, 300 for the combined set)")
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="combined", choices=["combined"] + sorted(WORKLOADS))
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU-oracle baseline")
    ap.add_argument("--cpu-budget", type=float, default=20.0,
                    help="seconds of oracle work for a single-instance workload")
    ap.add_argument("--no-kernel-timing", action="store_true")
    ap.add_argument("--extras", action="store_true", help="also run the other comparisons")
    ap.add_argument("--per-step", action="store_true",
                    help="instead of the bench: per-step iterations of the combined set's FCH instances, "
                         "extrapolated vs learned guess")
    ap.add_argument("--no-learned", action="store_true",
                    help="combined set: no network (headline = batched; counter runs)")
    ap.add_argument("--only", choices=["plain", "batched", "learned"],
                    help="combined set: run this variant besides the headline batched_learned "
                         "(profiling runs)")
    ap.add_argument("--learned-epochs", type=int, default=8)
    ap.add_argument("--learned3d-epochs", type=int, default=6,
                    help="epochs of the PFC 192^3 network in the extras (0 skips it)")
    ap.add_argument("--tune-file", default=os.path.join(ROOT, "paper_2204_07247_amd", "tune_mi355x.txt"),
                    help="plan choices of the autotuner to reuse (PFCH_TUNE_FILE; an already set "
                         "environment variable wins; '' times every plan afresh)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="before the run, copy a MIB-sized float64 buffer three times "
                         "(a plain copy kernel of known traffic for counter calibration)")
    args = ap.parse_args()
    if args.steps is None:
        args.steps = COMBINED_STEPS if args.workload == "combined" else WORKLOADS[args.workload].steps
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for {args.gpus}): the library runs on one "
              "device; independent instances would shard across GPUs with no communication, "
              "which is not implemented", file=sys.stderr)
        sys.exit(2)
    if args.per_step:
        if args.tune_file and "PFCH_TUNE_FILE" not in os.environ:
            os.environ["PFCH_TUNE_FILE"] = args.tune_file
        print(json.dumps(per_step_comparison(args)), flush=True)
        return
    # the CPU baseline first, before anything touches the GPU (its workers are forked)
    cpu = None
    if not args.no_cpu and args.workload == "combined":
        log("[bench] CPU oracle baseline: first step of every instance, one process each")
        cpu = cpu_baseline_set(combined_set())
    if args.tune_file and "PFCH_TUNE_FILE" not in os.environ:
        os.environ["PFCH_TUNE_FILE"] = args.tune_file
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
    if args.workload == "combined":
        res = combined_bench(args)
    else:
        w = WORKLOADS[args.workload]
        res = single_bench(args, w)
        if not args.no_cpu:
            log("[bench] CPU oracle baseline")
            cpu = cpu_baseline(w, w.steps, args.cpu_budget)
    if os.environ.get("PFCH_TUNE_FILE"):
        res["config"]["tune_file"] = os.path.relpath(os.environ["PFCH_TUNE_FILE"], ROOT)
    out = dict(metric=METRIC, value=res.pop("value"), unit="time-steps/s", n_gpus=1, steps=args.steps,
               warmup=args.warmup, ms_per_step=res.pop("ms_per_step"), higher_is_better=True,
               scaling="weak", vs_baseline=None, dtype="f64", data="synthetic")
    out.update(res)
    out["cpu_baseline"] = cpu
    if cpu:
        out["gpu_over_cpu"] = round(out["value"] / cpu["value"], 2)
    if args.extras:
        out["extras"] = extras(args)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
