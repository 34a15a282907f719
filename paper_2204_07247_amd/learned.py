"""Learned initial guess: training data from the solver itself, training of
the float32 FNO through its C entry points, and deployment on a context.

The network predicts the correction of the extrapolated guess
u^n + rho (u^n - u^{n-1}) (Alg. 2 input x_0) from (u^n, u^{n-1}).  Every
arithmetic step (solver steps, input preparation, forward, backward, Adam)
runs in libpfch; this module only orders the calls, draws minibatch
permutations and moves arrays.
"""
import dataclasses

import numpy as np

from . import pfch


@dataclasses.dataclass
class TrainConfig:
    width: int = 32
    modes: int = 16
    layers: int = 4
    batch: int = 16
    epochs: int = 8
    lr: float = 1e-3
    holdout: float = 0.1
    seed: int = 0
    # the network's own grid; None: the trajectories' grid.  A coarser 2D
    # grid (e.g. 4 * modes per axis) trains and runs the network on the
    # band-limited part of the fields sampled there
    grid: tuple = None


@dataclasses.dataclass
class Trained:
    fno: "pfch.Fno"
    norm: tuple          # (mu, su, sd, so)
    train_loss: list     # mean minibatch loss per epoch
    val_loss: list       # held-out loss per epoch
    n_train: int
    n_val: int


def desc_of(w, guess=0):
    return pfch.make_desc(w.model, w.scheme, w.shape, w.lengths, eps=w.eps, eta1=w.eta1,
                          eta2=w.eta2, tau=w.tau, mobility=w.mobility, s=w.s, etas=w.etas,
                          tol=w.tol, max_iter=w.max_iter, guess=guess)


def trajectories(ws, u0s, steps):
    """Advance the instances `ws` (one batched context) `steps` plain steps
    from u0s; returns a float64 GPU tensor [len(ws)][steps + 1][*grid]."""
    import torch
    shape = tuple(ws[0].shape)
    out = torch.empty((len(ws), steps + 1) + shape, dtype=torch.float64, device="cuda")
    ctx = pfch.Context([desc_of(w) for w in ws])
    ctx.set_stats_detail(0)
    for i, u in enumerate(u0s):
        out[i, 0].copy_(u)
        ctx.set_state(i, out[i, 0])
    for n in range(steps):
        rc, _ = ctx.step([w.dt for w in ws])
        if rc != pfch.PFCH_OK:
            raise RuntimeError(f"trajectory step {n} failed: {pfch.strerror(rc)}")
        for i in range(len(ws)):
            ctx.get_state(i, out[i, n + 1])
    ctx.close()
    return out


def normalisation(states):
    """(mu, su, sd, so) from the host copy of a subsample of the states:
    mean and spread of u^n, of u^n - u^{n-1} and of the target correction
    u^{n+1} - 2u^n + u^{n-1} (constant step)."""
    s = states[:, ::2].cpu().numpy() if states.shape[1] > 8 else states.cpu().numpy()
    u = s[:, 1:-1]
    d = s[:, 1:-1] - s[:, :-2]
    c = s[:, 2:] - 2 * s[:, 1:-1] + s[:, :-2]
    sd = float(d.std()) or 1.0
    return (float(u.mean()), float(u.std()) or 1.0, sd, float(c.std()) or sd)


def dataset(fno, states, norm, rho=1.0):
    """Network inputs X [N][2][*grid] and targets T [N][*grid] (float32,
    GPU, on the network's grid) for every triple (u^{n-1}, u^n, u^{n+1}) of
    the trajectories."""
    import torch
    ni, nt = states.shape[:2]
    grid = tuple(fno.shape)
    n = ni * (nt - 2)
    X = torch.empty((n, 2) + grid, dtype=torch.float32, device="cuda")
    T = torch.empty((n,) + grid, dtype=torch.float32, device="cuda")
    k = 0
    for i in range(ni):
        for j in range(1, nt - 1):
            fno.prepare(states[i, j - 1], states[i, j], states[i, j + 1], rho, norm, X[k], T[k])
            k += 1
    return X, T


def train(ws, u0s, steps, cfg=TrainConfig(), log=None):
    """Generate trajectories of the instances `ws` with the solver, then
    train an FNO on their triples; returns a Trained record."""
    import torch
    states = trajectories(ws, u0s, steps)
    norm = normalisation(states)
    fno = pfch.Fno(cfg.width, cfg.modes, cfg.layers, *(cfg.grid or ws[0].shape), max_batch=cfg.batch)
    fno.init_params(cfg.seed)
    X, T = dataset(fno, states, norm)
    del states
    n = X.shape[0]
    rng = np.random.default_rng(cfg.seed)
    perm = rng.permutation(n)
    n_val = max(1, int(round(cfg.holdout * n)))
    val_idx, tr_idx = perm[:n_val], perm[n_val:]
    Xv = X[torch.from_numpy(val_idx).cuda()].contiguous()
    Tv = T[torch.from_numpy(val_idx).cuda()].contiguous()
    step = 0
    tr_hist, val_hist = [], []
    for ep in range(cfg.epochs):
        order = rng.permutation(tr_idx)
        losses = []
        for b0 in range(0, len(order) - cfg.batch + 1, cfg.batch):
            idx = torch.from_numpy(order[b0:b0 + cfg.batch]).cuda()
            xb = X[idx].contiguous()
            tb = T[idx].contiguous()
            want = (b0 // cfg.batch) % 16 == 0
            loss, _ = fno.grad(xb, tb, want_grad=False, want_loss=want)
            if want:
                losses.append(loss)
            step += 1
            fno.adam_step(cfg.lr, step)
        vl = []
        for b0 in range(0, n_val, cfg.batch):
            xb = Xv[b0:b0 + cfg.batch].contiguous()
            tb = Tv[b0:b0 + cfg.batch].contiguous()
            loss, _ = fno.grad(xb, tb, want_grad=False)
            vl.append(loss * xb.shape[0])
        tr_hist.append(float(np.mean(losses)) if losses else float("nan"))
        val_hist.append(float(np.sum(vl) / n_val))
        if log:
            log(f"[learned] epoch {ep + 1}/{cfg.epochs}: train {tr_hist[-1]:.4g} held-out {val_hist[-1]:.4g}")
    return Trained(fno=fno, norm=norm, train_loss=tr_hist, val_loss=val_hist,
                   n_train=len(tr_idx), n_val=n_val)


def deploy(trained, *shape, cfg=TrainConfig()):
    """A copy of the trained network for another grid of the same rank (the
    weights act on mode indices and channels, so they transfer unchanged).
    A network on a coarse grid of its own needs no copy: it attaches to
    instances on any finer grid of the same periods."""
    f = pfch.Fno(cfg.width, cfg.modes, cfg.layers, *shape, max_batch=1)
    f.set_params(trained.fno.get_params())
    return f
