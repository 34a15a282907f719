"""Helpers shared by the GPU parity tests: oracle runs and library runs on
the same seeded inputs."""
import numpy as np

from oracle import driver as odriver
from oracle import models as omodels
from oracle import pagd as opagd
from oracle import schemes as oschemes
from oracle import spectral as ospectral


def oracle_sim(w, **over):
    g = ospectral.Grid(w.shape, w.lengths)
    m = omodels.make_model(w.model, **w.params())
    kw = dict(s=w.s, etas=w.etas, tol=w.tol, max_iter=w.max_iter, mobility=w.mobility)
    kw.update(over)
    return g, m, odriver.Simulation(g, m, w.scheme, **kw)


def oracle_run(w, u0, nsteps, **over):
    """Fixed-step oracle run; returns (final u, per-step iteration counts)."""
    _, _, sim = oracle_sim(w, **over)
    out = sim.run(u0, w.dt, nsteps)
    assert out["status"] == opagd.OK, out["status"]
    return out["u"], out["iters"]


def desc_for(w, **over):
    from paper_2204_07247_amd import pfch
    kw = dict(eps=w.eps, eta1=w.eta1, eta2=w.eta2, tau=w.tau, mobility=w.mobility, s=w.s,
              etas=w.etas, tol=w.tol, max_iter=w.max_iter)
    kw.update(over)
    return pfch.make_desc(w.model, w.scheme, w.shape, w.lengths, **kw)


def rel_l2(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))
