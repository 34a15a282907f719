"""Record the autotuner's plan choices for a set of grids in a tuning file.

    python -m paper_2204_07247_amd.tune OUT.txt

creates one context per (model, scheme, grid) of the workloads below with
PFCH_TUNE_FILE=OUT.txt: pfch_create times every transform plan and launch
geometry candidate on the device and appends its choice to the file (a
choice already in the file is reused, not timed again).  Later processes
that set PFCH_TUNE_FILE to that file run the same kernels without timing.
"""
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def grids():
    import workloads as W
    out = [W.FCH256_BDF2, W.PFC64_MP, W.PFC192_3D]
    out += W.fch_ensemble(count_per_size=1)
    out += W.pfc_ensemble(count=64)
    out.append(W.Workload(name="pfc2d_1024_mp", model="pfc", scheme="mp", shape=(1024, 1024),
                          lengths=(1024.0, 1024.0), dt=0.2, steps=1, mean=-0.25, amp=0.05, eps=0.25))
    seen, uniq = set(), []
    for w in out:
        key = (w.model, w.scheme, tuple(w.shape))
        if key not in seen:
            seen.add(key)
            uniq.append(w)
    return uniq


def main(path):
    os.environ["PFCH_TUNE_FILE"] = os.path.abspath(path)
    os.environ.pop("PFCH_AUTOTUNE", None)
    from paper_2204_07247_amd import pfch
    for w in grids():
        d = pfch.make_desc(w.model, w.scheme, w.shape, w.lengths, eps=w.eps, eta1=w.eta1, eta2=w.eta2,
                           tau=w.tau, s=w.s, etas=w.etas, tol=w.tol, max_iter=w.max_iter)
        ctx = pfch.Context([d])
        print(w.model, w.scheme, w.shape, ctx.plan(0), flush=True)
        ctx.close()


if __name__ == "__main__":
    if len(sys.argv) != 2:
        sys.exit("usage: python -m paper_2204_07247_amd.tune OUT.txt")
    main(sys.argv[1])
