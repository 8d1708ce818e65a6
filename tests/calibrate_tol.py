"""Calibrate the stopping rule of the batched CG against the FP64 oracle.

For a workload, sampled frames are solved to 1e-11 by the oracle's FP64 CG;
the GPU solves the whole batch at each candidate residual tolerance; the
relative L2 error of every sampled frame is printed.  The tolerances frozen in
paper_2008_01567_amd/calibration.py are the largest whose worst sampled error
stays at or below about 4e-5 (a 2.5x margin under the 1e-4 target).

    python tests/calibrate_tol.py c2 --frames 0 5 10 15 --tols 3e-6 5e-6 8e-6 1.2e-5
"""
from __future__ import annotations

import argparse
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(HERE))
sys.path.insert(0, HERE)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("config")
    ap.add_argument("--frames", type=int, nargs="+", default=[0])
    ap.add_argument("--tols", type=float, nargs="+", default=[3e-6])
    args = ap.parse_args()

    import torch
    import oracle
    from paper_2008_01567_amd import msf, synth
    from _problems import rel_l2

    cfg = synth.config(args.config)
    g = synth.make_geometry(cfg)
    x0 = synth.make_phantom(cfg).astype(np.float32).astype(np.float64)
    v = synth.make_v(cfg, x0).astype(np.float32).astype(np.float64)
    y, lam = oracle.make_measurement(cfg, g, x0)
    y = y.astype(np.float32).astype(np.float64)
    lam = lam.astype(np.float32).astype(np.float64)
    ref = {}
    for f in args.frames:
        t = time.perf_counter()
        s = g.sino_slice(f)
        M = oracle.FrameMatrix(g.subset([f]), 0)
        ref[f], st = M.prox_cg(v[f], y[s], lam[s], cfg.sigma, tol=1e-11, max_iter=20000)
        print("oracle frame %d: %d iterations, %.1fs" % (f, st["iters"], time.perf_counter() - t), flush=True)
    plan = msf.Plan(g)
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()
    for tol in args.tols:
        x, st = plan.prox_solve(dev(v), dev(y), dev(lam), cfg.sigma, tol=tol, max_iter=20000, check_every=16,
                                true_residual=True)
        x = x.cpu().numpy()
        errs = {f: rel_l2(x[f], ref[f]) for f in args.frames}
        print("tol %.1e: iterations mean %.1f max %d; true residual max %.2e; errors %s; "
              "worst %.2e" % (tol, np.mean(st["iters"]), np.max(st["iters"]),
                              np.max(st["true_rel_residual"]), " ".join("%d:%.2e" % kv for kv in errs.items()),
                              max(errs.values())), flush=True)


if __name__ == "__main__":
    main()
