"""Time the projector pair on one workload's geometry, outside the solver:

    python -m paper_2008_01567_amd.time_projector [--config c5] [--tiles 3,4,2,0] [--reps 3]

Runs msf_project (y = A x) and msf_backproject (x = A^T y) on a synthetic
phantom of the workload, after one untimed call each, and prints the mean
time per call (HIP events on the current stream).  Both calls include the
public <-> internal layout transposes; a kernel trace separates those from the
projector kernels.  --tiles sets the launch shape (rays per lane, waves per
group, adjoint mode, XCD remap); without it the plan's default shape is used.
"""
from __future__ import annotations

import argparse
import sys

import numpy as np


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--config", default="c2")
    ap.add_argument("--tiles", default=None)
    ap.add_argument("--reps", type=int, default=3)
    args = ap.parse_args(argv)
    import torch
    from paper_2008_01567_amd import msf, synth
    cfg = synth.config(args.config)
    geom = synth.make_geometry(cfg)
    plan = msf.Plan(geom)
    if args.tiles:
        r, w, b, xr = (int(t) for t in args.tiles.split(","))
        plan.set_tiles(rays_per_lane=r, waves_per_group=w, back_mode=b, xcd_remap=xr)
    x = torch.from_numpy(synth.make_phantom(cfg, dtype=np.float32)).cuda()
    y = plan.project(x)
    xb = plan.backproject(y)
    for name, call in (("project", lambda: plan.project(x, y)), ("backproject", lambda: plan.backproject(y, xb))):
        call()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(args.reps):
            call()
        e1.record()
        torch.cuda.synchronize()
        print("%s, %s %dx%dx%d x %d frames, tiles %s: %.2f ms per call" %
              (name, args.config, geom.nx, geom.ny, geom.nz, geom.n_frames, plan.get_tiles(),
               e0.elapsed_time(e1) / args.reps), flush=True)
    plan.close()
    return 0


if __name__ == "__main__":
    sys.exit(main())
