"""Time the three 2.5D denoiser agents (msf_denoise25, shipped weights) on the
128^3 x 16 benchmark volume (a synthetic phantom plus noise):

    python -m paper_2008_01567_amd.time_agents [--reps 5]

Prints the mean time per call of each plane's agent, measured with HIP events
on the current stream after one untimed call.
"""
from __future__ import annotations

import argparse
import sys

import numpy as np


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--reps", type=int, default=5)
    ap.add_argument("--config", default="c2")
    args = ap.parse_args(argv)
    import torch
    from paper_2008_01567_amd import msf, synth, train_denoiser
    params, scales, _ = train_denoiser.load()
    net = msf.Denoiser(params, scales)
    cfg = synth.config(args.config)
    w = torch.from_numpy(synth.make_phantom(cfg, dtype=np.float32)).cuda()
    w += 0.004 * torch.randn_like(w)
    out = torch.empty_like(w)
    T, nz, ny, nx = w.shape
    for plane in (1, 2, 3):
        net.agent(w, plane, out=out)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(args.reps):
            net.agent(w, plane, out=out)
        e1.record()
        torch.cuda.synchronize()
        print("agent plane %d on %dx%dx%d x %d: %.2f ms" % (plane, nx, ny, nz, T, e0.elapsed_time(e1) / args.reps),
              flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
