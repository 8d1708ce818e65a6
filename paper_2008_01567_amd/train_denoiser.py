"""Train the 2.5D CNN denoiser of the multi-slice fusion prior agents.

The paper's agents H_xy,t, H_yz,t, H_zx,t (Sec. IV) share one 2.5D network
trained to remove additive white Gaussian noise; its training volume and
weights are not available, so the network is trained here on seeded synthetic
4D phantoms of the moving-object class.  Inputs are the five time points
t-2 .. t+2 of one noisy 2D slice (indices clamped at the ends of the
sequence), the target is the clean centre slice; slices of the xy, yz and zx
planes are mixed, and each volume's noise level is drawn from NOISE_STDS so
that one network serves a range of levels.  Training runs the library's own
BF16 matrix-core forward and backward kernels and Adam (msf_cnn_train_step).

    python -m paper_2008_01567_amd.train_denoiser     # 24 volumes, 4000 steps of 48 crops of 48^2: ~11 s

writes weights/denoiser25.npz (the shipped weights were made by this command).

Seeds: training volume s uses phantom seed base 60000 + s, held-out
evaluation volumes 70000 + s.
"""
from __future__ import annotations

import argparse
import dataclasses
import json
import math
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
NOISE_STDS = (0.002, 0.004, 0.008)   # attenuation units; object values are 0.01-0.05
C_IN, C_OUT = 0.05, 0.005


def weights_path() -> str:
    return os.path.join(HERE, "weights", "denoiser25.npz")


def init_params(seed: int) -> np.ndarray:
    """He-normal 3x3 weights (5 -> 16 -> 16 -> 16 -> 1), zero biases, small last layer; flat FP32 [5521]."""
    rng = np.random.default_rng(seed)
    chans = (5, 16, 16, 16, 1)
    out = []
    for li in range(4):
        ci, co = chans[li], chans[li + 1]
        std = math.sqrt(2.0 / (9 * ci)) * (0.1 if li == 3 else 1.0)
        out.append((rng.standard_normal((co, ci, 3, 3)) * std).reshape(-1))
        out.append(np.zeros(co))
    return np.concatenate(out).astype(np.float32)


def volume_config(seed_base: int):
    from paper_2008_01567_amd import synth
    return dataclasses.replace(synth.config("c5s"), cid=seed_base, n=(64, 64, 48), n_frames=8, supersample=2)


def plane_sequence(a, plane):
    """[T][Z][Y][X] -> the plane's images [T][n_slices][h][w] (xy, yz, zx)."""
    if plane == 1:
        return a
    if plane == 2:
        return a.permute(0, 3, 1, 2).contiguous()
    return a.permute(0, 2, 1, 3).contiguous()


def stacks(seq, t_idx, s_idx):
    """[T][S][h][w] -> [n][5][h][w]: slices s_idx at times t_idx - 2 .. t_idx + 2 (clamped)."""
    import torch
    T = seq.shape[0]
    chans = [seq[torch.clamp(t_idx + d, 0, T - 1), s_idx] for d in (-2, -1, 0, 1, 2)]
    return torch.stack(chans, dim=1)


def make_volume(seed_base, noise_std, dev, rng):
    """(noisy, clean) [T][Z][Y][X] on the device."""
    import torch
    from paper_2008_01567_amd import synth
    cfg = volume_config(seed_base)
    x = torch.from_numpy(synth.make_phantom(cfg, dtype=np.float32)).to(dev)
    noise = torch.from_numpy(rng.standard_normal(tuple(x.shape)).astype(np.float32) * noise_std).to(dev)
    return x + noise, x


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--volumes", type=int, default=24)
    ap.add_argument("--eval", type=int, default=2)
    ap.add_argument("--steps", type=int, default=4000)
    ap.add_argument("--batch", type=int, default=48)
    ap.add_argument("--crop", type=int, default=48)
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--out", default=None)
    args = ap.parse_args(argv)

    import torch
    from paper_2008_01567_amd import msf
    dev = torch.device("cuda:0")
    log = lambda *a: print(*a, flush=True)
    rng = np.random.default_rng(11)

    # ---- the plane sequences of every training volume
    t0 = time.perf_counter()
    noisy_seqs, clean_seqs = [], []
    for s in range(args.volumes):
        noisy, clean = make_volume(60000 + s, NOISE_STDS[s % len(NOISE_STDS)], dev, rng)
        for plane in (1, 2, 3):
            noisy_seqs.append(plane_sequence(noisy, plane))
            clean_seqs.append(plane_sequence(clean, plane))
    log("made %d volumes in %.0fs" % (args.volumes, time.perf_counter() - t0))
    net = msf.Denoiser(init_params(3), (C_IN, C_OUT))
    history = []
    t1 = time.perf_counter()
    for step in range(args.steps):
        # one sequence per step (all crops of a batch share the image size)
        k = int(rng.integers(0, len(noisy_seqs)))
        seq, cl = noisy_seqs[k], clean_seqs[k]
        T, S, h, w = seq.shape
        ch, cw = min(args.crop, h), min(args.crop, w)
        t_idx = torch.from_numpy(rng.integers(0, T, args.batch)).to(dev)
        s_idx = torch.from_numpy(rng.integers(0, S, args.batch)).to(dev)
        a, b = int(rng.integers(0, h - ch + 1)), int(rng.integers(0, w - cw + 1))
        inp = stacks(seq, t_idx, s_idx)[:, :, a:a + ch, b:b + cw].contiguous()
        tgt = cl[t_idx, s_idx][:, a:a + ch, b:b + cw].contiguous()
        lr = args.lr * 0.5 * (1.0 + math.cos(math.pi * step / args.steps)) + 1e-5
        loss, _ = net.train_step(inp, tgt, lr=lr)
        history.append(loss)
        if step % 250 == 0 or step == args.steps - 1:
            log("step %d loss %.3e  lr %.2e  %.1fs" % (step, loss, lr, time.perf_counter() - t1))

    # ---- held-out evaluation: mean squared error of the slices before and after, per plane and noise level
    evals = []
    for s in range(args.eval):
        for std in NOISE_STDS:
            noisy, clean = make_volume(70000 + s, std, dev, rng)
            for plane in (1, 2, 3):
                out = net.agent(noisy, plane)
                before = float((noisy - clean).pow(2).mean())
                after = float((out - clean).pow(2).mean())
                evals.append({"seed": 70000 + s, "noise_std": std, "plane": plane, "mse_noisy": before,
                              "mse_denoised": after})
                log("eval seed %d std %.3f plane %d: mse %.3e -> %.3e" % (70000 + s, std, plane, before, after))
    out = args.out or weights_path()
    os.makedirs(os.path.dirname(os.path.abspath(out)), exist_ok=True)
    meta = {"volumes": args.volumes, "steps": args.steps, "batch": args.batch, "crop": args.crop, "lr": args.lr,
            "noise_stds": list(NOISE_STDS), "first_loss": float(np.mean(history[:20])),
            "final_loss": float(np.mean(history[-20:])), "eval": evals, "scales": [C_IN, C_OUT]}
    np.savez(out, params=net.params(), scales=np.asarray((C_IN, C_OUT), dtype=np.float32), meta=json.dumps(meta))
    log("saved", out)
    return 0


def load(path=None):
    """(params FP32 [5521], scales (c_in, c_o), meta) of a trained denoiser."""
    z = np.load(path or weights_path(), allow_pickle=False)
    return z["params"], tuple(float(x) for x in z["scales"]), json.loads(str(z["meta"]))


if __name__ == "__main__":
    sys.exit(main())
