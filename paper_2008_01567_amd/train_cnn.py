"""Train the warm-start network on triples that the plain batched solver makes.

For a scan geometry (a workload of ``synth.CONFIGS``), seeded problems are
generated (phantom, noisy measurement, v); the library computes the network's
residual feature g (msf_prox_features) and the target x* = F(v) by plain
batched CG; the network is trained by the library's own BF16 matrix-core
forward/backward kernels and Adam (msf_cnn_train_step) on random 64^3 crops;
finally CG iterations to the frozen tolerance are compared from v and from the
network's start on held-out seeds.

    python -m paper_2008_01567_amd.train_cnn --config c4 --problems 125 --steps 600

Seeds: problem s of training uses phantom/noise seed base 40000 + s, held-out
evaluation problems 50000 + s (never used for training).
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
N_PARAMS = 15169
CHANNELS = (2, 16, 16, 16, 1)
V_SCALE = 0.05           # attenuation scale of the phantoms (mu <= 0.05 per voxel)


def weights_path(config: str) -> str:
    return os.path.join(HERE, "weights", "warmstart_%s.npz" % config)


def init_params(seed: int) -> np.ndarray:
    """He-normal weights, zero biases, small last layer (the start is v)."""
    rng = np.random.default_rng(seed)
    out = []
    for li in range(4):
        ci, co = CHANNELS[li], CHANNELS[li + 1]
        std = math.sqrt(2.0 / (27 * ci)) * (0.1 if li == 3 else 1.0)
        out.append((rng.standard_normal((co, ci, 3, 3, 3)) * std).reshape(-1))
        out.append(np.zeros(co))
    return np.concatenate(out).astype(np.float32)


def make_problem(cfg, geom, plan, seed_base, dev):
    """(v, y, lam) on the device for one seeded problem of the geometry."""
    import torch
    from paper_2008_01567_amd import synth
    c = dataclasses.replace(cfg, cid=seed_base)
    x0 = synth.make_phantom(c, dtype=np.float32)
    v = synth.make_v(c, x0.astype(np.float64)).astype(np.float32)
    yc = plan.project(torch.from_numpy(x0).to(dev)).cpu().numpy()
    eps = synth.noise_eps(c, geom, dtype=np.float32)
    y, lam = synth.finish_measurement(yc, eps, synth.frame_counts(geom), geom.n_rays_per_view, dtype=np.float32,
                                      model=c.weights)
    return torch.from_numpy(v).to(dev), torch.from_numpy(y).to(dev), torch.from_numpy(lam).to(dev)


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--config", default="c4")
    ap.add_argument("--problems", type=int, default=125)
    ap.add_argument("--eval", type=int, default=2)
    ap.add_argument("--steps", type=int, default=600)
    ap.add_argument("--batch", type=int, default=4)
    ap.add_argument("--crop", type=int, default=64)
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--target-tol", type=float, default=1e-7)
    ap.add_argument("--out", default=None)
    args = ap.parse_args(argv)

    import torch
    from paper_2008_01567_amd import msf, synth
    from paper_2008_01567_amd.calibration import FROZEN_TOL

    dev = torch.device("cuda:0")
    cfg = synth.config(args.config)
    geom = synth.make_geometry(cfg)
    plan = msf.Plan(geom)
    log = lambda *a: print(*a, flush=True)

    # ---- training triples (v, g, x*) made by the plain solver
    t0 = time.perf_counter()
    V, G, T = [], [], []
    iters = []
    for s in range(args.problems):
        v, y, lam = make_problem(cfg, geom, plan, 40000 + s, dev)
        if geom.n_vox >= 1 << 24:
            log("problem %d/%d: inputs ready (%.0fs)" % (s, args.problems, time.perf_counter() - t0))
        g = plan.features(v, y, lam, cfg.sigma)
        x, st = plan.prox_solve(v, y, lam, cfg.sigma, tol=args.target_tol, max_iter=4000, check_every=16)
        V.append(v)
        G.append(g)
        T.append(x.clone())
        iters.append(int(st["iters"].max()))
        if s % 10 == 0 or geom.n_vox >= 1 << 24:
            log("problem %d/%d: target CG iterations %s (%.0fs)" % (s, args.problems, st["iters"].max(),
                                                                       time.perf_counter() - t0))
    V, G, T = torch.cat(V), torch.cat(G), torch.cat(T)      # [frames][nz][ny][nx]
    nfr = V.shape[0]
    log("made %d frame triples in %.0fs" % (nfr, time.perf_counter() - t0))

    # ---- scales: unit-RMS feature and correction over the training set
    sample = range(0, nfr, max(nfr // 64, 1))
    g_scale = float(np.sqrt(np.mean([G[f].pow(2).mean().item() for f in sample])))
    o_scale = float(np.sqrt(np.mean([(T[f] - V[f]).pow(2).mean().item() for f in sample])))
    scales = (V_SCALE, g_scale, o_scale)
    log("scales: v %.3g  g %.3g  (x* - v) %.3g" % scales)

    # ---- training on random crops
    rng = np.random.default_rng(7)
    net = msf.Cnn(init_params(1), scales)
    cz, cy, cx = (min(args.crop, n) for n in (geom.nz, geom.ny, geom.nx))
    history = []
    t1 = time.perf_counter()
    for step in range(args.steps):
        fr = rng.integers(0, nfr, args.batch)
        oz = rng.integers(0, geom.nz - cz + 1, args.batch)
        oy = rng.integers(0, geom.ny - cy + 1, args.batch)
        ox = rng.integers(0, geom.nx - cx + 1, args.batch)
        crop = lambda A: torch.stack([A[f, a:a + cz, b:b + cy, c:c + cx] for f, a, b, c in zip(fr, oz, oy, ox)]).contiguous()
        lr = args.lr * 0.5 * (1.0 + math.cos(math.pi * step / args.steps)) + 1e-5
        cv, cg, ct = crop(V), crop(G), crop(T)
        loss, _ = net.train_step(cv, cg, ct, lr=lr)
        history.append(loss)
        if step % 100 == 0 or step == args.steps - 1:
            base_b = (ct - cv).pow(2).mean().item()
            log("step %d loss %.4e  (start x0 = v: %.4e)  lr %.2e  %.1fs" % (step, loss, base_b, lr,
                                                                              time.perf_counter() - t1))
    # loss of the plain start v (x0 = v) on the same kind of crops, for reference
    base = float(np.mean([(T[f] - V[f]).pow(2).mean().item() for f in range(0, nfr, max(nfr // 32, 1))]))

    # ---- held-out evaluation: CG iterations to the frozen tolerance from v and from the network
    tol = FROZEN_TOL.get(args.config, cfg.tol)
    evals = []
    for s in range(args.eval):
        log("evaluation problem %d: generating inputs" % s)
        v, y, lam = make_problem(cfg, geom, plan, 50000 + s, dev)
        _, sp = plan.prox_solve(v, y, lam, cfg.sigma, tol=tol, max_iter=6000, check_every=16)
        _, sl = plan.prox_solve(v, y, lam, cfg.sigma, tol=tol, max_iter=6000, check_every=16, cnn=net)
        evals.append({"seed": 50000 + s, "iters_plain": sp["iters"].tolist(), "iters_learned": sl["iters"].tolist(),
                      "seconds_plain": sp["seconds"], "seconds_learned": sl["seconds"],
                      "cnn_used": int(sl["cnn_used"].sum()),
                      "start_residual_plain": float(np.mean(sp["start_rel_residual"])),
                      "start_residual_learned": float(np.mean(sl["start_rel_residual"]))})
        log("eval seed %d: mean iters plain %.1f learned %.1f; time %.3fs vs %.3fs; kept %d/%d; "
            "start residual %.3e -> %.3e" %
            (50000 + s, np.mean(sp["iters"]), np.mean(sl["iters"]), sp["seconds"], sl["seconds"],
             sl["cnn_used"].sum(), geom.n_frames, np.mean(sp["start_rel_residual"]),
             np.mean(sl["start_rel_residual"])))

    out = args.out or weights_path(args.config)
    os.makedirs(os.path.dirname(out), exist_ok=True)
    meta = {"config": args.config, "problems": args.problems, "frames": int(nfr), "steps": args.steps,
            "batch": args.batch, "crop": [cz, cy, cx], "lr": args.lr, "target_tol": args.target_tol,
            "final_loss": float(np.mean(history[-20:])), "loss_of_v": base, "target_iters_max": max(iters),
            "eval": evals, "scales": list(scales)}
    np.savez(out, params=net.params(), scales=np.asarray(scales, dtype=np.float32), meta=json.dumps(meta))
    log("saved", out, json.dumps(meta))


def load(config: str):
    """(params FP32 [15169], scales (c_v, c_g, c_o), meta dict) of a trained network."""
    z = np.load(weights_path(config), allow_pickle=False)
    return z["params"], tuple(float(x) for x in z["scales"]), json.loads(str(z["meta"]))


if __name__ == "__main__":
    sys.exit(main())
