#!/usr/bin/env python3
"""Benchmark of the batched forward-model proximal map on one MI355X.

One step = one call of the whole hot path on one batch: the proximal map of
the data term (paper eq. (4)) for all 16 frames of the 128^3 x 16
workload (192^2 detector, 16 interlaced views per frame over 360 degrees),
solved by the HIP library's batched CG to the frozen stopping rule, started
from the trained network's prediction (learned + batched; the network's
evaluation and the residual checks of its start are inside the step).  The
same step started from v (plain batched CG) is timed beside it.  Inputs are
resident in HBM before the timed region starts.

Prints ONE JSON line.  Metric: voxel.views per second of solved proximal maps
(sum over frames of voxels x views, divided by the wall time of the solve).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "prox-map voxel·views/s at 1e-4 rel err: learned+batched vs plain CG; HBM GB/s"
# ALU peak of the projector kernels: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz =
# 39.3 T lane-instructions/s, i.e. 78.6 TFLOP/s of non-packed FP32 (or FP64)
# FMA.  The published 157.3 TFLOP/s FP32 figure needs packed dual-FP32
# instructions, which the library is built without.
PEAK_ALU_TFLOPS = 78.6
PEAK_HBM_GBS = 8000.0

# HBM bytes per launch of the dominant kernel from rocprofv3 FETCH_SIZE and
# WRITE_SIZE (two passes over one plain solve of the 128^3 x 16 workload,
# launch shape 3,1,2,1), each scaled by what the same counter reads for the
# library's plain copy kernel of known size in the same run (read x2.0, write
# x1.0).  Valid only for the projector source they were taken on.
MEASURED_TRAFFIC = {
    "source_sha256": "47cf8e99ddf3b6692d3891c6ae5ff5b941d05a367604fbbdf3ae7a39c218c0c9",
    "config": "c2", "tiles": {"rays_per_lane": 3, "waves_per_group": 1, "back_mode": 2, "xcd_remap": 1},
    "kernel": "backprojector k_back_gather (cell table)", "bytes_per_launch": 1252.4e6,
    "read_bytes": 987.4e6, "write_bytes": 265.0e6, "l2_hit_rate": 0.933,
    # SQ_INSTS_VALU x 64 / nnz(A) of the same runs: VALU lane-instructions per intersection
    "valu_lane_instr_per_intersection": 34.8,
    "profile": "profiles/gather_update_c2_128x16_counters.md",
}



def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", default="c2")
    ap.add_argument("--tol", type=float, default=None)
    ap.add_argument("--max-iter", type=int, default=6000)
    ap.add_argument("--check-every", type=int, default=16)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-agents", action="store_true", help="skip timing the 2.5D denoiser agents")
    ap.add_argument("--no-learned", action="store_true", help="time plain batched CG only")
    ap.add_argument("--cpu-iters", type=int, default=40, help="FP64 CG iterations timed in the CPU sample")
    ap.add_argument("--tiles", default="", help="rays_per_lane,waves_per_group,back_mode,xcd_remap (default: autotune)")
    ap.add_argument("--no-autotune", action="store_true", help="keep the plan's default launch shape")
    return ap.parse_args()


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def cpu_baseline(cfg, geom, v_np, y_np, lam_np, gpu_iters, n_iter):
    """The FP64 oracle on a bounded sample: frame 0 of the same workload, CSR
    build + transpose + n_iter CG iterations, scaled to the iteration count the
    GPU needed for that frame."""
    import numpy as np
    import oracle
    g0 = geom.subset([0])
    s0 = geom.sino_slice(0)
    t0 = time.perf_counter()
    M = oracle.FrameMatrix(g0, 0)
    M._transpose()
    t_build = time.perf_counter() - t0
    t0 = time.perf_counter()
    _, st = M.prox_cg(v_np[0].astype(np.float64), y_np[s0].astype(np.float64), lam_np[s0].astype(np.float64),
                      cfg.sigma, tol=0.0, max_iter=n_iter)
    t_cg = time.perf_counter() - t0
    per_iter = t_cg / max(n_iter, 1)
    t_frame = t_build + per_iter * gpu_iters
    vv = g0.n_vox * g0.views_of(0)
    return {"value": vv / t_frame, "unit": "voxel·views/s", "cores": oracle.num_threads(), "kind": "oracle",
            "sample": "frame 0 of the same batch (%d^3 voxels x %d views, nnz %d): FP64 CSR build %.2fs + "
                      "%d FP64 CG iterations timed (%.3fs/iter), scaled to the %d iterations the GPU took on "
                      "that frame" % (geom.nx, g0.views_of(0), M.nnz, t_build, n_iter, per_iter, gpu_iters)}


def time_agents(msf, torch, w, dev, reps=5):
    """The three 2.5D denoiser agents (shipped weights) on the solved volume:
    mean ms per call (HIP events on the current stream) and the fraction of
    the HBM roofline for their algorithmic bytes (204 B per voxel in the xy
    plane, 220 B with the two transposes of the yz and zx planes)."""
    from paper_2008_01567_amd import train_denoiser
    params, scales, _ = train_denoiser.load()
    net = msf.Denoiser(params, scales)
    out = torch.empty_like(w)
    res = {}
    for plane, name, bpv in ((1, "xy", 204.0), (2, "yz", 220.0), (3, "zx", 220.0)):
        net.agent(w, plane, out=out)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            net.agent(w, plane, out=out)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        gbs = bpv * w.numel() / (ms * 1e-3) / 1e9
        res[name] = {"ms": ms, "hbm_gbs": gbs, "frac": gbs / PEAK_HBM_GBS}
    res["bytes_per_voxel"] = {"xy": 204, "yz": 220, "zx": 220}
    net.close()
    return res


def main():
    args = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py: the library runs on one GPU; the proximal map shards by frame across GPUs "
              "(design only), so --gpus %d is not supported" % max(args.gpus, world), file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2008_01567_amd import msf, synth
    from paper_2008_01567_amd.calibration import FROZEN_TOL

    dev = torch.device("cuda:0")
    cfg = synth.config(args.config)
    geom = synth.make_geometry(cfg)
    tol = args.tol if args.tol is not None else FROZEN_TOL.get(args.config, cfg.tol)
    t0 = time.perf_counter()
    x0 = synth.make_phantom(cfg, dtype=np.float32)
    v_np = synth.make_v(cfg, x0.astype(np.float64)).astype(np.float32)
    plan = msf.Plan(geom)
    if args.tiles:
        r, w, b, xr = (int(t) for t in args.tiles.split(","))
        plan.set_tiles(rays_per_lane=r, waves_per_group=w, back_mode=b, xcd_remap=xr)
    elif not args.no_autotune:
        t1 = time.perf_counter()
        log("autotune: %s (%.1fs)" % (plan.autotune(), time.perf_counter() - t1))
    y_clean = plan.project(torch.from_numpy(x0).to(dev)).cpu().numpy()
    eps = synth.noise_eps(cfg, geom, dtype=np.float32)
    y_np, lam_np = synth.finish_measurement(y_clean, eps, synth.frame_counts(geom), geom.n_rays_per_view,
                                            dtype=np.float32, model=cfg.weights)
    v = torch.from_numpy(v_np).to(dev)
    y = torch.from_numpy(y_np).to(dev)
    lam = torch.from_numpy(lam_np).to(dev)
    out = torch.empty_like(v)
    nnz = plan.count_intersections()
    log("setup %.1fs, nnz per frame %s" % (time.perf_counter() - t0, nnz[:4].tolist()))

    net = None
    if not args.no_learned:
        try:
            from paper_2008_01567_amd import train_cnn
            params, scales, meta = train_cnn.load(args.config)
            net = msf.Cnn(params, scales)
            log("warm-start network: trained on %d frames of %s" % (meta["frames"], meta["config"]))
        except FileNotFoundError:
            log("no trained warm-start network for %s: learned leg skipped" % args.config)

    def solve(cnn=None):
        return plan.prox_solve(v, y, lam, cfg.sigma, tol=tol, max_iter=args.max_iter,
                               check_every=args.check_every, use_graph=True, out=out, cnn=cnn)

    def timed(cnn):
        for i in range(args.warmup):
            _, st = solve(cnn)
            log("warmup %d (%s): iters %s steps %d %.3fs" % (i, "learned" if cnn else "plain", st["iters"].tolist(),
                                                            st["steps"], st["seconds"]))
        plan.set_timing(True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        stats = []
        for i in range(args.steps):
            _, st = solve(cnn)
            stats.append(st)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / max(args.steps, 1)
        log("step (%s): %.3fs, iters %s, status %d" % ("learned" if cnn else "plain", dt, stats[-1]["iters"].tolist(),
                                                       stats[-1]["status"]))
        return dt, stats[-1], plan.get_timing()

    dt_plain, st_plain, tm_plain = timed(None)
    if net is not None:
        dt, st, tm = timed(net)
    else:
        dt, st, tm = dt_plain, st_plain, tm_plain
    fwd_ms = tm["forward_ms"] / max(tm["forward_launches"], 1)
    back_ms = tm["back_ms"] / max(tm["back_launches"], 1)
    back_name = {0: "backprojector k_back_scatter", 1: "backprojector k_back_gather (on the fly)",
                 2: "backprojector k_back_gather (cell table)"}[plan.get_tiles()["back_mode"]]
    dominant, dom_ms = ("forward projector k_forward", fwd_ms) if fwd_ms >= back_ms else (back_name, back_ms)
    nnz_total = int(nnz.sum())
    flops = 2.0 * nnz_total        # one FMA per ray-voxel intersection (SpMV convention)
    achieved = flops / (dom_ms * 1e-3) / 1e12
    traffic = None
    try:
        import hashlib
        with open(os.path.join(ROOT, "paper_2008_01567_amd", "csrc", "projector.hip"), "rb") as fh:
            same_src = hashlib.sha256(fh.read()).hexdigest() == MEASURED_TRAFFIC["source_sha256"]
        if same_src and MEASURED_TRAFFIC["config"] == args.config and dominant == MEASURED_TRAFFIC["kernel"] \
                and plan.get_tiles() == MEASURED_TRAFFIC["tiles"]:
            traffic = MEASURED_TRAFFIC["bytes_per_launch"]
    except OSError:
        pass
    voxel_views = geom.voxel_views()
    value = voxel_views / dt
    result = {
        "metric": METRIC, "value": value, "unit": "voxel·views/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": dt * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "%s: prox map %dx%dx%d x %d frames, detector %dx%d, %d views/frame (%s), "
                               "sigma %.2g, stop at rel. residual %.0e" %
                               (args.config, geom.nx, geom.ny, geom.nz, geom.n_frames, geom.nu, geom.nv,
                                geom.views_of(0), cfg.schedule, cfg.sigma, tol),
                   "solver": "%s batched CG (FP32 vectors, FP64 scalars), hipGraph per %d steps" %
                             ("learned-warm-start +" if net is not None else "plain", args.check_every),
                   "tiles": plan.get_tiles()},
        "cg_iters": {"mean": float(np.mean(st["iters"])), "max": int(np.max(st["iters"]))},
        "plain_batched": {"value": voxel_views / dt_plain, "ms_per_step": dt_plain * 1e3,
                          "cg_iters_mean": float(np.mean(st_plain["iters"])),
                          "start_rel_residual": float(np.mean(st_plain["start_rel_residual"]))},
        "learned_batched": None if net is None else {
            "value": voxel_views / dt, "ms_per_step": dt * 1e3, "cg_iters_mean": float(np.mean(st["iters"])),
            "frames_kept": int(np.sum(st["cnn_used"])),
            "start_rel_residual": float(np.mean(st["start_rel_residual"]))},
        "speedup_learned_vs_plain": None if net is None else dt_plain / dt,
        "kernels_ms": {"forward": fwd_ms, "back": back_ms, "timed_launches": tm["forward_launches"]},
        "projector_voxel_views_per_s": {"forward": voxel_views / (fwd_ms * 1e-3),
                                        "back": voxel_views / (back_ms * 1e-3)},
        "nnz_A": nnz_total,
        "roofline": {"bound": "alu", "kernel": dominant, "achieved": achieved, "peak": PEAK_ALU_TFLOPS,
                     "unit": "TFLOP/s", "frac": achieved / PEAK_ALU_TFLOPS, "traffic": traffic,
                     "ms_per_launch": dom_ms,
                     "note": "2 FLOP per ray-voxel intersection (nnz of A counted by the projector); peak = "
                             "non-packed FP32 FMA rate 256 CU x 64 lanes x 2 x 2.4 GHz; traffic = HBM bytes per "
                             "launch from rocprofv3 FETCH_SIZE+WRITE_SIZE scaled by a copy kernel (null when the "
                             "kernel or launch shape differs from the profiled one)",
                     "hbm_gbs_of_traffic": None if traffic is None else traffic / (dom_ms * 1e-3) / 1e9,
                     "hbm_frac_of_traffic": None if traffic is None else
                     traffic / (dom_ms * 1e-3) / 1e9 / PEAK_HBM_GBS,
                     "l2_hit_rate": None if traffic is None else MEASURED_TRAFFIC["l2_hit_rate"],
                     # the kernel against its instruction-issue bound: the VALU lane-instructions it
                     # executes per intersection (counters) at 39.3 T lane-instructions/s, over its time
                     "issue_bound_frac": None if traffic is None else
                     nnz_total * MEASURED_TRAFFIC["valu_lane_instr_per_intersection"] / (PEAK_ALU_TFLOPS * 0.5e12)
                     / (dom_ms * 1e-3)},
    }
    if not args.no_agents:
        result["denoiser_agents"] = time_agents(msf, torch, out, dev)
    if not args.no_cpu_baseline:
        result["cpu_baseline"] = cpu_baseline(cfg, geom, v_np, y_np, lam_np, int(st_plain["iters"][0]),
                                              args.cpu_iters)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
