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
# Issue rate of plain vector instructions: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz
# = 39.3 T lane-instructions/s, i.e. 78.6 TFLOP/s of non-packed FP32 (or FP64)
# FMA.  The published 157.3 TFLOP/s FP32 figure needs packed dual-FP32
# instructions, which the library is built without.
PEAK_VALU_TLANEOPS = 39.32
PEAK_FMA_TFLOPS = 78.6
PEAK_HBM_GBS = 8000.0
# Algorithmic work of one ray-voxel intersection (a nonzero of A) in the
# projector kernels: about 12 vector lane-operations (exact crossing, piece
# length, row / voxel index, the multiply-add and its share of the loop).
VALU_OPS_PER_INTERSECTION = 12

# HBM bytes per launch of the dominant kernel from rocprofv3 FETCH_SIZE and
# WRITE_SIZE (two passes over one plain solve of the 128^3 x 16 workload),
# each scaled by what the same counter reads for the library's plain copy
# kernel of known size in the same run (read x2.0, write x1.0).  Valid only
# for the projector source and launch shape they were taken on.
MEASURED_TRAFFIC = {
    "source_sha256": "61284055c580349d772911a619e07c013a897b30ebb23b51b6eb9b9d1de85100",
    "config": "c2", "tiles": {"rays_per_lane": 3, "waves_per_group": 1, "back_mode": 2, "xcd_remap": 1},
    "kernel": "backprojector k_back_gather (cell table)", "bytes_per_launch": 1252.4e6,
    "read_bytes": 987.3e6, "write_bytes": 265.1e6, "l2_hit_rate": 0.929,
    # SQ_INSTS_VALU x 64 / nnz(A) of the same runs: VALU lane-instructions per intersection
    "valu_lane_instr_per_intersection": 27.1,
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
    ap.add_argument("--large", default="c5", help="largest one-GPU workload, timed once per leg after the "
                                                    "main loop ('' to skip)")
    ap.add_argument("--cpu-1thread-iters", type=int, default=4, help="FP64 CG iterations timed on one thread")
    ap.add_argument("--tiles", default="", help="rays_per_lane,waves_per_group,back_mode,xcd_remap (default: autotune)")
    ap.add_argument("--no-autotune", action="store_true", help="keep the plan's default launch shape")
    return ap.parse_args()


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def host_cpu():
    """(nproc, CPU model name) of this host."""
    try:
        nproc = len(os.sched_getaffinity(0))
    except AttributeError:
        nproc = os.cpu_count()
    model = None
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return nproc, model


def rel_l2(a, b):
    import numpy as np
    a = np.asarray(a, dtype=np.float64).reshape(-1)
    b = np.asarray(b, dtype=np.float64).reshape(-1)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def cpu_baseline(cfg, geom, v_np, y_np, lam_np, tol, gpu_frames0, one_thread_iters):
    """The FP64 oracle on frame 0 of the same batch: its CSR matrix (built once per
    geometry, like the GPU plan; timed apart), then FP64 CG to the same stopping
    rule as the GPU, timed in full on all host threads.  A second oracle solve to
    1e-11 (not timed) is the reference for the error of the CPU result and of
    the GPU legs' frame 0 (gpu_frames0: leg name -> array).  A few iterations
    on one thread give the 1-thread rate."""
    import numpy as np
    import oracle
    g0 = geom.subset([0])
    s0 = geom.sino_slice(0)
    v0, y0, l0 = (a.astype(np.float64) for a in (v_np[0], y_np[s0], lam_np[s0]))
    threads = oracle.num_threads()
    nproc, model = host_cpu()
    t0 = time.perf_counter()
    M = oracle.FrameMatrix(g0, 0)
    M._transpose()
    t_build = time.perf_counter() - t0
    log("cpu baseline: CSR of frame 0 (nnz %d) in %.1fs" % (M.nnz, t_build))
    t0 = time.perf_counter()
    xc, st = M.prox_cg(v0, y0, l0, cfg.sigma, tol=tol, max_iter=20000)
    t_solve = time.perf_counter() - t0
    log("cpu baseline: FP64 CG to %.0e: %d iterations, %.1fs on %d threads" % (tol, st["iters"], t_solve, threads))
    xr, sr = M.prox_cg(v0, y0, l0, cfg.sigma, tol=1e-11, max_iter=40000)
    oracle.set_num_threads(1)
    try:
        t0 = time.perf_counter()
        M.prox_cg(v0, y0, l0, cfg.sigma, tol=0.0, max_iter=one_thread_iters)
        per_iter_1 = (time.perf_counter() - t0) / max(one_thread_iters, 1)
    finally:
        oracle.set_num_threads(threads)
    vv = g0.n_vox * g0.views_of(0)
    return {"value": vv / t_solve, "unit": "voxel·views/s", "cores": threads, "kind": "oracle",
            "sample": "frame 0 of the same batch (%dx%dx%d voxels x %d views, nnz %d): FP64 CG from v to the GPU's "
                      "stopping rule (rel. residual %.0e), %d iterations timed in full (%.2fs); the CSR build "
                      "(%.2fs, once per geometry like the GPU plan) is not in the rate" %
                      (geom.nx, geom.ny, geom.nz, g0.views_of(0), M.nnz, tol, st["iters"], t_solve, t_build),
            "threads": threads, "nproc": nproc, "cpu_model": model,
            "solve_s": t_solve, "iters": st["iters"], "csr_build_s": t_build,
            "per_iter_s": t_solve / max(st["iters"], 1), "per_iter_s_1thread": per_iter_1,
            "value_1thread": vv / (per_iter_1 * max(st["iters"], 1)),
            "err_vs_oracle": rel_l2(xc, xr), "reference": "FP64 CG to 1e-11 (%d iterations)" % sr["iters"],
            "gpu_err_vs_oracle_frame0": {k: rel_l2(x, xr) for k, x in gpu_frames0.items()}}


def roofline(nnz_total, geom, dom_name, dom_ms, fused_update, traffic):
    """Bound-aware fraction of the dominant kernel: its algorithmic time at the HBM
    peak (bytes it must move) and at the vector-issue peak (12 lane-ops per
    intersection), whichever is larger, over its measured time."""
    n_vox = geom.n_vox * geom.n_frames
    n_meas = geom.n_views * geom.n_rays_per_view
    if dom_name.startswith("forward"):
        alg_bytes = 4.0 * n_vox + 8.0 * n_meas                   # read p; read Lambda, write Lambda A p
    elif fused_update:
        alg_bytes = 4.0 * n_meas + 20.0 * n_vox                  # read the sinogram; p, x, r in; x, r out
    else:
        alg_bytes = 4.0 * n_meas + 8.0 * n_vox                   # read the sinogram; write the FP64 sum
    t = dom_ms * 1e-3
    t_hbm = alg_bytes / (PEAK_HBM_GBS * 1e9)
    t_valu = nnz_total * VALU_OPS_PER_INTERSECTION / (PEAK_VALU_TLANEOPS * 1e12)
    if t_valu >= t_hbm:
        rf = {"bound": "alu", "achieved": nnz_total * VALU_OPS_PER_INTERSECTION / t / 1e12,
              "peak": PEAK_VALU_TLANEOPS, "unit": "T VALU lane-ops/s"}
    else:
        rf = {"bound": "hbm", "achieved": alg_bytes / t / 1e9, "peak": PEAK_HBM_GBS, "unit": "GB/s"}
    rf["frac"] = rf["achieved"] / rf["peak"]
    rf.update({
        "traffic": traffic, "kernel": dom_name, "ms_per_launch": dom_ms,
        "algorithmic_bytes_per_launch": alg_bytes, "intersections_per_launch": nnz_total,
        "hbm_bound_ms": t_hbm * 1e3, "valu_bound_ms": t_valu * 1e3,
        "hbm_frac_algorithmic": t_hbm / t,
        "fma_tflops": 2.0 * nnz_total / t / 1e12, "fma_frac": 2.0 * nnz_total / t / 1e12 / PEAK_FMA_TFLOPS,
        "note": "frac = max(algorithmic bytes / 8 TB/s, intersections x %d VALU lane-ops / 39.32 T/s) / measured "
                "launch time (HIP events on the solver's stream); fma_* count one FMA per intersection against "
                "78.6 TFLOP/s; traffic = HBM bytes per launch from rocprofv3 FETCH_SIZE + WRITE_SIZE scaled by a "
                "copy kernel (null when the kernel source or launch shape differs from the profiled one)"
                % VALU_OPS_PER_INTERSECTION,
    })
    if traffic is not None:
        rf["hbm_gbs_of_traffic"] = traffic / t / 1e9
        rf["hbm_frac_of_traffic"] = traffic / t / 1e9 / PEAK_HBM_GBS
        rf["l2_hit_rate"] = MEASURED_TRAFFIC["l2_hit_rate"]
        rf["issue_bound_frac"] = (nnz_total * MEASURED_TRAFFIC["valu_lane_instr_per_intersection"] /
                                  (PEAK_VALU_TLANEOPS * 1e12) / t)
    return rf


def load_net(msf, config):
    from paper_2008_01567_amd import train_cnn
    try:
        params, scales, meta = train_cnn.load(config)
    except FileNotFoundError:
        log("no trained warm-start network for %s: learned leg skipped" % config)
        return None
    log("warm-start network for %s: trained on %d frames of %s" % (config, meta["frames"], meta["config"]))
    return msf.Cnn(params, scales)


def make_inputs(cfg, geom, plan, synth, torch, dev):
    """Phantom, v, and the noisy measurement (y from the library's projector) on the device."""
    import numpy as np
    x0 = synth.make_phantom(cfg, dtype=np.float32)
    v_np = synth.make_v(cfg, x0).astype(np.float32)
    xd = torch.from_numpy(x0).to(dev)
    del x0
    y_clean = plan.project(xd).cpu().numpy()
    del xd
    eps = synth.noise_eps(cfg, geom, dtype=np.float32)
    y_np, lam_np = synth.finish_measurement(y_clean, eps, synth.frame_counts(geom), geom.n_rays_per_view,
                                            dtype=np.float32, model=cfg.weights)
    return v_np, y_np, lam_np


def large_record(name, args, msf, torch, dev):
    """The largest one-GPU workload: one plain and one learned solve, each timed once
    (HIP-synchronised wall clock), after a short solve that captures the CG graph.
    Plan creation, autotuning and input generation are outside the timed region."""
    import numpy as np
    from paper_2008_01567_amd import synth
    from paper_2008_01567_amd.calibration import FROZEN_TOL
    cfg = synth.config(name)
    geom = synth.make_geometry(cfg)
    tol = FROZEN_TOL.get(name, cfg.tol)
    t0 = time.perf_counter()
    plan = msf.Plan(geom)
    t_plan = time.perf_counter() - t0
    t0 = time.perf_counter()
    tiles = plan.autotune()
    t_tune = time.perf_counter() - t0
    log("%s: plan %.1fs, autotune %s (%.1fs)" % (name, t_plan, tiles, t_tune))
    t0 = time.perf_counter()
    v_np, y_np, lam_np = make_inputs(cfg, geom, plan, synth, torch, dev)
    v = torch.from_numpy(v_np).to(dev)
    del v_np
    y = torch.from_numpy(y_np).to(dev)
    lam = torch.from_numpy(lam_np).to(dev)
    del y_np, lam_np
    out = torch.empty_like(v)
    t_inputs = time.perf_counter() - t0
    nnz = int(plan.count_intersections().sum())
    log("%s: inputs %.1fs, nnz %d" % (name, t_inputs, nnz))
    net = None if args.no_learned else load_net(msf, name)

    def solve(cnn, max_iter):
        return plan.prox_solve(v, y, lam, cfg.sigma, tol=tol, max_iter=max_iter, check_every=args.check_every,
                               use_graph=True, out=out, cnn=cnn)

    solve(None, args.check_every)          # captures the graph of check_every CG steps
    torch.cuda.synchronize()
    rec = {"workload": "%s: prox map %dx%dx%d x %d frames, detector %dx%d, %d views/frame (%s over %g deg), "
                       "sigma %.2g, stop at rel. residual %.0e" %
                       (name, geom.nx, geom.ny, geom.nz, geom.n_frames, geom.nu, geom.nv, geom.views_of(0),
                        cfg.schedule, cfg.arc_deg, cfg.sigma, tol),
           "voxel_views": geom.voxel_views(), "nnz_A": nnz, "tiles": tiles,
           "setup_s": {"plan": t_plan, "autotune": t_tune, "inputs": t_inputs}}
    legs = [("plain_batched", None)] + ([("learned_batched", net)] if net is not None else [])
    for key, cnn in legs:
        plan.set_timing(True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, st = solve(cnn, args.max_iter)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        tm = plan.get_timing()
        log("%s %s: %.2fs, iters %d-%d, status %d" % (name, key, dt, st["iters"].min(), st["iters"].max(),
                                                      st["status"]))
        rec[key] = {"value": geom.voxel_views() / dt, "seconds": dt, "status": int(st["status"]),
                    "cg_iters_mean": float(np.mean(st["iters"])), "cg_iters_max": int(np.max(st["iters"])),
                    "start_rel_residual": float(np.mean(st["start_rel_residual"])),
                    "kernels_ms": {"forward": tm["forward_ms"] / max(tm["forward_launches"], 1),
                                   "back": tm["back_ms"] / max(tm["back_launches"], 1)}}
        if cnn is not None:
            rec[key]["frames_kept"] = int(np.sum(st["cnn_used"]))
    rec["learned_batched"] = rec.get("learned_batched")
    rec["speedup_learned_vs_plain"] = (rec["plain_batched"]["seconds"] / rec["learned_batched"]["seconds"]
                                       if rec["learned_batched"] else None)
    rec["accuracy"] = "stopping rule calibrated against the FP64 oracle; frame 0 of this workload is checked " \
                      "against a full FP64 oracle solve by the test suite"
    plan.close()
    if net is not None:
        net.close()
    del v, y, lam, out
    torch.cuda.empty_cache()
    return rec


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
    plan = msf.Plan(geom)
    if args.tiles:
        r, w, b, xr = (int(t) for t in args.tiles.split(","))
        plan.set_tiles(rays_per_lane=r, waves_per_group=w, back_mode=b, xcd_remap=xr)
    elif not args.no_autotune:
        t1 = time.perf_counter()
        log("autotune: %s (%.1fs)" % (plan.autotune(), time.perf_counter() - t1))
    v_np, y_np, lam_np = make_inputs(cfg, geom, plan, synth, torch, dev)
    v = torch.from_numpy(v_np).to(dev)
    y = torch.from_numpy(y_np).to(dev)
    lam = torch.from_numpy(lam_np).to(dev)
    out = torch.empty_like(v)
    nnz = plan.count_intersections()
    log("setup %.1fs, nnz per frame %s" % (time.perf_counter() - t0, nnz[:4].tolist()))
    net = None if args.no_learned else load_net(msf, args.config)

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
    frames0 = {"plain_batched": out[0].cpu().numpy()}
    if net is not None:
        dt, st, tm = timed(net)
        frames0["learned_batched"] = out[0].cpu().numpy()
    else:
        dt, st, tm = dt_plain, st_plain, tm_plain
    fwd_ms = tm["forward_ms"] / max(tm["forward_launches"], 1)
    back_ms = tm["back_ms"] / max(tm["back_launches"], 1)
    tiles = plan.get_tiles()
    back_name = {0: "backprojector k_back_scatter", 1: "backprojector k_back_gather (on the fly)",
                 2: "backprojector k_back_gather (cell table)"}[tiles["back_mode"]]
    dominant, dom_ms = ("forward projector k_forward", fwd_ms) if fwd_ms >= back_ms else (back_name, back_ms)
    nnz_total = int(nnz.sum())
    traffic = None
    try:
        import hashlib
        with open(os.path.join(ROOT, "paper_2008_01567_amd", "csrc", "projector.hip"), "rb") as fh:
            same_src = hashlib.sha256(fh.read()).hexdigest() == MEASURED_TRAFFIC["source_sha256"]
        if same_src and MEASURED_TRAFFIC["config"] == args.config and dominant == MEASURED_TRAFFIC["kernel"] \
                and tiles == MEASURED_TRAFFIC["tiles"]:
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
                   "tiles": tiles},
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
        "roofline": roofline(nnz_total, geom, dominant, dom_ms, tiles["back_mode"] != 0, traffic),
    }
    if not args.no_agents:
        result["denoiser_agents"] = time_agents(msf, torch, out, dev)
    plan.close()
    if net is not None:
        net.close()
    del v, y, lam, out
    torch.cuda.empty_cache()
    if not args.no_cpu_baseline:
        result["cpu_baseline"] = cpu_baseline(cfg, geom, v_np, y_np, lam_np, tol, frames0,
                                              args.cpu_1thread_iters)
        # the timed GPU solves' relative L2 error on frame 0 against the FP64 oracle
        result["err_vs_oracle"] = result["cpu_baseline"]["gpu_err_vs_oracle_frame0"]
    if args.large and args.large != args.config:
        result["large_workload"] = large_record(args.large, args, msf, torch, dev)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
