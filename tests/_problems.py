"""Seeded test problems: inputs from the generator, measurements and expected
values from the FP64 oracle only."""
import functools

import numpy as np

import oracle
from paper_2008_01567_amd import synth


@functools.lru_cache(maxsize=8)
def problem(name, frames=None):
    """(cfg, geometry of the frames, x_true, v, y, lam) with float64 arrays."""
    cfg = synth.config(name)
    g = synth.make_geometry(cfg)
    fr = list(range(g.n_frames)) if frames is None else list(frames)
    x0 = synth.make_phantom(cfg, fr)
    v = synth.make_v(cfg, x0, fr)
    y, lam = oracle.make_measurement(cfg, g, x0, fr)
    gs = g if frames is None else g.subset(fr)
    # the library takes FP32 inputs: both sides solve the problem with the rounded values
    f32 = lambda a: a.astype(np.float32).astype(np.float64)
    return cfg, gs, f32(x0), f32(v), f32(y), f32(lam)


@functools.lru_cache(maxsize=8)
def oracle_solution(name, frames=None, tol=1e-12):
    cfg, g, x0, v, y, lam = problem(name, frames)
    x, st = oracle.prox_cg(g, v, y, lam, cfg.sigma, tol=tol, max_iter=20000)
    return x, st


def rel_l2(a, b):
    a = np.asarray(a, dtype=np.float64).reshape(-1)
    b = np.asarray(b, dtype=np.float64).reshape(-1)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))
