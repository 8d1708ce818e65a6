"""Analytic sinograms of the continuous phantom (test inputs at full size).

Line integrals of mu over ellipsoids and finite right-circular cylinders, in
closed form, for every ray of a scan: the measurement y of the full-size
parity tests.  It stands in for A x0 where the FP64 oracle cannot build A
(hundreds of millions of rays).  Any y defines a valid proximal-map problem;
this one has the workloads' structure (projections of a few piecewise
constant objects).

Rays follow the scan geometry of the paper's cone-beam model (Sec. II): point
source S = (R_s cos t, R_s sin t, 0), detector pixel centre
D = S + R_sd (-cos t, -sin t, 0) + u e_u + v e_v.
"""
from __future__ import annotations

from concurrent.futures import ThreadPoolExecutor
import os

import numpy as np

from paper_2008_01567_amd import synth


def view_rays(g, theta):
    """(S [3], D [nv*nu, 3]) of one view, rows iv-major (u fastest)."""
    c, s = np.cos(theta), np.sin(theta)
    u = (np.arange(g.nu) - 0.5 * (g.nu - 1)) * g.du + g.det_off_u
    v = (np.arange(g.nv) - 0.5 * (g.nv - 1)) * g.dv + g.det_off_v
    S = np.array([g.src_iso * c, g.src_iso * s, 0.0])
    d0 = S + g.src_det * np.array([-c, -s, 0.0])
    U, V = np.meshgrid(u, v)          # [nv][nu]
    D = np.empty((g.nv * g.nu, 3))
    D[:, 0] = d0[0] - U.reshape(-1) * s
    D[:, 1] = d0[1] + U.reshape(-1) * c
    D[:, 2] = V.reshape(-1)
    return S, D


def _chords(S, D, shape, centre):
    """Length of each segment S -> D[i] inside the shape (vectorised over rays)."""
    Rt = shape.rot.T
    p = Rt @ (S - centre)                       # source in the shape's frame
    d = (D - S) @ shape.rot                     # directions in the shape's frame, [n, 3]
    L = np.linalg.norm(D - S, axis=1)
    if shape.kind == "ellipsoid":
        ps = p / shape.axes
        ds = d / shape.axes
        a = np.einsum("ij,ij->i", ds, ds)
        b = ds @ ps
        cc = ps @ ps - 1.0
        disc = b * b - a * cc
        root = np.sqrt(np.maximum(disc, 0.0))
        t0 = np.clip((-b - root) / a, 0.0, 1.0)
        t1 = np.clip((-b + root) / a, 0.0, 1.0)
        return np.where(disc > 0, (t1 - t0) * L, 0.0)
    # cylinder: radius axes[0] about the local z axis, half-length axes[2]
    r, h = shape.axes[0], shape.axes[2]
    a = d[:, 0] ** 2 + d[:, 1] ** 2
    b = d[:, 0] * p[0] + d[:, 1] * p[1]
    cc = p[0] ** 2 + p[1] ** 2 - r * r
    disc = b * b - a * cc
    root = np.sqrt(np.maximum(disc, 0.0))
    with np.errstate(divide="ignore", invalid="ignore"):
        t0 = np.where(a > 0, (-b - root) / a, -np.inf)
        t1 = np.where(a > 0, (-b + root) / a, np.inf)
        inside_inf = (a > 0) & (disc > 0) | (a == 0) & (cc < 0)
        z0 = np.where(d[:, 2] != 0, (-h - p[2]) / d[:, 2], -np.inf)
        z1 = np.where(d[:, 2] != 0, (h - p[2]) / d[:, 2], np.inf)
    zlo, zhi = np.minimum(z0, z1), np.maximum(z0, z1)
    zin = (d[:, 2] != 0) | (np.abs(p[2]) <= h)
    lo = np.maximum(np.maximum(t0, zlo), 0.0)
    hi = np.minimum(np.minimum(t1, zhi), 1.0)
    return np.where(inside_inf & zin & (hi > lo), (hi - lo) * L, 0.0)


def sinogram(cfg, g, frames=None, threads=None):
    """Analytic y (float64) of the listed frames, concatenated like the library's sinograms."""
    frames = range(g.n_frames) if frames is None else list(frames)
    shapes = synth.make_shapes(cfg)
    jobs = []
    for f in frames:
        centres = [synth.frame_centre(s, cfg, f) for s in shapes]
        for view in range(int(g.view_offset[f]), int(g.view_offset[f + 1])):
            jobs.append((view, centres))

    def one(job):
        view, centres = job
        S, D = view_rays(g, g.angles[view])
        acc = np.zeros(len(D))
        for s, c in zip(shapes, centres):
            acc += s.mu * _chords(S, D, s, c)
        return acc

    n = threads or min(16, os.cpu_count() or 1)
    with ThreadPoolExecutor(n) as ex:
        parts = list(ex.map(one, jobs))
    return np.concatenate(parts) if parts else np.zeros(0)
