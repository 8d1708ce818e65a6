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


def _radius(shape):
    """Radius of a sphere about the centre that holds the shape."""
    if shape.kind == "ellipsoid":
        return float(np.max(shape.axes))
    return float(np.hypot(shape.axes[0], shape.axes[2]))


def _pixel_box(g, theta, centre, radius):
    """Detector rows / columns whose rays can meet the sphere (conservative)."""
    c, s = np.cos(theta), np.sin(theta)
    S = np.array([g.src_iso * c, g.src_iso * s, 0.0])
    rel = centre - S
    depth = -(rel[0] * c + rel[1] * s)            # along the central ray
    lat = -rel[0] * s + rel[1] * c                 # along e_u
    if depth - radius <= 0:
        return 0, g.nv, 0, g.nu
    mag = g.src_det / depth
    m2 = g.src_det / (depth - radius)
    uc, vc = lat * mag, rel[2] * mag
    half = radius * m2 + max(g.du, g.dv) + abs(uc) * (m2 / mag - 1.0) + abs(vc) * (m2 / mag - 1.0)
    iu0 = int(np.floor((uc - half - g.det_off_u) / g.du + 0.5 * (g.nu - 1)))
    iu1 = int(np.ceil((uc + half - g.det_off_u) / g.du + 0.5 * (g.nu - 1))) + 1
    iv0 = int(np.floor((vc - half - g.det_off_v) / g.dv + 0.5 * (g.nv - 1)))
    iv1 = int(np.ceil((vc + half - g.det_off_v) / g.dv + 0.5 * (g.nv - 1))) + 1
    return max(iv0, 0), min(iv1, g.nv), max(iu0, 0), min(iu1, g.nu)


def fixture_tubes(cfg, n_tubes=2, radius=1.5, mu=0.05):
    """Vertical tubes just outside the volume (inside the detector's field of
    view), the fixtures of the paper's Appendix A: static cylinders parallel to
    the rotation axis, placed on the y axis beyond the volume's face."""
    nx, ny, nz = cfg.n
    out = []
    for k in range(n_tubes):
        side = 1.0 if k % 2 == 0 else -1.0
        centre = np.array([0.0, side * (0.5 * ny + 2.0 * radius + 1.0 + 2.0 * (k // 2)), 0.0])
        out.append(synth.Shape("cylinder", centre, np.array([radius, radius, 2.0 * nz]), np.eye(3), mu,
                               np.zeros(3)))
    return out


def shapes_sinogram(g, shapes, frames=None):
    """Analytic sinogram of fixed shapes (no motion) for the listed frames."""
    frames = range(g.n_frames) if frames is None else list(frames)
    parts = []
    for f in frames:
        for view in range(int(g.view_offset[f]), int(g.view_offset[f + 1])):
            S, D = view_rays(g, g.angles[view])
            acc = np.zeros(len(D))
            for s in shapes:
                acc += s.mu * _chords(S, D, s, s.centre)
            parts.append(acc)
    return np.concatenate(parts) if parts else np.zeros(0)


def sinogram(cfg, g, frames=None, threads=None):
    """Analytic y (float64) of the listed frames, concatenated like the library's sinograms.
    Each shape is evaluated only on the detector box that its bounding sphere projects to."""
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
        D = D.reshape(g.nv, g.nu, 3)
        acc = np.zeros((g.nv, g.nu))
        for s, c in zip(shapes, centres):
            v0, v1, u0, u1 = _pixel_box(g, g.angles[view], c, _radius(s))
            if v1 > v0 and u1 > u0:
                sub = np.ascontiguousarray(D[v0:v1, u0:u1]).reshape(-1, 3)
                acc[v0:v1, u0:u1] += s.mu * _chords(S, sub, s, c).reshape(v1 - v0, u1 - u0)
        return acc.reshape(-1)

    n = threads or min(16, os.cpu_count() or 1)
    with ThreadPoolExecutor(n) as ex:
        parts = list(ex.map(one, jobs))
    return np.concatenate(parts) if parts else np.zeros(0)
