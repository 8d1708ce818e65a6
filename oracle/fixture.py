"""FP64 oracle of the blind fixture correction (TEST INFRASTRUCTURE ONLY).

Paper, Appendix A (algorithm "Blind fixture correction"): from a reconstruction
x, mask it with a cylinder slightly smaller than the field of view, take the
error sinogram e = y - A x_m (mostly the projection of the fixtures outside
the field of view), blur it to p (the fixtures' projection is smooth, the
object's residue is not), fit the scalar c minimising ||e - c p||^2, and
return y - c p.

Readings: the mask keeps the voxels whose centre lies within `radius` of the
rotation axis; the blur is a separable Gaussian over the detector's u and v
within each view (2 ceil(3 std) + 1 normalised taps, zero outside the
detector); c is fitted per time frame (each frame's sinogram is corrected on
its own).
"""
from __future__ import annotations

import math

import numpy as np


def cylinder_mask(x: np.ndarray, radius: float) -> np.ndarray:
    """Zero the voxels of x [frames][nz][ny][nx] whose centre is farther than
    radius from the rotation axis (voxel centre i - (nx - 1)/2, j - (ny - 1)/2)."""
    nz, ny, nx = x.shape[1:]
    cx = np.arange(nx) - 0.5 * (nx - 1)
    cy = np.arange(ny) - 0.5 * (ny - 1)
    inside = (cx[None, :] ** 2 + cy[:, None] ** 2) <= radius * radius
    return x * inside[None, None, :, :]


def gaussian_taps(std: float) -> np.ndarray:
    r = int(math.ceil(3.0 * std))
    t = np.arange(-r, r + 1, dtype=np.float64)
    w = np.exp(-0.5 * t * t / (std * std))
    return w / w.sum()


def blur_view(img: np.ndarray, std: float) -> np.ndarray:
    """Separable Gaussian blur of one view [nv][nu], values outside taken as zero."""
    w = gaussian_taps(std)
    r = len(w) // 2
    out = img.astype(np.float64)
    for axis in (0, 1):
        n = out.shape[axis]
        pad = [(0, 0), (0, 0)]
        pad[axis] = (r, r)
        p = np.pad(out, pad)
        acc = np.zeros_like(out)
        for k, wk in enumerate(w):
            sl = [slice(None), slice(None)]
            sl[axis] = slice(k, k + n)
            acc += wk * p[tuple(sl)]
        out = acc
    return out


def correct(geom, x: np.ndarray, y: np.ndarray, radius: float, std: float):
    """Algorithm 'Blind fixture correction' for every frame.
    Returns (y_corr, c [frames], e, p) with sinograms concatenated like y."""
    import oracle
    xm = cylinder_mask(x, radius)
    y = np.asarray(y, dtype=np.float64)
    e = np.empty_like(y)
    p = np.empty_like(y)
    c = np.zeros(geom.n_frames)
    rpv = geom.nu * geom.nv
    for f in range(geom.n_frames):
        s = geom.sino_slice(f)
        ax = oracle.FrameMatrix(geom.subset([f]), 0).A(xm[f]) if geom.views_of(f) else np.zeros(0)
        e[s] = y[s] - ax
        for k in range(geom.views_of(f)):
            a = s.start + k * rpv
            p[a:a + rpv] = blur_view(e[a:a + rpv].reshape(geom.nv, geom.nu), std).reshape(-1)
        pp = float(p[s] @ p[s])
        c[f] = float(e[s] @ p[s]) / pp if pp > 0 else 0.0
    y_corr = y.copy()
    for f in range(geom.n_frames):
        s = geom.sino_slice(f)
        y_corr[s] = y[s] - c[f] * p[s]
    return y_corr, c, e, p
