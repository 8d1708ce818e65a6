"""Seeded synthetic inputs for the forward-model proximal map.

This module is the only code that both the HIP path and the FP64 oracle use.
It renders phantoms, draws angle schedules and Gaussian noise, and turns a
noiseless sinogram into the noisy measurement and its weights.  It holds none
of the method's arithmetic: no ray geometry, no projector, no solver.  The
noiseless sinogram ``A x0`` is computed by whichever side consumes the inputs.

Workload structure follows the paper's simulated experiments (Sec. VII,
"Simulated Data 360 / 90 degrees"): a few piecewise-constant materials, the
object translated vertically by one voxel per time point, sparse views per
time point and limited-angle arcs.  The paper's own phantom and scans are not
available, so seeded ellipsoid/cylinder phantoms stand in for them.

Conventions shared by both sides (a data format, not arithmetic):

* volume arrays are ``[frame][nz][ny][nx]`` (x fastest);
* sinogram arrays are the frames' views concatenated, each view ``[nv][nu]``
  (u fastest); frame ``n`` owns views ``view_offset[n] .. view_offset[n+1]-1``;
* angles are radians, one per view.
"""
from __future__ import annotations

from dataclasses import dataclass, field
import math

import numpy as np

GOLDEN_DEG = 180.0 * (math.sqrt(5.0) - 1.0) / 2.0  # 111.2461 degrees

# seed streams: seed = 1000 * config_id + stream
STREAM_PHANTOM, STREAM_YNOISE, STREAM_VNOISE, STREAM_VIEWS, STREAM_CNN = 0, 1, 2, 3, 4


@dataclass(frozen=True)
class Geometry:
    """Circular cone-beam scan of a 4D volume (plain data, no arithmetic).

    Distances are in voxel units (voxel side = 1).  ``du``/``dv`` are the
    detector pixel pitch on the detector plane.
    """
    nx: int
    ny: int
    nz: int
    n_frames: int
    nu: int
    nv: int
    du: float
    dv: float
    src_iso: float
    src_det: float
    view_offset: np.ndarray          # int64 [n_frames + 1]
    angles: np.ndarray               # float64 [n_views], radians
    det_off_u: float = 0.0
    det_off_v: float = 0.0

    @property
    def n_views(self) -> int:
        return int(self.view_offset[-1])

    @property
    def n_vox(self) -> int:
        return self.nx * self.ny * self.nz

    @property
    def n_rays_per_view(self) -> int:
        return self.nu * self.nv

    def views_of(self, f: int) -> int:
        return int(self.view_offset[f + 1] - self.view_offset[f])

    def voxel_views(self) -> int:
        """Sum over frames of voxels x views (the metric's work unit)."""
        return self.n_vox * self.n_views

    def subset(self, frames) -> "Geometry":
        """Geometry of a subset of frames (same per-frame views and angles)."""
        frames = list(frames)
        counts = [self.views_of(f) for f in frames]
        off = np.zeros(len(frames) + 1, dtype=np.int64)
        off[1:] = np.cumsum(counts)
        ang = np.concatenate([self.angles[self.view_offset[f]:self.view_offset[f + 1]] for f in frames])
        return Geometry(self.nx, self.ny, self.nz, len(frames), self.nu, self.nv, self.du, self.dv,
                        self.src_iso, self.src_det, off, ang, self.det_off_u, self.det_off_v)

    def sino_slice(self, f: int) -> slice:
        r = self.n_rays_per_view
        return slice(int(self.view_offset[f]) * r, int(self.view_offset[f + 1]) * r)


# ---------------------------------------------------------------------------
# workload configurations
# ---------------------------------------------------------------------------

@dataclass(frozen=True)
class Config:
    cid: int                 # seed base (seed = 1000 * cid + stream)
    n: tuple                 # (nx, ny, nz)
    n_frames: int
    det: tuple               # (nu, nv)
    schedule: str            # "golden" | "interlaced" | "arcs"
    views: int               # views per frame (golden / interlaced)
    arc_deg: float           # angular range for interlaced schedules
    src_iso: float
    src_det: float
    n_objects: int
    cylinders: int = 0       # number of cylinders (moving-object class)
    moving: bool = False     # per-object velocities instead of +1 z / frame
    ragged_views: tuple = (6, 40)
    ragged_arc: tuple = (60.0, 150.0)
    sigma: float = 0.5
    tol: float = 1e-6
    supersample: int = 4
    pitch_at_iso: float = 1.0    # detector pitch measured at the isocentre
    weights: str = "clipped"     # noise / weight model: "clipped" or "paper" (see finish_measurement)
    extra: dict = field(default_factory=dict)

    @property
    def du(self) -> float:
        return self.pitch_at_iso * self.src_det / self.src_iso


def _ratio_geom(n: int):
    # distances keep the 32^3 problem's ratios: R_s = 6.25 n, R_sd = 12.5 n
    return 6.25 * n, 12.5 * n


CONFIGS = {
    # 8^3 / 16^3: tiny problems for dense-solve and brute-force pins
    "tiny8": Config(90, (8, 8, 8), 2, (12, 12), "golden", 8, 180.0, 50.0, 100.0, 2, supersample=4, tol=1e-10),
    "tiny16": Config(91, (16, 16, 16), 2, (24, 24), "golden", 8, 180.0, 100.0, 200.0, 3, tol=1e-10),
    # config 1: 32^3 x 4, 48^2 detector, 8 golden-angle views per frame over 180 deg
    "c1": Config(1, (32, 32, 32), 4, (48, 48), "golden", 8, 180.0, 200.0, 400.0, 3, tol=1e-8),
    # config 2: 128^3 x 16, 192^2 detector, 16 interlaced views per frame over 360 deg
    "c2": Config(2, (128, 128, 128), 16, (192, 192), "interlaced", 16, 360.0, *_ratio_geom(128), 8, tol=1e-6),
    # config 3: 256^3 x 24, 384^2 detector, ragged views / arcs
    "c3": Config(3, (256, 256, 256), 24, (384, 384), "arcs", 0, 0.0, *_ratio_geom(256), 8, tol=1e-6),
    # config 4: 128^3 x 16 with config-1 ratios, 8 golden views per frame over 180 deg
    "c4": Config(4, (128, 128, 128), 16, (192, 192), "golden", 8, 180.0, *_ratio_geom(128), 8, tol=1e-4),
    # config 5: 512x512x256 x 32, 768x512 detector, 20 interlaced views over 180 deg
    "c5": Config(5, (512, 512, 256), 32, (768, 512), "interlaced", 20, 180.0, *_ratio_geom(512), 12,
                 cylinders=4, moving=True, tol=1e-6, supersample=1),
    # reduced-size variants used by parity tests (same structure, faster oracle)
    "c2s": Config(12, (48, 48, 40), 6, (72, 64), "interlaced", 16, 360.0, *_ratio_geom(48), 6, tol=1e-6),
    "c3s": Config(13, (40, 44, 36), 5, (64, 56), "arcs", 0, 0.0, *_ratio_geom(40), 5, tol=1e-6),
    "c5s": Config(15, (48, 40, 32), 4, (72, 48), "interlaced", 20, 180.0, *_ratio_geom(48), 6,
                  cylinders=2, moving=True, tol=1e-6, supersample=2),
    # the paper's own noise / weight model on the 128^3 x 16 and reduced 48^2 x 40 workloads
    "c2p": Config(22, (128, 128, 128), 16, (192, 192), "interlaced", 16, 360.0, *_ratio_geom(128), 8, tol=1e-6,
                  weights="paper"),
    "c2sp": Config(32, (48, 48, 40), 6, (72, 64), "interlaced", 16, 360.0, *_ratio_geom(48), 6, tol=1e-6,
                   weights="paper"),
    # odd sizes everywhere (voxel planes at half-integers, a voxel straddling z = 0, the detector
    # centre between pixels) and a detector shifted off the central ray
    "odd": Config(18, (21, 17, 23), 3, (33, 29), "golden", 7, 180.0, *_ratio_geom(21), 3, tol=1e-6,
                  extra={"det_off": (0.37, -0.61)}),
    # an odd number of detector rows and no offset: the middle row is level (zp = 0) and, nz being
    # even, runs in the face z = 0 between two voxel slabs (the upper one takes it, half-open voxels)
    "level": Config(19, (24, 20, 16), 2, (31, 31), "golden", 6, 180.0, *_ratio_geom(24), 3, tol=1e-6),
    # a source close to a tall volume: rays climb up to ~2 (steep) and ~3 (steeper) voxels in z per
    # voxel of xy path, so one ray crosses several z planes inside one xy cell; steeper's cells
    # also meet more than three detector columns
    "steep": Config(24, (16, 16, 48), 3, (48, 96), "golden", 6, 180.0, 28.0, 56.0, 3, tol=1e-6),
    "steeper": Config(25, (16, 16, 48), 2, (48, 112), "golden", 6, 180.0, 20.0, 40.0, 3, tol=1e-6),
    # a single voxel slab (nz = 1); the shifted rows put one ray (zp = -1) through the slab's lower
    # face near the isocentre and one (zp = 0.2) inside the slab all the way
    "flat": Config(26, (24, 20, 1), 3, (64, 8), "golden", 7, 180.0, 200.0, 400.0, 2, pitch_at_iso=0.6,
                   tol=1e-6, extra={"det_off": (0.0, -0.4)}),
    # tall volumes (nz > 128): several z voxels per lane in the voxel-driven adjoint
    "tall3": Config(16, (20, 18, 150), 2, (32, 164), "golden", 6, 180.0, 1000.0, 2000.0, 3, tol=1e-6),
    "tall4": Config(17, (16, 14, 230), 2, (28, 244), "interlaced", 5, 360.0, 1000.0, 2000.0, 3, tol=1e-6),
    # taller than one gather wave's 256 voxels (two z-chunks per voxel column), and about 300 detector
    # rows meeting the volume (five rays per lane by default)
    "tall5": Config(27, (12, 10, 300), 2, (20, 316), "golden", 5, 180.0, 1000.0, 2000.0, 3, tol=1e-6),
}


def config(name: str) -> Config:
    return CONFIGS[name]


# ---------------------------------------------------------------------------
# angle schedules
# ---------------------------------------------------------------------------

def angles_golden(n_frames: int, views: int, range_deg: float = 180.0) -> np.ndarray:
    """Golden-angle interlaced acquisition: global index k, theta_k = k*111.25 deg mod range."""
    k = np.arange(n_frames * views, dtype=np.float64)
    return np.deg2rad(np.mod(k * GOLDEN_DEG, range_deg))


def angles_interlaced(n_frames: int, views: int, range_deg: float) -> np.ndarray:
    """Offset-interlaced: theta_{n,j} = (j + n / N_t) * range / V."""
    n = np.arange(n_frames, dtype=np.float64)[:, None]
    j = np.arange(views, dtype=np.float64)[None, :]
    return np.deg2rad(((j + n / n_frames) * range_deg / views).reshape(-1))


def angles_arcs(n_frames: int, seed: int, vrange=(6, 40), arange=(60.0, 150.0)):
    """Contiguous limited-angle arcs: frame n starts where frame n-1 ended."""
    rng = np.random.default_rng(seed)
    counts = rng.integers(vrange[0], vrange[1] + 1, size=n_frames)
    arcs = rng.uniform(arange[0], arange[1], size=n_frames)
    out, start = [], 0.0
    for c, a in zip(counts, arcs):
        out.append(start + np.arange(c, dtype=np.float64) * a / c)
        start += a
    return counts.astype(np.int64), np.deg2rad(np.mod(np.concatenate(out), 360.0))


def make_geometry(cfg: Config, n_frames: int | None = None) -> Geometry:
    nf = cfg.n_frames if n_frames is None else n_frames
    if cfg.schedule == "golden":
        counts = np.full(nf, cfg.views, dtype=np.int64)
        ang = angles_golden(nf, cfg.views, cfg.arc_deg)
    elif cfg.schedule == "interlaced":
        counts = np.full(nf, cfg.views, dtype=np.int64)
        ang = angles_interlaced(nf, cfg.views, cfg.arc_deg)
    elif cfg.schedule == "arcs":
        counts, ang = angles_arcs(nf, 1000 * cfg.cid + STREAM_VIEWS, cfg.ragged_views, cfg.ragged_arc)
    else:
        raise ValueError(cfg.schedule)
    off = np.zeros(nf + 1, dtype=np.int64)
    off[1:] = np.cumsum(counts)
    nx, ny, nz = cfg.n
    ou, ov = cfg.extra.get("det_off", (0.0, 0.0))
    return Geometry(nx, ny, nz, nf, cfg.det[0], cfg.det[1], cfg.du, cfg.du, cfg.src_iso, cfg.src_det,
                    off, ang, ou, ov)


# ---------------------------------------------------------------------------
# phantoms
# ---------------------------------------------------------------------------

@dataclass(frozen=True)
class Shape:
    kind: str                # "ellipsoid" | "cylinder"
    centre: np.ndarray       # (x, y, z) at frame 0, voxel units, origin at the volume centre
    axes: np.ndarray         # ellipsoid semi-axes, or (radius, radius, half-length)
    rot: np.ndarray          # 3x3, columns are the shape's principal axes
    mu: float                # attenuation per voxel
    vel: np.ndarray          # displacement per frame (voxel units)


def _random_rotation(rng) -> np.ndarray:
    q = rng.normal(size=4)
    q /= np.linalg.norm(q)
    a, b, c, d = q
    return np.array([[a*a + b*b - c*c - d*d, 2*(b*c - a*d), 2*(b*d + a*c)],
                     [2*(b*c + a*d), a*a - b*b + c*c - d*d, 2*(c*d - a*b)],
                     [2*(b*d - a*c), 2*(c*d + a*b), a*a - b*b - c*c + d*d]])


def make_shapes(cfg: Config, seed: int | None = None) -> list:
    """Seeded scene: centres within radius 0.3 n (xy) and |z| <= 0.25 n_z,
    semi-axes U(0.06 n, 0.2 n), uniform random rotation, mu ~ U(0.01, 0.05)."""
    rng = np.random.default_rng(1000 * cfg.cid + STREAM_PHANTOM if seed is None else seed)
    nx, ny, nz = cfg.n
    n = min(nx, ny)
    shapes = []
    for i in range(cfg.n_objects + cfg.cylinders):
        r = 0.3 * n * math.sqrt(rng.uniform())
        phi = rng.uniform(0, 2 * math.pi)
        c = np.array([r * math.cos(phi), r * math.sin(phi), rng.uniform(-0.25, 0.25) * nz])
        rot = _random_rotation(rng)
        mu = rng.uniform(0.01, 0.05)
        if cfg.moving:
            d = rng.normal(size=3)
            vel = d / np.linalg.norm(d) * rng.uniform(0.0, 1.0)
        else:
            vel = np.array([0.0, 0.0, 1.0])
        if i < cfg.n_objects:
            axes = rng.uniform(0.06 * n, 0.2 * n, size=3)
            shapes.append(Shape("ellipsoid", c, axes, rot, mu, vel))
        else:
            rad = rng.uniform(0.03 * n, 0.1 * n)
            half = rng.uniform(0.1 * n, 0.3 * n)
            shapes.append(Shape("cylinder", c, np.array([rad, rad, half]), rot, mu, vel))
    return shapes


def _inside(shape: Shape, px, py, pz):
    """Indicator of the closed shape for points given relative to its centre."""
    R = shape.rot
    a = px * R[0, 0] + py * R[1, 0] + pz * R[2, 0]
    b = px * R[0, 1] + py * R[1, 1] + pz * R[2, 1]
    c = px * R[0, 2] + py * R[1, 2] + pz * R[2, 2]
    if shape.kind == "ellipsoid":
        return (a / shape.axes[0]) ** 2 + (b / shape.axes[1]) ** 2 + (c / shape.axes[2]) ** 2 <= 1.0
    return ((a / shape.axes[0]) ** 2 + (b / shape.axes[1]) ** 2 <= 1.0) & (np.abs(c) <= shape.axes[2])


def _half_extent(shape: Shape) -> np.ndarray:
    R = shape.rot
    if shape.kind == "ellipsoid":
        return np.sqrt((R ** 2) @ (shape.axes ** 2))
    # cylinder: bound by the enclosing box of its axis-aligned (local) box
    return np.abs(R) @ shape.axes


def _render_shape(shape: Shape, centre, n, ss: int, out: np.ndarray):
    """Add mu x (supersampled occupancy fraction) of one shape into out[nz][ny][nx]."""
    nx, ny, nz = n
    he = _half_extent(shape) + 1.0
    lo = [int(math.floor(centre[k] - he[k] + (n[k] - 1) / 2.0)) for k in range(3)]
    hi = [int(math.ceil(centre[k] + he[k] + (n[k] - 1) / 2.0)) + 1 for k in range(3)]
    lo = [max(0, v) for v in lo]
    hi = [min(n[k], hi[k]) for k in range(3)]
    if any(hi[k] <= lo[k] for k in range(3)):
        return
    sub = (np.arange(ss) + 0.5) / ss - 0.5
    xs = np.arange(lo[0], hi[0]) - (nx - 1) / 2.0 - centre[0]
    ys = np.arange(lo[1], hi[1]) - (ny - 1) / 2.0 - centre[1]
    zs = np.arange(lo[2], hi[2]) - (nz - 1) / 2.0 - centre[2]
    occ = np.zeros((len(zs), len(ys), len(xs)), dtype=np.float64)
    for oz in sub:
        pz = (zs + oz)[:, None, None]
        for oy in sub:
            py = (ys + oy)[None, :, None]
            for ox in sub:
                px = (xs + ox)[None, None, :]
                occ += _inside(shape, px, py, pz)
    out[lo[2]:hi[2], lo[1]:hi[1], lo[0]:hi[0]] += (shape.mu / ss ** 3) * occ


def frame_centre(shape: Shape, cfg: Config, f: int) -> np.ndarray:
    """Object centre at frame f.  Without per-object velocities the scene moves
    +1 voxel per frame along +z, centred on the middle frame."""
    if cfg.moving:
        return shape.centre + shape.vel * (f - (cfg.n_frames - 1) / 2.0)
    return shape.centre + np.array([0.0, 0.0, float(f - cfg.n_frames // 2)])


def make_phantom(cfg: Config, frames=None, dtype=np.float64, shapes=None) -> np.ndarray:
    """Voxelised phantom x0 for the requested frames: [len(frames)][nz][ny][nx]."""
    frames = range(cfg.n_frames) if frames is None else list(frames)
    shapes = make_shapes(cfg) if shapes is None else shapes
    nx, ny, nz = cfg.n
    out = np.zeros((len(frames), nz, ny, nx), dtype=dtype)
    if cfg.moving:
        for i, f in enumerate(frames):
            vol = np.zeros((nz, ny, nx))
            for s in shapes:
                _render_shape(s, frame_centre(s, cfg, f), cfg.n, cfg.supersample, vol)
            out[i] = vol
        return out
    # rigid +1 voxel / frame motion along z: render the scene once on a z-extended
    # grid and cut every frame out of it (frame f sees the scene shifted by d_f)
    d = [f - cfg.n_frames // 2 for f in range(cfg.n_frames)]
    dmin, dmax = min(d), max(d)
    ne = nz + dmax - dmin
    ext = np.zeros((ne, ny, nx))
    # frame f, slice k  <->  extended slice e = k - d_f + dmax; in the extended
    # grid's own centred coordinates the scene sits (dmax + dmin)/2 higher
    shift = (dmax + dmin) / 2.0
    for s in shapes:
        c = s.centre + np.array([0.0, 0.0, shift])
        _render_shape(s, c, (nx, ny, ne), cfg.supersample, ext)
    for i, f in enumerate(frames):
        lo = dmax - d[f]
        out[i] = ext[lo:lo + nz]
    return out


def make_v(cfg: Config, x0: np.ndarray, frames=None, std: float = 0.002) -> np.ndarray:
    """v = x0 + N(0, std^2) per voxel, one seeded stream per frame."""
    frames = range(x0.shape[0]) if frames is None else list(frames)
    out = np.empty_like(x0)
    for i, f in enumerate(frames):
        rng = np.random.default_rng([1000 * cfg.cid + STREAM_VNOISE, f])
        out[i] = x0[i] + std * rng.standard_normal(x0[i].shape)
    return out


def noise_eps(cfg: Config, geom: Geometry, frames=None, dtype=np.float64) -> np.ndarray:
    """Unit normal draws for the sinogram noise of the requested frames (concatenated)."""
    frames = range(geom.n_frames) if frames is None else list(frames)
    parts = []
    for f in frames:
        rng = np.random.default_rng([1000 * cfg.cid + STREAM_YNOISE, f])
        parts.append(rng.standard_normal(geom.views_of(f) * geom.n_rays_per_view).astype(dtype))
    return np.concatenate(parts) if parts else np.zeros(0, dtype=dtype)


def finish_measurement(y_clean: np.ndarray, eps: np.ndarray, counts, rays_per_view: int,
                       noise_frac: float = 0.01, dtype=np.float64, model: str = "clipped"):
    """Noisy measurement and weights, frame by frame, s = noise_frac * max(y_clean of the frame).

    model "clipped" (the workloads' stated recipe): y = y_clean + s * eps,
    Lambda = 1 / max(y, s) (inverse of the clipped measurement).
    model "paper" (the paper's simulation, Sec. VII): y ~ N(y_clean, Lambda^-1) with
    inverse variance Lambda = c exp(-y_clean); the paper leaves c to be chosen,
    here c = 1 / s^2, so a ray of zero attenuation has noise s and the noise
    grows as exp(y_clean / 2) with attenuation (Poisson-like).
    ``counts`` are the views per frame of the concatenated arrays.
    """
    if model not in ("clipped", "paper"):
        raise ValueError("unknown noise model %r" % model)
    y = np.empty(y_clean.shape, dtype=dtype)
    lam = np.empty(y_clean.shape, dtype=dtype)
    o = 0
    for c in counts:
        m = int(c) * rays_per_view
        yc = y_clean[o:o + m].astype(np.float64)
        s = noise_frac * float(yc.max()) if m else 0.0
        e = eps[o:o + m].astype(np.float64)
        if model == "clipped":
            yy = yc + s * e
            y[o:o + m] = yy
            lam[o:o + m] = 1.0 / np.maximum(yy, s) if s > 0 else 0.0
        else:
            w = np.exp(-yc) / (s * s) if s > 0 else np.zeros_like(yc)
            y[o:o + m] = yc + (s * np.exp(0.5 * yc) * e if s > 0 else 0.0)
            lam[o:o + m] = w
        o += m
    return y, lam


def frame_counts(geom: Geometry) -> np.ndarray:
    return np.diff(geom.view_offset)
