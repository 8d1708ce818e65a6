"""FP64 CPU oracle for the forward-model proximal map (multi-slice fusion, Sec. II-III).

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, the smoke check and the benchmark's
CPU-baseline leg may import this package.  It shares no code with the HIP
library (``paper_2008_01567_amd``): the only thing both sides use is the seeded
input generator ``paper_2008_01567_amd.synth``, which holds none of the
method's arithmetic.

Contents
--------
* ``FrameMatrix``: the system matrix A_n of one time frame (paper eq.
  (2)) as an FP64 CSR matrix of exact ray-voxel lengths, built by
  Siddon's method or by brute force (see ``oracle.c``), its transpose, and
  the FP64 conjugate-gradient solve of the proximal map (eq. (4)).
* ``prox_dense``: the proximal map as the dense normal-equation solve
  (Cholesky), for volumes up to 16^3.
* ``oracle.cnn``: FP64 3D convolutional network forward/backward and Adam.
* ``oracle.mace``: Algorithm 1 (partial-update Mann iteration) in FP64.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_SRC = os.path.join(_HERE, "oracle.c")
_lib = None


def build(force: bool = True) -> str:
    """Compile the C oracle with gcc (FP64, OpenMP)."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared", _SRC,
                               "-o", tmp, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


class _Geom(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32), ("nu", C.c_int32),
                ("nv", C.c_int32), ("pad_", C.c_int32), ("du", C.c_double), ("dv", C.c_double),
                ("src_iso", C.c_double), ("src_det", C.c_double), ("off_u", C.c_double),
                ("off_v", C.c_double)]


def _p(a, ct):
    return a.ctypes.data_as(C.POINTER(ct))


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build(force=False)
        L = C.CDLL(_LIB_PATH)
        dp, ip, lp = C.POINTER(C.c_double), C.POINTER(C.c_int32), C.POINTER(C.c_int64)
        gp = C.POINTER(_Geom)
        L.or_ray.argtypes = [gp, C.c_double, C.c_int32, C.c_int32, dp, dp]
        L.or_brute.argtypes = [gp, dp, dp, ip, dp, C.c_int32]
        L.or_brute.restype = C.c_int32
        L.or_siddon.argtypes = [gp, dp, dp, ip, dp, C.c_int32]
        L.or_siddon.restype = C.c_int32
        L.or_voxel_length.argtypes = [gp, dp, dp, C.c_int64]
        L.or_voxel_length.restype = C.c_double
        L.or_csr_count.argtypes = [gp, dp, C.c_int32, C.c_int32, lp]
        L.or_csr_count.restype = C.c_int64
        L.or_csr_fill.argtypes = [gp, dp, C.c_int32, C.c_int32, lp, ip, dp]
        L.or_csr_transpose.argtypes = [C.c_int64, C.c_int64, lp, ip, dp, lp, ip, dp]
        L.or_spmv.argtypes = [C.c_int64, lp, ip, dp, dp, dp]
        L.or_prox_cg.argtypes = [C.c_int64, C.c_int64, lp, ip, dp, lp, ip, dp, dp, dp, dp, C.c_double,
                                 dp, C.c_double, C.c_int32, dp, dp]
        L.or_prox_cg.restype = C.c_int32
        L.or_backproject_voxels.argtypes = [gp, dp, C.c_int32, dp, lp, C.c_int32, dp]
        L.or_project_rays.argtypes = [gp, dp, ip, ip, ip, C.c_int32, dp, dp]
        L.or_voxel_columns.argtypes = [gp, dp, C.c_int32, lp, C.c_int32, ip, lp, dp, C.c_int32]
        L.or_num_threads.restype = C.c_int32
        L.or_set_num_threads.argtypes = [C.c_int32]
        _lib = L
    return _lib


def num_threads() -> int:
    return int(lib().or_num_threads())


def set_num_threads(n: int) -> None:
    """OpenMP threads of the oracle's following calls (for timing it)."""
    lib().or_set_num_threads(int(n))


def cgeom(geom) -> _Geom:
    return _Geom(geom.nx, geom.ny, geom.nz, geom.nu, geom.nv, 0, geom.du, geom.dv, geom.src_iso,
                 geom.src_det, geom.det_off_u, geom.det_off_v)


def ray(geom, theta: float, iu: int, iv: int):
    """Source and detector-pixel centre of one ray (FP64)."""
    S = np.zeros(3)
    D = np.zeros(3)
    lib().or_ray(C.byref(cgeom(geom)), float(theta), int(iu), int(iv), _p(S, C.c_double), _p(D, C.c_double))
    return S, D


def ray_entries(geom, S, D, method: str = "siddon"):
    """(voxel indices, lengths) of one segment S->D."""
    S = np.ascontiguousarray(S, dtype=np.float64)
    D = np.ascontiguousarray(D, dtype=np.float64)
    cap = geom.nx * geom.ny * geom.nz if method == "brute" else geom.nx + geom.ny + geom.nz + 4
    idx = np.zeros(cap, dtype=np.int32)
    ln = np.zeros(cap, dtype=np.float64)
    fn = lib().or_brute if method == "brute" else lib().or_siddon
    n = fn(C.byref(cgeom(geom)), _p(S, C.c_double), _p(D, C.c_double), _p(idx, C.c_int32),
           _p(ln, C.c_double), cap)
    return idx[:n].copy(), ln[:n].copy()


class FrameMatrix:
    """System matrix A_n of one frame: rows = (view, iv, iu), u fastest;
    columns = voxels [nz][ny][nx]; entries = exact ray-voxel lengths (FP64)."""

    def __init__(self, geom, frame: int, method: str = "siddon"):
        self.geom = geom
        self.frame = frame
        a0, a1 = int(geom.view_offset[frame]), int(geom.view_offset[frame + 1])
        self.angles = np.ascontiguousarray(geom.angles[a0:a1], dtype=np.float64)
        self.nviews = a1 - a0
        self.nrows = self.nviews * geom.nv * geom.nu
        self.ncols = geom.nx * geom.ny * geom.nz
        m = 1 if method == "brute" else 0
        g = cgeom(geom)
        self.rowptr = np.zeros(self.nrows + 1, dtype=np.int64)
        nnz = lib().or_csr_count(C.byref(g), _p(self.angles, C.c_double), self.nviews, m,
                                 _p(self.rowptr, C.c_int64))
        self.col = np.zeros(max(nnz, 1), dtype=np.int32)
        self.val = np.zeros(max(nnz, 1), dtype=np.float64)
        lib().or_csr_fill(C.byref(g), _p(self.angles, C.c_double), self.nviews, m, _p(self.rowptr, C.c_int64),
                          _p(self.col, C.c_int32), _p(self.val, C.c_double))
        self.nnz = int(nnz)
        self._t = None

    def _transpose(self):
        if self._t is None:
            trp = np.zeros(self.ncols + 1, dtype=np.int64)
            tc = np.zeros(max(self.nnz, 1), dtype=np.int32)
            tv = np.zeros(max(self.nnz, 1), dtype=np.float64)
            lib().or_csr_transpose(self.nrows, self.ncols, _p(self.rowptr, C.c_int64), _p(self.col, C.c_int32),
                                   _p(self.val, C.c_double), _p(trp, C.c_int64), _p(tc, C.c_int32),
                                   _p(tv, C.c_double))
            self._t = (trp, tc, tv)
        return self._t

    def A(self, x):
        x = np.ascontiguousarray(x, dtype=np.float64).reshape(-1)
        out = np.zeros(self.nrows)
        lib().or_spmv(self.nrows, _p(self.rowptr, C.c_int64), _p(self.col, C.c_int32), _p(self.val, C.c_double),
                      _p(x, C.c_double), _p(out, C.c_double))
        return out

    def AT(self, y):
        trp, tc, tv = self._transpose()
        y = np.ascontiguousarray(y, dtype=np.float64).reshape(-1)
        out = np.zeros(self.ncols)
        lib().or_spmv(self.ncols, _p(trp, C.c_int64), _p(tc, C.c_int32), _p(tv, C.c_double), _p(y, C.c_double),
                      _p(out, C.c_double))
        return out

    def dense(self) -> np.ndarray:
        M = np.zeros((self.nrows, self.ncols))
        for r in range(self.nrows):
            s, e = self.rowptr[r], self.rowptr[r + 1]
            np.add.at(M[r], self.col[s:e], self.val[s:e])
        return M

    def prox_cg(self, v, y, lam, sigma, tol=1e-12, max_iter=10000, x0=None):
        """FP64 CG on (A^T Lam A + sigma^-2 I) x = A^T Lam y + sigma^-2 v; returns (x, stats)."""
        trp, tc, tv = self._transpose()
        v = np.ascontiguousarray(v, dtype=np.float64).reshape(-1)
        y = np.ascontiguousarray(y, dtype=np.float64).reshape(-1)
        lam = np.ascontiguousarray(lam, dtype=np.float64).reshape(-1)
        x = np.zeros(self.ncols)
        st = np.zeros(4)
        x0p = None
        if x0 is not None:
            x0 = np.ascontiguousarray(x0, dtype=np.float64).reshape(-1)
            x0p = _p(x0, C.c_double)
        lib().or_prox_cg(self.nrows, self.ncols, _p(self.rowptr, C.c_int64), _p(self.col, C.c_int32),
                         _p(self.val, C.c_double), _p(trp, C.c_int64), _p(tc, C.c_int32), _p(tv, C.c_double),
                         _p(lam, C.c_double), _p(y, C.c_double), _p(v, C.c_double), float(sigma), x0p,
                         float(tol), int(max_iter), _p(x, C.c_double), _p(st, C.c_double))
        return x, {"iters": int(st[0]), "rel_res": st[1], "true_rel_res": st[2], "bnorm": st[3]}


def _frames(geom, frames):
    return range(geom.n_frames) if frames is None else list(frames)


def project(geom, x, frames=None, method="siddon"):
    """y = A x for the given frames (x: [len(frames)][nz][ny][nx]); sinograms concatenated."""
    fr = _frames(geom, frames)
    return np.concatenate([FrameMatrix(geom, f, method).A(x[i]) for i, f in enumerate(fr)])


def backproject(geom, y, frames=None, method="siddon"):
    """x = A^T y for the given frames; y holds the frames' sinograms concatenated."""
    fr = _frames(geom, frames)
    out, o = [], 0
    for f in fr:
        M = FrameMatrix(geom, f, method)
        out.append(M.AT(y[o:o + M.nrows]).reshape(geom.nz, geom.ny, geom.nx))
        o += M.nrows
    return np.stack(out)


def prox_cg(geom, v, y, lam, sigma, tol=1e-12, max_iter=10000, frames=None, x0=None):
    """Proximal map of every requested frame by FP64 CG; returns (x, list of stats)."""
    fr = _frames(geom, frames)
    xs, stats, o = [], [], 0
    for i, f in enumerate(fr):
        M = FrameMatrix(geom, f)
        sl = slice(o, o + M.nrows)
        x, st = M.prox_cg(v[i], y[sl], lam[sl], sigma, tol, max_iter, None if x0 is None else x0[i])
        xs.append(x.reshape(geom.nz, geom.ny, geom.nx))
        stats.append(st)
        o += M.nrows
    return np.stack(xs), stats


def prox_dense(geom, v, y, lam, sigma, frames=None, method="brute"):
    """Proximal map by the dense normal equations (Cholesky), per frame."""
    fr = _frames(geom, frames)
    xs, o = [], 0
    for i, f in enumerate(fr):
        M = FrameMatrix(geom, f, method)
        A = M.dense()
        lam_f = np.asarray(lam[o:o + M.nrows], dtype=np.float64)
        H = A.T @ (lam_f[:, None] * A) + np.eye(M.ncols) / sigma ** 2
        b = A.T @ (lam_f * y[o:o + M.nrows]) + np.asarray(v[i], dtype=np.float64).reshape(-1) / sigma ** 2
        Lc = np.linalg.cholesky(H)
        x = np.linalg.solve(Lc.T, np.linalg.solve(Lc, b))
        xs.append(x.reshape(geom.nz, geom.ny, geom.nx))
        o += M.nrows
    return np.stack(xs)


def project_rays(geom, frame, views, ivs, ius, x_frame):
    """Siddon projection of selected rays of one frame; views are frame-local."""
    a0, a1 = int(geom.view_offset[frame]), int(geom.view_offset[frame + 1])
    ang = np.ascontiguousarray(geom.angles[a0:a1], dtype=np.float64)
    vw = np.ascontiguousarray(views, dtype=np.int32)
    iv = np.ascontiguousarray(ivs, dtype=np.int32)
    iu = np.ascontiguousarray(ius, dtype=np.int32)
    x = np.ascontiguousarray(x_frame, dtype=np.float64).reshape(-1)
    out = np.zeros(len(vw))
    lib().or_project_rays(C.byref(cgeom(geom)), _p(ang, C.c_double), _p(vw, C.c_int32), _p(iv, C.c_int32),
                          _p(iu, C.c_int32), len(vw), _p(x, C.c_double), _p(out, C.c_double))
    return out


def backproject_voxels(geom, frame, y_frame, voxels):
    """(A^T y)_j of one frame at selected voxel indices j (slab test per ray)."""
    a0, a1 = int(geom.view_offset[frame]), int(geom.view_offset[frame + 1])
    ang = np.ascontiguousarray(geom.angles[a0:a1], dtype=np.float64)
    y = np.ascontiguousarray(y_frame, dtype=np.float64).reshape(-1)
    vx = np.ascontiguousarray(voxels, dtype=np.int64)
    out = np.zeros(len(vx))
    lib().or_backproject_voxels(C.byref(cgeom(geom)), _p(ang, C.c_double), a1 - a0, _p(y, C.c_double),
                                _p(vx, C.c_int64), len(vx), _p(out, C.c_double))
    return out


def voxel_columns(geom, frame, voxels, cap=4096):
    """Columns of one frame's A at selected voxels: [(ray indices, lengths)] with
    frame-local ray index view*nv*nu + iv*nu + iu (slab test against every ray)."""
    a0, a1 = int(geom.view_offset[frame]), int(geom.view_offset[frame + 1])
    ang = np.ascontiguousarray(geom.angles[a0:a1], dtype=np.float64)
    vx = np.ascontiguousarray(voxels, dtype=np.int64)
    cnt = np.zeros(len(vx), dtype=np.int32)
    ray = np.zeros(len(vx) * cap, dtype=np.int64)
    ln = np.zeros(len(vx) * cap)
    lib().or_voxel_columns(C.byref(cgeom(geom)), _p(ang, C.c_double), a1 - a0, _p(vx, C.c_int64), len(vx),
                           _p(cnt, C.c_int32), _p(ray, C.c_int64), _p(ln, C.c_double), cap)
    if (cnt > cap).any():
        raise ValueError("voxel column longer than cap")
    return [(ray[s * cap:s * cap + cnt[s]].copy(), ln[s * cap:s * cap + cnt[s]].copy()) for s in range(len(vx))]


def project_ray_ids(geom, frame, rays, x_frame):
    """Siddon projection of frame-local ray indices (view*nv*nu + iv*nu + iu)."""
    rays = np.asarray(rays, dtype=np.int64)
    view, rem = np.divmod(rays, geom.nu * geom.nv)
    iv, iu = np.divmod(rem, geom.nu)
    return project_rays(geom, frame, view, iv, iu, x_frame)


def gradient_at_voxels(geom, frame, voxels, x, v, y, lam, sigma):
    """Components j of the proximal objective's gradient
    A^T Lambda (A x - y) + (x - v) / sigma^2 of one frame, and of b = A^T Lambda y + v / sigma^2,
    at selected voxels (FP64; x, v [nvox], y, lam the frame's sinogram)."""
    cols = voxel_columns(geom, frame, voxels)
    rays = np.unique(np.concatenate([c[0] for c in cols])) if cols else np.zeros(0, np.int64)
    ax = dict(zip(rays.tolist(), project_ray_ids(geom, frame, rays, x).tolist()))
    x = np.asarray(x, dtype=np.float64).reshape(-1)
    v = np.asarray(v, dtype=np.float64).reshape(-1)
    grad = np.zeros(len(voxels))
    b = np.zeros(len(voxels))
    for s, (rr, ll) in enumerate(cols):
        axr = np.array([ax[r] for r in rr.tolist()])
        grad[s] = np.sum(ll * lam[rr] * (axr - y[rr])) + (x[voxels[s]] - v[voxels[s]]) / sigma ** 2
        b[s] = np.sum(ll * lam[rr] * y[rr]) + v[voxels[s]] / sigma ** 2
    return grad, b


def make_measurement(cfg, geom, x0, frames=None):
    """Noisy sinogram and weights for the given frames: y_clean = A x0 (oracle
    projector), then the generator's noise/weight recipe."""
    from paper_2008_01567_amd import synth
    fr = _frames(geom, frames)
    yc = project(geom, x0, fr)
    eps = synth.noise_eps(cfg, geom, fr)
    counts = [geom.views_of(f) for f in fr]
    return synth.finish_measurement(yc, eps, counts, geom.n_rays_per_view, model=cfg.weights)
