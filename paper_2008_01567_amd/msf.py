"""Python binding of libmsf.so (argument marshalling only).

Every step of the computation runs in the HIP library; this module turns
torch tensors into device pointers and the current HIP stream, and C status
codes into exceptions.  The names follow include/msf.h.

If ``libmsf.so`` has not been built, importing works but every call raises:
there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmsf.so")

MSF_OK, MSF_NOT_CONVERGED, MSF_CNN_FALLBACK = 0, 1, 2
MSF_EINVAL, MSF_ENOMEM, MSF_EHIP, MSF_EBREAKDOWN = -1, -2, -3, -4
MSF_X0_V, MSF_X0_USER, MSF_X0_CNN = 0, 1, 2
STATUS_NAMES = {0: "MSF_OK", 1: "MSF_NOT_CONVERGED", 2: "MSF_CNN_FALLBACK", -1: "MSF_EINVAL",
                -2: "MSF_ENOMEM", -3: "MSF_EHIP", -4: "MSF_EBREAKDOWN"}


class MsfError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("%s: %s" % (STATUS_NAMES.get(status, status), msg))
        self.status = status


class msf_geometry(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32), ("n_frames", C.c_int32),
                ("nu", C.c_int32), ("nv", C.c_int32), ("du", C.c_double), ("dv", C.c_double),
                ("src_iso", C.c_double), ("src_det", C.c_double), ("det_off_u", C.c_double),
                ("det_off_v", C.c_double), ("view_offset", C.POINTER(C.c_int64)),
                ("angles", C.POINTER(C.c_double))]


class msf_tiles(C.Structure):
    _fields_ = [("rays_per_lane", C.c_int32), ("waves_per_group", C.c_int32), ("back_mode", C.c_int32),
                ("xcd_remap", C.c_int32)]


class msf_solve_opts(C.Structure):
    _fields_ = [("tol", C.c_double), ("max_iter", C.c_int32), ("check_every", C.c_int32),
                ("x0_mode", C.c_int32), ("use_graph", C.c_int32), ("true_residual", C.c_int32),
                ("refine_every", C.c_int32), ("x0", C.c_void_p), ("cnn", C.c_void_p)]


class msf_solve_stats(C.Structure):
    _fields_ = [("iters", C.POINTER(C.c_int32)), ("rel_residual", C.POINTER(C.c_double)),
                ("true_rel_residual", C.POINTER(C.c_double)), ("converged", C.POINTER(C.c_uint8)),
                ("cnn_used", C.POINTER(C.c_uint8)), ("start_rel_residual", C.POINTER(C.c_double)),
                ("steps", C.c_int32), ("reserved", C.c_int32),
                ("seconds", C.c_double)]


class msf_mace_opts(C.Structure):
    _fields_ = [("n_iter", C.c_int32), ("prior", C.c_int32), ("partial_iters", C.c_int32), ("max_iter", C.c_int32),
                ("beta", C.c_double), ("rho", C.c_double), ("prior_param", C.c_double), ("tol", C.c_double),
                ("cnn", C.c_void_p), ("prior_cnn", C.c_void_p)]


class msf_mace_stats(C.Structure):
    _fields_ = [("cg_iters", C.POINTER(C.c_int64)), ("capacity", C.c_int32), ("reserved", C.c_int32),
                ("cg_total", C.c_int64), ("seconds", C.c_double)]


MSF_PRIOR_PLANE_GAUSS, MSF_PRIOR_RIDGE, MSF_PRIOR_CNN = 0, 1, 2


class msf_timing(C.Structure):
    _fields_ = [("forward_ms", C.c_double), ("forward_launches", C.c_int64), ("back_ms", C.c_double),
                ("back_launches", C.c_int64)]


_lib = None

# every symbol the header declares (checked by the ABI test)
EXPORTS = ["msf_solve_opts_default", "msf_plan_create", "msf_plan_destroy", "msf_plan_set_tiles",
           "msf_plan_get_tiles", "msf_plan_sizes", "msf_project", "msf_backproject", "msf_prox_solve",
           "msf_last_error", "msf_version", "msf_plan_set_timing", "msf_plan_get_timing",
           "msf_count_intersections", "msf_prox_features", "msf_cnn_create", "msf_cnn_destroy",
           "msf_cnn_get_params", "msf_cnn_infer", "msf_cnn_train_step", "msf_mace_opts_default", "msf_mace_run", "msf_plan_autotune",
           "msf_fixture_correct", "msf_fixture_correct_noalloc", "msf_cnn_create_denoiser", "msf_cnn_kind", "msf_cnn_n_params", "msf_denoise25"]


def lib():
    """Load libmsf.so (raises if it is missing: there is no fallback)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libmsf.so is not built (python -m paper_2008_01567_amd.build)")
        L = C.CDLL(LIB_PATH)
        vp = C.c_void_p
        L.msf_last_error.restype = C.c_char_p
        L.msf_version.restype = C.c_char_p
        L.msf_solve_opts_default.argtypes = [C.POINTER(msf_solve_opts)]
        L.msf_plan_create.argtypes = [C.POINTER(msf_geometry), C.POINTER(vp)]
        L.msf_plan_destroy.argtypes = [vp]
        L.msf_plan_set_tiles.argtypes = [vp, C.POINTER(msf_tiles)]
        L.msf_plan_get_tiles.argtypes = [vp, C.POINTER(msf_tiles)]
        L.msf_plan_sizes.argtypes = [vp, C.POINTER(C.c_int64), C.POINTER(C.c_int64), C.POINTER(C.c_int64)]
        L.msf_project.argtypes = [vp, vp, vp, vp]
        L.msf_backproject.argtypes = [vp, vp, vp, vp]
        L.msf_prox_solve.argtypes = [vp, vp, vp, vp, C.c_double, C.POINTER(msf_solve_opts), vp,
                                     C.POINTER(msf_solve_stats), vp]
        L.msf_plan_set_timing.argtypes = [vp, C.c_int32]
        L.msf_plan_get_timing.argtypes = [vp, C.POINTER(msf_timing)]
        L.msf_count_intersections.argtypes = [vp, C.POINTER(C.c_int64), vp]
        L.msf_fixture_correct.argtypes = [vp, vp, vp, C.c_double, C.c_double, vp, C.POINTER(C.c_double), vp]
        L.msf_fixture_correct_noalloc.argtypes = L.msf_fixture_correct.argtypes
        L.msf_prox_features.argtypes = [vp, vp, vp, vp, C.c_double, vp, vp]
        L.msf_mace_opts_default.argtypes = [C.POINTER(msf_mace_opts)]
        L.msf_plan_autotune.argtypes = [vp, C.c_char_p, C.POINTER(msf_tiles), vp]
        L.msf_mace_run.argtypes = [vp, vp, vp, vp, C.c_double, C.POINTER(msf_mace_opts), vp,
                                   C.POINTER(msf_mace_stats), vp]
        L.msf_cnn_create.argtypes = [C.POINTER(C.c_float), C.c_int64, C.POINTER(C.c_float), C.POINTER(vp)]
        L.msf_cnn_create_denoiser.argtypes = [C.POINTER(C.c_float), C.c_int64, C.POINTER(C.c_float), C.POINTER(vp)]
        L.msf_cnn_destroy.argtypes = [vp]
        L.msf_cnn_kind.argtypes = [vp]
        L.msf_cnn_n_params.argtypes = [vp]
        L.msf_cnn_n_params.restype = C.c_int64
        L.msf_denoise25.argtypes = [vp, vp, C.c_int32, C.c_int32, C.c_int32, C.c_int32, C.c_int32, vp, vp]
        L.msf_cnn_get_params.argtypes = [vp, C.POINTER(C.c_float)]
        L.msf_cnn_infer.argtypes = [vp, vp, vp, C.c_int32, C.c_int32, C.c_int32, C.c_int32, vp, vp]
        L.msf_cnn_train_step.argtypes = [vp, vp, vp, vp, C.c_int32, C.c_int32, C.c_int32, C.c_int32, C.c_double,
                                         C.c_int32, C.POINTER(C.c_double), C.POINTER(C.c_float), vp]
        for name in EXPORTS:
            if name not in ("msf_last_error", "msf_version", "msf_plan_destroy", "msf_solve_opts_default",
                            "msf_cnn_destroy", "msf_mace_opts_default", "msf_cnn_n_params"):
                getattr(L, name).restype = C.c_int
        _lib = L
    return _lib


def last_error() -> str:
    return lib().msf_last_error().decode()


def _check(status):
    if status < 0:
        raise MsfError(status, last_error())
    return status


def _stream(stream):
    if stream is None:
        import torch
        return C.c_void_p(torch.cuda.current_stream().cuda_stream)
    return C.c_void_p(int(stream))


def _ptr(t, numel=None):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != torch.float32 or not t.is_contiguous():
        raise TypeError("expected a contiguous float32 device tensor")
    if numel is not None and t.numel() != numel:
        raise ValueError("expected %d elements, got %d" % (numel, t.numel()))
    return C.c_void_p(t.data_ptr())


class Plan:
    """A plan for one scan geometry (``geom`` has the fields of msf_geometry;
    ``paper_2008_01567_amd.synth.Geometry`` works)."""

    def __init__(self, geom):
        self._vo = np.ascontiguousarray(geom.view_offset, dtype=np.int64)
        self._an = np.ascontiguousarray(geom.angles, dtype=np.float64)
        g = msf_geometry(geom.nx, geom.ny, geom.nz, geom.n_frames, geom.nu, geom.nv, geom.du, geom.dv,
                         geom.src_iso, geom.src_det, geom.det_off_u, geom.det_off_v,
                         self._vo.ctypes.data_as(C.POINTER(C.c_int64)),
                         self._an.ctypes.data_as(C.POINTER(C.c_double)))
        h = C.c_void_p()
        _check(lib().msf_plan_create(C.byref(g), C.byref(h)))
        self._h = h
        self.geom = geom
        self.vol_shape = (geom.n_frames, geom.nz, geom.ny, geom.nx)
        self.n_vox = geom.n_frames * geom.nz * geom.ny * geom.nx
        self.n_meas = int(self._vo[-1]) * geom.nv * geom.nu

    def close(self):
        if getattr(self, "_h", None):
            lib().msf_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_tiles(self, rays_per_lane=3, waves_per_group=4, back_mode=2, xcd_remap=1):
        """Set the launch shapes (msf_plan_set_tiles); get_tiles() reads back what the plan keeps."""
        t = msf_tiles(rays_per_lane, waves_per_group, back_mode, xcd_remap)
        _check(lib().msf_plan_set_tiles(self._h, C.byref(t)))

    def autotune(self, cache_path=None, stream=None) -> dict:
        """Time every launch shape on this geometry and keep the fastest (msf_plan_autotune)."""
        t = msf_tiles()
        cp = cache_path.encode() if cache_path else None
        _check(lib().msf_plan_autotune(self._h, cp, C.byref(t), _stream(stream)))
        return {k: getattr(t, k) for k, _ in msf_tiles._fields_}

    def get_tiles(self) -> dict:
        t = msf_tiles()
        _check(lib().msf_plan_get_tiles(self._h, C.byref(t)))
        return {k: getattr(t, k) for k, _ in msf_tiles._fields_}

    def sizes(self) -> dict:
        a, b, c = C.c_int64(), C.c_int64(), C.c_int64()
        _check(lib().msf_plan_sizes(self._h, C.byref(a), C.byref(b), C.byref(c)))
        return {"n_vox": a.value, "n_meas": b.value, "workspace_bytes": c.value}

    def set_timing(self, enable=True):
        _check(lib().msf_plan_set_timing(self._h, int(bool(enable))))

    def get_timing(self) -> dict:
        t = msf_timing()
        _check(lib().msf_plan_get_timing(self._h, C.byref(t)))
        return {k: getattr(t, k) for k, _ in msf_timing._fields_}

    def fixture_correct(self, x, y, mask_radius, blur_std, out=None, stream=None):
        """Blind fixture correction (msf_fixture_correct); returns (y_corr, c per frame)."""
        import torch
        if out is None:
            out = torch.empty(self.n_meas, dtype=torch.float32, device=y.device)
        c = np.zeros(self.geom.n_frames)
        _check(lib().msf_fixture_correct(self._h, _ptr(x, self.n_vox), _ptr(y, self.n_meas), float(mask_radius),
                                         float(blur_std), _ptr(out, self.n_meas),
                                         c.ctypes.data_as(C.POINTER(C.c_double)), _stream(stream)))
        return out, c

    def fixture_correct_noalloc(self, x, y, mask_radius, blur_std, out, stream=None):
        """msf_fixture_correct_noalloc: the same correction with the library's fixed
        scratch and no device allocation (out must be given); returns (out, c)."""
        c = np.zeros(self.geom.n_frames)
        _check(lib().msf_fixture_correct_noalloc(self._h, _ptr(x, self.n_vox), _ptr(y, self.n_meas),
                                                 float(mask_radius), float(blur_std), _ptr(out, self.n_meas),
                                                 c.ctypes.data_as(C.POINTER(C.c_double)), _stream(stream)))
        return out, c

    def count_intersections(self, stream=None) -> np.ndarray:
        out = np.zeros(self.geom.n_frames, dtype=np.int64)
        _check(lib().msf_count_intersections(self._h, out.ctypes.data_as(C.POINTER(C.c_int64)), _stream(stream)))
        return out

    def project(self, x, y=None, stream=None):
        import torch
        if y is None:
            y = torch.empty(self.n_meas, dtype=torch.float32, device=x.device)
        _check(lib().msf_project(self._h, _ptr(x, self.n_vox), _ptr(y, self.n_meas), _stream(stream)))
        return y

    def backproject(self, y, x=None, stream=None):
        import torch
        if x is None:
            x = torch.empty(self.vol_shape, dtype=torch.float32, device=y.device)
        _check(lib().msf_backproject(self._h, _ptr(y, self.n_meas), _ptr(x, self.n_vox), _stream(stream)))
        return x

    def features(self, v, y, lam, sigma, out=None, stream=None):
        """The learned start's residual feature g (msf_prox_features)."""
        import torch
        if out is None:
            out = torch.empty(self.vol_shape, dtype=torch.float32, device=v.device)
        _check(lib().msf_prox_features(self._h, _ptr(v, self.n_vox), _ptr(y, self.n_meas), _ptr(lam, self.n_meas),
                                       float(sigma), _ptr(out, self.n_vox), _stream(stream)))
        return out

    def mace(self, y, lam, sigma, x_init=None, n_iter=10, prior=MSF_PRIOR_PLANE_GAUSS, prior_param=1.0, beta=1.0,
             rho=0.5, partial_iters=0, tol=1e-6, max_iter=2000, cnn=None, prior_cnn=None, out=None, stream=None):
        """Algorithm 1 (msf_mace_run); returns (X_0, stats)."""
        import torch
        if out is None:
            out = torch.empty(self.vol_shape, dtype=torch.float32, device=y.device)
        o = msf_mace_opts()
        lib().msf_mace_opts_default(C.byref(o))
        o.n_iter, o.prior, o.partial_iters, o.max_iter = int(n_iter), int(prior), int(partial_iters), int(max_iter)
        o.beta, o.rho, o.prior_param, o.tol = float(beta), float(rho), float(prior_param), float(tol)
        o.cnn = cnn._h.value if cnn is not None else None
        o.prior_cnn = prior_cnn._h.value if prior_cnn is not None else None
        it = np.zeros(max(n_iter, 1), dtype=np.int64)
        st = msf_mace_stats(it.ctypes.data_as(C.POINTER(C.c_int64)), len(it), 0, 0, 0.0)
        xi = _ptr(x_init, self.n_vox) if x_init is not None else None
        status = _check(lib().msf_mace_run(self._h, xi, _ptr(y, self.n_meas), _ptr(lam, self.n_meas), float(sigma),
                                           C.byref(o), _ptr(out, self.n_vox), C.byref(st), _stream(stream)))
        return out, {"status": status, "cg_iters": it[:n_iter], "cg_total": st.cg_total, "seconds": st.seconds}

    def prox_solve(self, v, y, lam, sigma, tol=1e-6, max_iter=1000, check_every=8, x0=None, use_graph=True,
                   true_residual=False, out=None, stream=None, cnn=None, refine_every=0):
        """Returns (x, stats) with stats a dict of per-frame arrays and the status code."""
        import torch
        nf = self.geom.n_frames
        if out is None:
            out = torch.empty(self.vol_shape, dtype=torch.float32, device=v.device)
        o = msf_solve_opts()
        lib().msf_solve_opts_default(C.byref(o))
        o.tol, o.max_iter, o.check_every = float(tol), int(max_iter), int(check_every)
        o.use_graph, o.true_residual = int(bool(use_graph)), int(bool(true_residual))
        o.refine_every = int(refine_every)
        if x0 is not None:
            o.x0_mode = MSF_X0_USER
            o.x0 = _ptr(x0, self.n_vox).value
        if cnn is not None:
            o.x0_mode = MSF_X0_CNN
            o.cnn = cnn._h.value
        iters = np.zeros(nf, dtype=np.int32)
        rel = np.zeros(nf)
        trel = np.zeros(nf)
        conv = np.zeros(nf, dtype=np.uint8)
        used = np.zeros(nf, dtype=np.uint8)
        rel0 = np.zeros(nf)
        st = msf_solve_stats(iters.ctypes.data_as(C.POINTER(C.c_int32)), rel.ctypes.data_as(C.POINTER(C.c_double)),
                             trel.ctypes.data_as(C.POINTER(C.c_double)), conv.ctypes.data_as(C.POINTER(C.c_uint8)),
                             used.ctypes.data_as(C.POINTER(C.c_uint8)), rel0.ctypes.data_as(C.POINTER(C.c_double)),
                             0, 0, 0.0)
        status = _check(lib().msf_prox_solve(self._h, _ptr(v, self.n_vox), _ptr(y, self.n_meas),
                                             _ptr(lam, self.n_meas), float(sigma), C.byref(o),
                                             _ptr(out, self.n_vox), C.byref(st), _stream(stream)))
        return out, {"status": status, "iters": iters, "rel_residual": rel, "true_rel_residual": trel,
                     "converged": conv.astype(bool), "cnn_used": used.astype(bool), "start_rel_residual": rel0,
                     "steps": st.steps,
                     "seconds": st.seconds}


N_CNN_PARAMS = 15169


class Cnn:
    """The warm-start network (msf_cnn_*).  params: FP32 [15169] (per layer
    W[out][in][3][3][3] then b[out]); scales: c or (c_v, c_g, c_o)."""

    def __init__(self, params, scales):
        p = np.ascontiguousarray(params, dtype=np.float32).reshape(-1)
        sc = np.full(3, scales, dtype=np.float32) if np.isscalar(scales) else np.asarray(scales, dtype=np.float32)
        h = C.c_void_p()
        _check(lib().msf_cnn_create(p.ctypes.data_as(C.POINTER(C.c_float)), p.size,
                                    sc.ctypes.data_as(C.POINTER(C.c_float)), C.byref(h)))
        self._h = h
        self.scales = tuple(float(x) for x in sc)

    def close(self):
        if getattr(self, "_h", None):
            lib().msf_cnn_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def params(self) -> np.ndarray:
        out = np.zeros(N_CNN_PARAMS, dtype=np.float32)
        _check(lib().msf_cnn_get_params(self._h, out.ctypes.data_as(C.POINTER(C.c_float))))
        return out

    def infer(self, v, g, out=None, stream=None):
        import torch
        n, nz, ny, nx = v.shape
        if out is None:
            out = torch.empty_like(v)
        _check(lib().msf_cnn_infer(self._h, _ptr(v), _ptr(g, v.numel()), n, nz, ny, nx, _ptr(out, v.numel()),
                                   _stream(stream)))
        return out

    def train_step(self, v, g, target, lr=1e-3, apply=True, want_grad=False, stream=None):
        n, nz, ny, nx = v.shape
        loss = C.c_double()
        grad = np.zeros(N_CNN_PARAMS, dtype=np.float32) if want_grad else None
        gp = grad.ctypes.data_as(C.POINTER(C.c_float)) if want_grad else None
        _check(lib().msf_cnn_train_step(self._h, _ptr(v), _ptr(g, v.numel()), _ptr(target, v.numel()), n, nz, ny, nx,
                                        float(lr), int(bool(apply)), C.byref(loss), gp, _stream(stream)))
        return loss.value, grad


N_DENOISER_PARAMS = 5521


class Denoiser(Cnn):
    """The 2.5D denoiser of the multi-slice fusion prior agents (paper Sec. IV;
    msf_cnn_create_denoiser).  params: FP32 [5521] (per layer W[out][in][3][3]
    then b[out]); scales: (c_in, c_o)."""

    def __init__(self, params, scales):
        p = np.ascontiguousarray(params, dtype=np.float32).reshape(-1)
        sc = np.asarray(scales, dtype=np.float32).reshape(-1)
        if sc.size != 2:
            raise ValueError("scales must be (c_in, c_o)")
        h = C.c_void_p()
        _check(lib().msf_cnn_create_denoiser(p.ctypes.data_as(C.POINTER(C.c_float)), p.size,
                                             sc.ctypes.data_as(C.POINTER(C.c_float)), C.byref(h)))
        self._h = h
        self.scales = tuple(float(x) for x in sc)

    def params(self) -> np.ndarray:
        out = np.zeros(N_DENOISER_PARAMS, dtype=np.float32)
        _check(lib().msf_cnn_get_params(self._h, out.ctypes.data_as(C.POINTER(C.c_float))))
        return out

    def infer(self, stack, out=None, stream=None):
        """stack [n][5][h][w] (time points t-2 .. t+2) -> denoised centre slices [n][h][w]."""
        import torch
        n, c, h, w = stack.shape
        if c != 5:
            raise ValueError("expected 5 time points per image")
        if out is None:
            out = torch.empty((n, h, w), dtype=stack.dtype, device=stack.device)
        _check(lib().msf_cnn_infer(self._h, _ptr(stack), None, n, 1, h, w, _ptr(out, n * h * w), _stream(stream)))
        return out

    def train_step(self, stack, target, lr=1e-3, apply=True, want_grad=False, stream=None):
        n, c, h, w = stack.shape
        if c != 5:
            raise ValueError("expected 5 time points per image")
        loss = C.c_double()
        grad = np.zeros(N_DENOISER_PARAMS, dtype=np.float32) if want_grad else None
        gp = grad.ctypes.data_as(C.POINTER(C.c_float)) if want_grad else None
        _check(lib().msf_cnn_train_step(self._h, _ptr(stack), None, _ptr(target, n * h * w), n, 1, h, w, float(lr),
                                        int(bool(apply)), C.byref(loss), gp, _stream(stream)))
        return loss.value, grad

    def agent(self, w, plane, out=None, stream=None):
        """H_xy,t (plane 1), H_yz,t (2) or H_zx,t (3) on a [T][nz][ny][nx] volume (msf_denoise25)."""
        import torch
        T, nz, ny, nx = w.shape
        if out is None:
            out = torch.empty_like(w)
        _check(lib().msf_denoise25(self._h, _ptr(w), T, nz, ny, nx, int(plane), _ptr(out, w.numel()),
                                   _stream(stream)))
        return out
