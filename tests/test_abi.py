"""C ABI: libmsf.so loads, exports every symbol include/msf.h declares, and
rejects invalid geometries on the host before touching the GPU."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from paper_2008_01567_amd import msf

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "msf.h")).read()
    return sorted(set(re.findall(r"\b(msf_[a-z0-9_]+)\s*\(", src)))


def test_header_and_binding_agree():
    assert sorted(msf.EXPORTS) == _declared()


def test_library_exports_every_symbol():
    L = msf.lib()
    for name in _declared():
        assert hasattr(L, name), name
    assert L.msf_version().startswith(b"msf")


def _geom(**kw):
    d = dict(nx=8, ny=8, nz=8, n_frames=1, nu=12, nv=12, du=2.0, dv=2.0, src_iso=50.0, src_det=100.0,
             det_off_u=0.0, det_off_v=0.0)
    d.update(kw)
    vo = np.array(kw.pop("vo", [0, 2]), dtype=np.int64)
    an = np.array([0.1, 0.2])
    g = msf.msf_geometry(*[d[k] for k in ("nx", "ny", "nz", "n_frames", "nu", "nv", "du", "dv", "src_iso",
                                          "src_det", "det_off_u", "det_off_v")],
                         vo.ctypes.data_as(C.POINTER(C.c_int64)), an.ctypes.data_as(C.POINTER(C.c_double)))
    return g, vo, an


@pytest.mark.parametrize("bad", [dict(nx=0), dict(n_frames=0), dict(du=-1.0), dict(src_iso=4.0),
                                 dict(src_det=55.0), dict(dv=float("nan"))])
def test_plan_create_rejects_bad_geometry(bad):
    g, vo, an = _geom(**bad)
    h = C.c_void_p()
    st = msf.lib().msf_plan_create(C.byref(g), C.byref(h))
    assert st == msf.MSF_EINVAL and h.value is None
    assert msf.last_error() != ""


def test_plan_create_rejects_bad_view_offset():
    g, vo, an = _geom()
    vo[:] = [1, 2]
    h = C.c_void_p()
    assert msf.lib().msf_plan_create(C.byref(g), C.byref(h)) == msf.MSF_EINVAL


def test_solve_rejects_null_plan_and_defaults():
    o = msf.msf_solve_opts()
    msf.lib().msf_solve_opts_default(C.byref(o))
    assert o.tol == 1e-6 and o.max_iter == 1000 and o.check_every == 8 and o.use_graph == 1
    st = msf.lib().msf_prox_solve(None, None, None, None, 0.5, None, None, None, None)
    assert st == msf.MSF_EINVAL


@pytest.mark.parametrize("bad", [dict(nx=1 << 11, ny=1 << 11, nz=1 << 10, src_iso=3000.0, src_det=6000.0),
                                 dict(det_off_u=float("inf"))])
def test_plan_create_rejects_oversize_and_non_finite(bad):
    g, vo, an = _geom(**bad)
    h = C.c_void_p()
    assert msf.lib().msf_plan_create(C.byref(g), C.byref(h)) == msf.MSF_EINVAL and h.value is None


def test_plan_create_rejects_bad_angles():
    g, vo, an = _geom()
    an[1] = float("nan")
    h = C.c_void_p()
    assert msf.lib().msf_plan_create(C.byref(g), C.byref(h)) == msf.MSF_EINVAL
    g.angles = None
    assert msf.lib().msf_plan_create(C.byref(g), C.byref(h)) == msf.MSF_EINVAL
    assert "angle" in msf.last_error()


def test_entry_points_reject_null_handles():
    """Every call on a plan or a network checks its handle before any device work."""
    L = msf.lib()
    t = msf.msf_tiles()
    tm = msf.msf_timing()
    mo = msf.msf_mace_opts()
    L.msf_mace_opts_default(C.byref(mo))
    calls = {
        "msf_project": lambda: L.msf_project(None, None, None, None),
        "msf_backproject": lambda: L.msf_backproject(None, None, None, None),
        "msf_prox_features": lambda: L.msf_prox_features(None, None, None, None, 0.5, None, None),
        "msf_plan_set_tiles": lambda: L.msf_plan_set_tiles(None, C.byref(t)),
        "msf_plan_get_tiles": lambda: L.msf_plan_get_tiles(None, C.byref(t)),
        "msf_plan_sizes": lambda: L.msf_plan_sizes(None, None, None, None),
        "msf_plan_set_timing": lambda: L.msf_plan_set_timing(None, 1),
        "msf_plan_get_timing": lambda: L.msf_plan_get_timing(None, C.byref(tm)),
        "msf_plan_autotune": lambda: L.msf_plan_autotune(None, None, None, None),
        "msf_count_intersections": lambda: L.msf_count_intersections(None, None, None),
        "msf_fixture_correct": lambda: L.msf_fixture_correct(None, None, None, 10.0, 1.0, None, None, None),
        "msf_fixture_correct_noalloc": lambda: L.msf_fixture_correct_noalloc(None, None, None, 10.0, 1.0, None, None,
                                                                             None),
        "msf_mace_run": lambda: L.msf_mace_run(None, None, None, None, 0.5, C.byref(mo), None, None, None),
        "msf_cnn_get_params": lambda: L.msf_cnn_get_params(None, None),
        "msf_cnn_infer": lambda: L.msf_cnn_infer(None, None, None, 1, 1, 8, 8, None, None),
        "msf_cnn_train_step": lambda: L.msf_cnn_train_step(None, None, None, None, 1, 1, 8, 8, 1e-3, 1, None,
                                                           None, None),
        "msf_denoise25": lambda: L.msf_denoise25(None, None, 1, 8, 8, 8, 1, None, None),
    }
    for name, call in calls.items():
        assert call() == msf.MSF_EINVAL, name
        assert msf.last_error() != "", name
    assert L.msf_cnn_kind(None) == -1 and L.msf_cnn_n_params(None) == 0
    L.msf_plan_destroy(None)
    L.msf_cnn_destroy(None)


@pytest.mark.parametrize("create,n,nsc", [("msf_cnn_create", msf.N_CNN_PARAMS, 3),
                                          ("msf_cnn_create_denoiser", msf.N_DENOISER_PARAMS, 2)])
def test_network_create_validates(create, n, nsc):
    fn = getattr(msf.lib(), create)
    p = np.zeros(n, dtype=np.float32)
    sc = np.ones(3, dtype=np.float32)
    P = lambda a: a.ctypes.data_as(C.POINTER(C.c_float))
    h = C.c_void_p()
    assert fn(P(p), n - 1, P(sc), C.byref(h)) == msf.MSF_EINVAL and h.value is None    # wrong count
    bad = sc.copy()
    bad[nsc - 1] = 0.0
    assert fn(P(p), n, P(bad), C.byref(h)) == msf.MSF_EINVAL                            # scale <= 0
    pn = p.copy()
    pn[n // 2] = np.nan
    assert fn(P(pn), n, P(sc), C.byref(h)) == msf.MSF_EINVAL and h.value is None        # non-finite weight
    assert "msf_cnn_create" in msf.last_error()


def test_mace_defaults():
    o = msf.msf_mace_opts()
    msf.lib().msf_mace_opts_default(C.byref(o))
    assert (o.n_iter, o.prior, o.partial_iters, o.max_iter) == (10, msf.MSF_PRIOR_PLANE_GAUSS, 0, 2000)
    assert (o.beta, o.rho, o.prior_param, o.tol) == (1.0, 0.5, 1.0, 1e-6)
    assert not o.cnn and not o.prior_cnn
