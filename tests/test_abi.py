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
