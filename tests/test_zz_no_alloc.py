"""The allocation-free fixture correction (msf_fixture_correct_noalloc) against
the allocating entry point (msf_fixture_correct) through the C ABI: the same
kernels on the same inputs, so the corrected sinograms and the per-frame fits
must agree bit for bit.  Two calls in a row, the second on a smaller problem
(the shared scratch still holds the first call's values beyond it); a
geometry whose scratch would exceed the limit is rejected before any device
work, its output untouched."""
import ctypes as C

import numpy as np
import pytest

from paper_2008_01567_amd import synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def msf():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2008_01567_amd import msf as m
    m.lib()
    return m


def _inputs(name, seed):
    cfg = synth.config(name)
    g = synth.make_geometry(cfg)
    x = synth.make_phantom(cfg, dtype=np.float32)
    rng = np.random.default_rng(seed)
    y = (1.0 + 0.1 * rng.standard_normal(g.n_views * g.n_rays_per_view)).astype(np.float32)
    return cfg, g, torch.from_numpy(x).cuda(), torch.from_numpy(y).cuda()


@pytest.mark.parametrize("name,radius,std", [("c1", 14.0, 1.5), ("tiny16", 7.0, 1.0)])
def test_noalloc_equals_allocating_entry_point(msf, name, radius, std):
    """Run for c1 (32^3 x 4, 73,728 rays) first, then for the smaller 16^3 x 2."""
    print("case", name, flush=True)
    cfg, g, x, y = _inputs(name, 3)
    plan = msf.Plan(g)
    ref, c_ref = plan.fixture_correct(x, y, radius, std)
    out = torch.full_like(ref, float("nan"))
    got, c = plan.fixture_correct_noalloc(x, y, radius, std, out=out)
    torch.cuda.synchronize()
    print(name, "c", c.tolist(), flush=True)
    assert torch.equal(got, ref)
    assert np.array_equal(c, c_ref)
    assert np.all(np.isfinite(c)) and np.any(c != 0.0)
    plan.close()


def test_noalloc_rejects_oversize_geometry(msf):
    """480 views of a 192^2 detector need 71 MB of scratch, above the 64 MiB limit."""
    views = 480
    off = np.array([0, views], dtype=np.int64)
    ang = np.linspace(0.0, np.pi, views, endpoint=False)
    g = synth.Geometry(8, 8, 8, 1, 192, 192, 2.0, 2.0, 50.0, 100.0, off, ang)
    plan = msf.Plan(g)
    x = torch.zeros(g.n_vox, device="cuda")
    y = torch.ones(g.n_views * g.n_rays_per_view, device="cuda")
    out = torch.full_like(y, 7.0)
    c = np.full(1, -1.0)
    st = msf.lib().msf_fixture_correct_noalloc(plan._h, C.c_void_p(x.data_ptr()), C.c_void_p(y.data_ptr()), 4.0,
                                               1.0, C.c_void_p(out.data_ptr()),
                                               c.ctypes.data_as(C.POINTER(C.c_double)), None)
    assert st == msf.MSF_EINVAL
    assert "scratch" in msf.last_error()
    torch.cuda.synchronize()
    assert bool((out == 7.0).all()) and c[0] == -1.0
    plan.close()
