"""Autotuner: the chosen launch shape changes speed only, and the cache reproduces it."""
import numpy as np
import pytest

from _problems import problem, rel_l2

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def msf():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2008_01567_amd import msf as m
    m.lib()
    return m


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def test_autotune_keeps_results_and_caches(msf, tmp_path):
    cfg, g, x0, v, y, lam = problem("c3s")
    plan = msf.Plan(g)
    base_p = plan.project(_dev(x0)).cpu().numpy()
    base_x, _ = plan.prox_solve(_dev(v), _dev(y), _dev(lam), cfg.sigma, tol=1e-7, max_iter=5000)
    cache = str(tmp_path / "tiles.txt")
    t = plan.autotune(cache)
    print("chosen", t, flush=True)
    assert plan.get_tiles() == t
    assert np.array_equal(plan.project(_dev(x0)).cpu().numpy(), base_p)
    x, st = plan.prox_solve(_dev(v), _dev(y), _dev(lam), cfg.sigma, tol=1e-7, max_iter=5000)
    assert rel_l2(x.cpu().numpy(), base_x.cpu().numpy()) <= 1e-4
    # a second plan of the same geometry reads the cache
    plan2 = msf.Plan(g)
    assert plan2.autotune(cache) == t
    assert open(cache).read().count("\n") == 1


def test_autotune_on_steep_rays_keeps_one_ray_per_lane(msf, tmp_path):
    """Rays that cross several z planes inside one xy cell run the general z walk, which is
    compiled for one ray per lane: the autotuner times no other shape, a cached shape that asks
    for more is read back as one, and the result is unchanged."""
    cfg, g, x0, v, y, lam = problem("steep")
    plan = msf.Plan(g)
    base_p = plan.project(_dev(x0)).cpu().numpy()
    cache = str(tmp_path / "tiles.txt")
    t = plan.autotune(cache)
    print("chosen", t, flush=True)
    assert t["rays_per_lane"] == 1 and plan.get_tiles() == t
    assert np.array_equal(plan.project(_dev(x0)).cpu().numpy(), base_p)
    # a cache line written with three rays per lane (say by a hand edit) is normalised on reading
    key = open(cache).read().rsplit(" ", 4)[0]
    with open(cache, "w") as f:
        f.write("%s 3 %d %d %d\n" % (key, t["waves_per_group"], t["back_mode"], t["xcd_remap"]))
    plan2 = msf.Plan(g)
    assert plan2.autotune(cache)["rays_per_lane"] == 1
    assert plan2.get_tiles()["rays_per_lane"] == 1
    assert np.array_equal(plan2.project(_dev(x0)).cpu().numpy(), base_p)
