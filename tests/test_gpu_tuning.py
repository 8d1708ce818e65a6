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
