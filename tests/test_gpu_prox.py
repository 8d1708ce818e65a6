"""GPU parity of the batched proximal-map solve against the FP64 oracle."""
import numpy as np
import pytest

import oracle
from paper_2008_01567_amd import synth
from _problems import oracle_solution, problem, rel_l2

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


def _solve(msf, name, **kw):
    cfg, g, x0, v, y, lam = problem(name)
    plan = msf.Plan(g)
    x, st = plan.prox_solve(_dev(v), _dev(y), _dev(lam), cfg.sigma, **kw)
    return cfg, g, x.cpu().numpy(), st


# frozen stopping rule per workload: the recursive residual that brings the relative
# error to <= 1e-4 (the limited-angle arcs of c3s are the worst conditioned).  The
# tall volumes (nz 150 and 230) run the adjoint fused with the CG update at 3 and 4 z
# voxels per lane, the instantiation that the 256^3 and 512x512x256 solves use.  At nz 300 (two
# z-chunks per voxel column) plain FP32 CG stalls at a true residual of 1.1e-5, an error of about
# 1e-4 (the FP32 floor, as the fused and the unfused update paths both show); that workload is
# solved with iterative refinement (the FP64 residual every 512 steps; observed 3.1e-8).
REFINE = {"tall5": 512}


@pytest.mark.parametrize("name,tol", [("c1", 1e-8), ("c2s", 1e-6), ("c3s", 1e-7), ("tall3", 1e-8),
                                      ("tall4", 1e-8), ("tall5", 1e-8), ("odd", 1e-8), ("level", 1e-8), ("steep", 1e-8),
                                      ("steeper", 1e-8), ("flat", 1e-8)])
def test_prox_matches_oracle(msf, name, tol):
    print("case", name, flush=True)
    cfg, g, x, st = _solve(msf, name, tol=tol, max_iter=5000 + 15000 * (name in REFINE), true_residual=True,
                           refine_every=REFINE.get(name, 0))
    xs, ost = oracle_solution(name)
    errs = [rel_l2(x[f], xs[f]) for f in range(g.n_frames)]
    print(name, "iters", st["iters"].tolist(), "oracle", [s["iters"] for s in ost], "err", errs,
          "true", st["true_rel_residual"].tolist(), flush=True)
    assert st["status"] == msf.MSF_OK and st["converged"].all()
    assert max(errs) <= 1e-4


def test_paper_weight_model_with_refinement_meets_1e4(msf):
    """Iterative refinement (the iterate in FP64, its residual from the FP64 operator every
    2048 CG steps, FP32 CG for each correction) removes the FP32 floor below: the paper's
    weights reach 1e-4 against the FP64 oracle (observed 3.9e-6 at tol 1e-8)."""
    from paper_2008_01567_amd.calibration import REFINED
    tol, every = REFINED["c2sp"]
    cfg, g, x, st = _solve(msf, "c2sp", tol=tol, max_iter=30000, check_every=16, refine_every=every)
    xs, _ = oracle_solution("c2sp", tol=1e-11)
    errs = [rel_l2(x[f], xs[f]) for f in range(g.n_frames)]
    print("c2sp refined: iters", st["iters"].tolist(), "FP64 residual", st["true_rel_residual"].tolist(),
          "err", errs, flush=True)
    assert st["status"] == msf.MSF_OK and st["converged"].all()
    assert (st["true_rel_residual"] <= tol).all()
    assert max(errs) <= 1e-4


def test_refinement_on_a_plain_workload(msf):
    """On the 32^3 workload refinement changes nothing but the accuracy: the FP64 residual
    meets tol and the error falls well below the plain solve's (observed 2.9e-8 vs 8.9e-6)."""
    cfg, g, xp, sp = _solve(msf, "c1", tol=1e-8, max_iter=4000)
    _, _, xr, sr = _solve(msf, "c1", tol=1e-8, max_iter=4000, refine_every=256)
    xs, _ = oracle_solution("c1")
    ep = max(rel_l2(xp[f], xs[f]) for f in range(g.n_frames))
    er = max(rel_l2(xr[f], xs[f]) for f in range(g.n_frames))
    print("c1 plain err", ep, "refined err", er, "iters", sp["iters"].tolist(), sr["iters"].tolist(), flush=True)
    assert sr["status"] == msf.MSF_OK and (sr["true_rel_residual"] <= 1e-8).all()
    assert er <= 1e-6 and er < ep


def test_paper_weight_model_reaches_the_fp32_floor(msf):
    """The paper's weights Lambda = exp(-A x0) / s^2 make the system far stiffer (about 8x
    the iterations); at the frozen rule the error reaches the FP32 floor of such systems,
    2-4e-4 against the FP64 oracle (tighter tolerances do not lower it), not 1e-4."""
    from paper_2008_01567_amd.calibration import FROZEN_TOL
    cfg, g, x, st = _solve(msf, "c2sp", tol=FROZEN_TOL["c2sp"], max_iter=20000)
    xs, _ = oracle_solution("c2sp", tol=1e-11)
    errs = [rel_l2(x[f], xs[f]) for f in range(g.n_frames)]
    print("c2sp iters", st["iters"].tolist(), "err", errs, flush=True)
    assert st["status"] == msf.MSF_OK
    assert max(errs) <= 5e-4


def test_graph_equals_eager(msf):
    """The same 300 CG steps replayed from captured graphs and launched eagerly."""
    cfg, g, xa, sa = _solve(msf, "c2s", tol=0.0, max_iter=300, check_every=16, use_graph=True)
    _, _, xb, sb = _solve(msf, "c2s", tol=0.0, max_iter=300, check_every=16, use_graph=False)
    assert (sa["iters"] == 300).all() and (sb["iters"] == 300).all()
    assert rel_l2(xa, xb) <= 1e-5


def test_repeated_solves_replay_the_graph(msf):
    """A plan captures its CG steps once and replays the graph in later solves: three solves on
    one plan (inputs a, b, a, with other device work and synchronisations between them) equal
    fresh plans' solves bit for bit, iteration counts included."""
    cfg, g, x0, v, y, lam = problem("c2s")
    rng = np.random.default_rng(2024)
    v2 = (v + 0.01 * rng.standard_normal(v.shape)).astype(np.float32).astype(np.float64)
    y2 = (y * (1.0 + 0.01 * rng.standard_normal(y.shape))).astype(np.float32).astype(np.float64)

    def solve(plan, vv, yy):
        x, st = plan.prox_solve(_dev(vv), _dev(yy), _dev(lam), cfg.sigma, tol=1e-6, max_iter=3000, check_every=8)
        return x.cpu().numpy(), st["iters"].copy()

    want = {}
    for key, vv, yy in (("a", v, y), ("b", v2, y2)):
        fresh = msf.Plan(g)
        want[key] = solve(fresh, vv, yy)
        fresh.close()
    assert not np.array_equal(want["a"][0], want["b"][0])
    plan = msf.Plan(g)
    for key, vv, yy in (("a", v, y), ("b", v2, y2), ("a", v, y)):
        junk = torch.randn(1 << 20, device="cuda")
        junk.mul_(2.0).sum().item()   # eager work between the solves
        x, iters = solve(plan, vv, yy)
        print(key, "iters", iters.tolist(), flush=True)
        assert np.array_equal(iters, want[key][1])
        assert np.array_equal(x, want[key][0])


def test_table_and_on_the_fly_gather_give_identical_solves(msf):
    """The CG solve with the voxel-driven adjoint reading the cell table (default) and
    computing the pieces on the fly: the same arithmetic in the same order, bit for bit."""
    cfg, g, x0, v, y, lam = problem("c2s")
    out = []
    for bm in (2, 1):
        plan = msf.Plan(g)
        plan.set_tiles(back_mode=bm)
        x, st = plan.prox_solve(_dev(v), _dev(y), _dev(lam), cfg.sigma, tol=1e-6, max_iter=3000)
        out.append((x.cpu().numpy(), st["iters"]))
    assert np.array_equal(out[0][1], out[1][1])
    assert np.array_equal(out[0][0], out[1][0])


def test_batched_equals_per_frame(msf):
    name = "c3s"
    cfg, g, x0, v, y, lam = problem(name)
    plan = msf.Plan(g)
    xb, _ = plan.prox_solve(_dev(v), _dev(y), _dev(lam), cfg.sigma, tol=0.0, max_iter=400)
    xb = xb.cpu().numpy()
    for f in (0, g.n_frames - 1):
        gs = g.subset([f])
        s = g.sino_slice(f)
        p1 = msf.Plan(gs)
        x1, _ = p1.prox_solve(_dev(v[f:f + 1]), _dev(y[s]), _dev(lam[s]), cfg.sigma, tol=0.0, max_iter=400)
        assert rel_l2(x1.cpu().numpy()[0], xb[f]) <= 1e-5


def test_frame_shards_equal_batch(msf):
    """The frames split into two shards (as across two GPUs: separate plans, no
    exchange) give the batched result on every frame."""
    name = "c3s"
    cfg, g, x0, v, y, lam = problem(name)
    xb, _ = msf.Plan(g).prox_solve(_dev(v), _dev(y), _dev(lam), cfg.sigma, tol=0.0, max_iter=300)
    xb = xb.cpu().numpy()
    half = g.n_frames // 2
    for frames in (list(range(half)), list(range(half, g.n_frames))):
        gs = g.subset(frames)
        ys = np.concatenate([y[g.sino_slice(f)] for f in frames])
        ls = np.concatenate([lam[g.sino_slice(f)] for f in frames])
        xs, _ = msf.Plan(gs).prox_solve(_dev(v[frames]), _dev(ys), _dev(ls), cfg.sigma, tol=0.0, max_iter=300)
        xs = xs.cpu().numpy()
        for i, f in enumerate(frames):
            assert rel_l2(xs[i], xb[f]) <= 1e-5, (frames, f)


def test_special_cases(msf):
    cfg, g, x0, v, y, lam = problem("c1")
    plan = msf.Plan(g)
    # Lambda = 0: L(v) = v with zero iterations
    x, st = plan.prox_solve(_dev(v), _dev(y), _dev(np.zeros_like(lam)), cfg.sigma, tol=1e-8)
    assert np.array_equal(x.cpu().numpy(), v.astype(np.float32)) and (st["iters"] == 0).all()
    # y = A v (the GPU's own projection): v is the minimiser
    vy = plan.project(_dev(v))
    x, st = plan.prox_solve(_dev(v), vy, _dev(lam), cfg.sigma, tol=1e-8)
    assert rel_l2(x.cpu().numpy(), v) <= 1e-5
    # max_iter = 0 returns v and reports non-convergence
    x, st = plan.prox_solve(_dev(v), _dev(y), _dev(lam), cfg.sigma, tol=1e-8, max_iter=0)
    assert st["status"] == msf.MSF_NOT_CONVERGED and np.array_equal(x.cpu().numpy(), v.astype(np.float32))


def test_invalid_inputs_rejected(msf):
    cfg, g, x0, v, y, lam = problem("c1")
    plan = msf.Plan(g)
    bad = lam.copy()
    bad[5] = -1.0
    out = torch.full(plan.vol_shape, 7.0, device="cuda")
    with pytest.raises(msf.MsfError) as e:
        plan.prox_solve(_dev(v), _dev(y), _dev(bad), cfg.sigma, out=out)
    assert e.value.status == msf.MSF_EINVAL and "lambda" in str(e.value)
    assert (out == 7.0).all()          # outputs untouched on EINVAL
    with pytest.raises(msf.MsfError):
        plan.prox_solve(_dev(v), _dev(y), _dev(lam), 0.0)
