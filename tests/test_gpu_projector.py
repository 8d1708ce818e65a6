"""GPU parity of the HIP projector A and backprojector A^T against the FP64 oracle.

The `odd` workload has odd sizes everywhere (voxel planes at half-integers, a voxel straddling
z = 0, the detector centre between pixels) and a detector shifted off the central ray; `level` has a
level middle row (zp = 0) that runs in the voxel face z = 0.  `steep` and `steeper` put the source
close to a tall volume, so that rays cross several z planes inside one xy cell; `flat` is a single
voxel slab; `tall5` (nz 300) splits each voxel column of the gather into two z-chunks."""
import numpy as np
import pytest

import oracle
from paper_2008_01567_amd import synth
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


def _frame_rel(g, got, want):
    errs = []
    for f in range(g.n_frames):
        s = g.sino_slice(f)
        errs.append(rel_l2(got[s], want[s]))
    return max(errs)


@pytest.mark.parametrize("name", ["c1", "c2s", "c3s", "c5s", "tall4", "tall5", "odd", "level"])
def test_project_matches_oracle(msf, name):
    cfg, g, x0, v, y, lam = problem(name)
    print("case", name, flush=True)
    plan = msf.Plan(g)
    if name == "tall5":   # 304 rows meet the volume: one chunk of five rays per lane
        assert plan.get_tiles()["rays_per_lane"] == 5
    want = oracle.project(g, x0)
    got = plan.project(_dev(x0)).cpu().numpy()
    assert _frame_rel(g, got, want) <= 2e-6
    # rows whose ray misses the volume (an empty row of A: zero chord through the box) are
    # exactly zero.  (A ray through a zero-valued region is not such a row: where its xy line
    # runs through a corner shared by four cells, as the central column's does through the
    # rotation axis, the FP32 piece ends near s = 0 can leave a piece of ~1e-16 in a cell the
    # exact line only touches.)
    miss = oracle.project(g, np.ones_like(x0)) == 0.0
    assert miss.any()
    assert np.all(got[miss] == 0.0)


@pytest.mark.parametrize("name,back", [("c1", 2), ("c3s", 2), ("c5s", 2), ("c1", 1), ("c3s", 1), ("c5s", 1), ("c1", 0),
                                       ("c3s", 0), ("tall3", 2), ("tall3", 1), ("tall4", 2), ("tall4", 1),
                                       ("tall4", 0), ("tall5", 2), ("tall5", 1), ("tall5", 0), ("odd", 2),
                                       ("odd", 1), ("odd", 0), ("level", 2), ("level", 1), ("level", 0)])
def test_backproject_matches_oracle(msf, name, back):
    """Every adjoint: voxel-driven gather from the cell table (2, default) or on the fly (1),
    and the ray-driven scatter (0)."""
    cfg, g, x0, v, y, lam = problem(name)
    print("case", name, back, flush=True)
    plan = msf.Plan(g)
    plan.set_tiles(back_mode=back)
    want = oracle.backproject(g, lam * y)
    got = plan.backproject(_dev(lam * y)).cpu().numpy()
    for f in range(g.n_frames):
        assert rel_l2(got[f], want[f]) <= 2e-6


@pytest.mark.parametrize("name,back", [("c1", 2), ("c2s", 2), ("c3s", 2), ("c1", 1), ("c2s", 1), ("c3s", 1), ("c2s", 0),
                                       ("odd", 2), ("odd", 1), ("level", 2), ("level", 1)])
def test_dot_product_adjoint(msf, name, back):
    """<A x, y> = <x, A^T y> for the FP32 kernels (products summed in FP64)."""
    cfg, g, *_ = problem(name)
    plan = msf.Plan(g)
    plan.set_tiles(back_mode=back)
    rng = np.random.default_rng(7)
    x = rng.uniform(size=plan.vol_shape).astype(np.float32)
    yy = rng.uniform(size=plan.n_meas).astype(np.float32)
    ax = plan.project(_dev(x)).cpu().numpy().astype(np.float64)
    aty = plan.backproject(_dev(yy)).cpu().numpy().astype(np.float64)
    lhs = float(ax @ yy.astype(np.float64))
    rhs = float(aty.reshape(-1) @ x.reshape(-1).astype(np.float64))
    assert abs(lhs - rhs) <= 1e-5 * abs(lhs)


@pytest.mark.parametrize("rpl,wpg,xcd", [(1, 1, 0), (1, 4, 1), (2, 2, 1), (3, 4, 1), (4, 4, 0), (5, 2, 0), (6, 1, 1)])
def test_tile_shapes_give_same_results(msf, rpl, wpg, xcd):
    """Launch shapes change only the mapping of work: the forward projection is
    bit-identical; both gather adjoints are bit-identical too (the same pieces, in
    the same fixed order per voxel, from the table or computed on the fly)."""
    cfg, g, x0, v, y, lam = problem("c2s")
    plan = msf.Plan(g)
    assert plan.get_tiles()["back_mode"] == 2
    base = plan.project(_dev(x0)).cpu().numpy()
    bbase = plan.backproject(_dev(lam * y)).cpu().numpy()
    for bm in (2, 1):
        plan.set_tiles(rays_per_lane=rpl, waves_per_group=wpg, back_mode=bm, xcd_remap=xcd)
        assert plan.get_tiles()["rays_per_lane"] == rpl
        got = plan.project(_dev(x0)).cpu().numpy()
        assert np.array_equal(got, base)
        assert np.array_equal(plan.backproject(_dev(lam * y)).cpu().numpy(), bbase), bm
    plan.set_tiles(rays_per_lane=rpl, waves_per_group=wpg, back_mode=0, xcd_remap=xcd)
    sc = plan.backproject(_dev(lam * y)).cpu().numpy()
    assert rel_l2(sc, bbase) <= 1e-6


@pytest.mark.parametrize("back", [2, 1])
def test_gather_is_deterministic(msf, back):
    cfg, g, x0, v, y, lam = problem("c3s")
    plan = msf.Plan(g)
    plan.set_tiles(back_mode=back)
    a = plan.backproject(_dev(lam * y)).cpu().numpy()
    b = plan.backproject(_dev(lam * y)).cpu().numpy()
    assert np.array_equal(a, b)


@pytest.mark.parametrize("back", [2, 1, 0])
def test_truncated_detector(msf, back):
    """A detector smaller than the volume's shadow (20 rows, 40 columns for a 32^3
    volume): its first and last rows and columns cut through the volume, so every
    adjoint reads the ends of the sinogram rows; A and A^T against the oracle."""
    import dataclasses
    cfg = dataclasses.replace(synth.config("c1"), det=(40, 20), cid=61)
    g = synth.make_geometry(cfg)
    x0 = synth.make_phantom(cfg).astype(np.float32).astype(np.float64)
    plan = msf.Plan(g)
    plan.set_tiles(back_mode=back)
    want = oracle.project(g, x0)
    got = plan.project(_dev(x0)).cpu().numpy()
    assert _frame_rel(g, got, want) <= 2e-6
    rng = np.random.default_rng(62)
    yy = rng.uniform(0.5, 1.5, size=plan.n_meas).astype(np.float32).astype(np.float64)
    # the end rows carry the largest values, so a lost end row shows
    rows = yy.reshape(-1, g.nv, g.nu)
    rows[:, 0, :] *= 4.0
    rows[:, -1, :] *= 4.0
    want_b = oracle.backproject(g, yy)
    got_b = plan.backproject(_dev(yy)).cpu().numpy()
    for f in range(g.n_frames):
        assert rel_l2(got_b[f], want_b[f]) <= 2e-6


@pytest.mark.parametrize("pitch,det,back", [(0.6, 64, 2), (0.6, 64, 1), (0.4, 96, 1)])
def test_fine_detector_rows(msf, pitch, det, back):
    """Detector pitch 0.6 and 0.4 voxel at the isocentre: a ray can meet one voxel
    in three or four detector rows inside one xy piece, so the gathers take their
    path for rows beyond the two candidates they always read (at pitch 0.4 more
    than three columns meet a cell, so only the on-the-fly gather applies); A and
    A^T against the oracle."""
    import dataclasses
    print("pitch", pitch, "back", back, flush=True)
    cfg = dataclasses.replace(synth.config("c1"), det=(det, det), pitch_at_iso=pitch, cid=63)
    g = synth.make_geometry(cfg)
    x0 = synth.make_phantom(cfg).astype(np.float32).astype(np.float64)
    plan = msf.Plan(g)
    plan.set_tiles(back_mode=back)
    want = oracle.project(g, x0)
    got = plan.project(_dev(x0)).cpu().numpy()
    assert _frame_rel(g, got, want) <= 2e-6
    rng = np.random.default_rng(64)
    yy = rng.uniform(0.5, 1.5, size=plan.n_meas).astype(np.float32).astype(np.float64)
    want_b = oracle.backproject(g, yy)
    got_b = plan.backproject(_dev(yy)).cpu().numpy()
    for f in range(g.n_frames):
        assert rel_l2(got_b[f], want_b[f]) <= 2e-6


@pytest.mark.parametrize("name,back", [("steep", 2), ("steep", 1), ("steep", 0), ("steeper", 1), ("steeper", 0),
                                       ("flat", 2), ("flat", 1), ("flat", 0)])
def test_degenerate_geometries(msf, name, back):
    """Steep rays (the forward projector and the scatter adjoint take their general z walk,
    which runs one ray per lane, and the gathers read rows past their two candidates) and a
    one-voxel slab: A and A^T of random volumes and sinograms against the oracle, exact zeros
    on rows that miss the volume, and the tile shape the plan keeps.  On `steeper` more than
    three detector columns meet a cell, so there is no cell table (back_mode 2)."""
    print("case", name, back, flush=True)
    cfg = synth.config(name)
    g = synth.make_geometry(cfg)
    nx, ny, nz = cfg.n
    steep = name.startswith("steep")
    plan = msf.Plan(g)
    if steep:
        assert plan.get_tiles()["rays_per_lane"] == 1   # 96 and 112 rows would ask for 2
    if name == "steeper":
        assert plan.get_tiles()["back_mode"] == 1
        with pytest.raises(msf.MsfError):
            plan.set_tiles(back_mode=2)
    plan.set_tiles(rays_per_lane=3, back_mode=back)
    tiles = plan.get_tiles()
    assert tiles["back_mode"] == back
    assert tiles["rays_per_lane"] == (1 if steep else 3)
    rng = np.random.default_rng(1000 * cfg.cid + 91)
    x = rng.uniform(0.5, 1.5, size=(g.n_frames, nz, ny, nx)).astype(np.float32).astype(np.float64)
    want = oracle.project(g, x)
    got = plan.project(_dev(x)).cpu().numpy()
    assert _frame_rel(g, got, want) <= 2e-6
    miss = want == 0.0   # x > 0 everywhere: exactly the rows with a zero chord through the box
    assert miss.any() and not miss.all()
    assert np.all(got[miss] == 0.0)
    yy = rng.uniform(0.5, 1.5, size=plan.n_meas).astype(np.float32).astype(np.float64)
    want_b = oracle.backproject(g, yy)
    got_b = plan.backproject(_dev(yy)).cpu().numpy()
    for f in range(g.n_frames):
        assert rel_l2(got_b[f], want_b[f]) <= 2e-6
    # the pair is adjoint to FP32 rounding: <A x, y> = <x, A^T y>
    lhs, rhs = float(np.dot(got.reshape(-1), yy)), float(np.dot(x.reshape(-1), got_b.reshape(-1)))
    assert abs(lhs - rhs) <= 1e-6 * abs(lhs)
