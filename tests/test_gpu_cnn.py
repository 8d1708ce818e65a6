"""GPU parity of the warm-start network's BF16 matrix-core kernels against the
FP64 oracle (same BF16 rounding points), and of the learned start inside the
solver."""
import numpy as np
import pytest

import oracle
from oracle import cnn as ocnn
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


def _params(seed, scale=1.0):
    rng = np.random.default_rng(seed)
    ps = []
    for li in range(4):
        ci, co = ocnn.CHANNELS[li], ocnn.CHANNELS[li + 1]
        ps.append((rng.standard_normal((co, ci, 3, 3, 3)) * np.sqrt(2.0 / (27 * ci)) * scale,
                   rng.standard_normal(co) * 0.1))
    # FP32 master weights on both sides
    return [(w.astype(np.float32).astype(np.float64), b.astype(np.float32).astype(np.float64)) for w, b in ps]


SHAPE = (2, 9, 10, 21)      # ragged x (21 = 16 + 5) and small y, z: zero padding on every face
# The 3D kernel's workgroup tile is 4 rows x 64 x voxels and walks 16-slice z
# chunks: 150 = 64 + 64 + 22 x voxels (three x tiles, two interior halos),
# 40 = 16 + 16 + 8 slices (three chunks, the later ones seeded from the one
# before), 9 = 4 + 4 + 1 rows (a partial row tile).
TILED = (1, 40, 9, 150)
SHAPES = [SHAPE, TILED]


def _inputs(seed, shape=SHAPE):
    rng = np.random.default_rng(seed)
    v = (0.03 + 0.01 * rng.standard_normal(shape)).astype(np.float32)
    g = (0.01 * rng.standard_normal(shape)).astype(np.float32)
    t = (v + 0.005 * rng.standard_normal(shape)).astype(np.float32)
    return v, g, t


@pytest.mark.parametrize("shape", SHAPES, ids=["small", "tiled"])
def test_forward_matches_oracle(msf, shape):
    params = _params(0)
    v, g, _ = _inputs(1, shape)
    c = (0.05, 0.01, 0.02)
    net = msf.Cnn(ocnn.flatten(params), c)
    got = net.infer(_dev(v), _dev(g)).cpu().numpy()
    inp = np.stack([v, g], axis=1).astype(np.float64)
    want, _ = ocnn.forward(params, inp, bf16=True, scale=c)
    want = want[:, 0]
    err = rel_l2(got - v, want - v)
    print(shape, "forward residual rel err %.2e" % err, flush=True)
    assert err <= 1e-3        # observed 2.2e-6 (small), 9.8e-5 (tiled)
    assert np.abs(got - want).max() <= 1e-3 * np.abs(want - v).max() * 10


@pytest.mark.parametrize("shape", SHAPES, ids=["small", "tiled"])
def test_gradients_match_oracle(msf, shape):
    params = _params(2)
    v, g, t = _inputs(3, shape)
    c = (0.05, 0.01, 0.02)
    net = msf.Cnn(ocnn.flatten(params), c)
    loss, grad = net.train_step(_dev(v), _dev(g), _dev(t), lr=0.0, apply=False, want_grad=True)
    inp = np.stack([v, g], axis=1).astype(np.float64)
    out, cache = ocnn.forward(params, inp, bf16=True, scale=c)
    oloss, dx0 = ocnn.mse(out, t[:, None].astype(np.float64))
    ograd = ocnn.flatten(ocnn.backward(params, cache, dx0))
    assert abs(loss - oloss) <= 1e-3 * oloss
    o = 0
    for li in range(4):
        ci, co = ocnn.CHANNELS[li], ocnn.CHANNELS[li + 1]
        n = co * ci * 27 + co
        err = rel_l2(grad[o:o + n], ograd[o:o + n])
        print(shape, "layer", li, "grad rel err %.2e" % err, flush=True)
        assert err <= 1e-3    # observed 1.8e-6 ... 1.3e-4 over both shapes and all layers
        o += n
    assert np.array_equal(net.params(), ocnn.flatten(params).astype(np.float32))   # apply=0 leaves weights


@pytest.mark.parametrize("shape", SHAPES, ids=["small", "tiled"])
def test_adam_step_and_training_reduces_loss(msf, shape):
    params = _params(4, scale=0.5)
    v, g, t = _inputs(5, shape)
    c = 0.05
    net = msf.Cnn(ocnn.flatten(params), c)
    p0 = net.params().astype(np.float64)
    loss0, grad = net.train_step(_dev(v), _dev(g), _dev(t), lr=1e-3, apply=True, want_grad=True)
    p1 = net.params().astype(np.float64)
    want = ocnn.flatten(ocnn.adam(ocnn.unflatten(p0), ocnn.unflatten(grad.astype(np.float64)), {}, lr=1e-3))
    assert np.allclose(p1, want, rtol=1e-5, atol=1e-7)
    losses = [loss0]
    for _ in range(40):
        losses.append(net.train_step(_dev(v), _dev(g), _dev(t), lr=3e-3)[0])
    assert losses[-1] < 0.7 * losses[0], losses[::10]


def _jacobi_net(alpha, c):
    """Hand-built weights: x0 = v + alpha * g exactly (ReLU pair of +g and -g)."""
    ps = []
    w = np.zeros((16, 2, 3, 3, 3)); w[0, 1, 1, 1, 1] = 1.0; w[1, 1, 1, 1, 1] = -1.0
    ps.append((w, np.zeros(16)))
    for _ in range(2):
        w = np.zeros((16, 16, 3, 3, 3)); w[0, 0, 1, 1, 1] = 1.0; w[1, 1, 1, 1, 1] = 1.0
        ps.append((w, np.zeros(16)))
    w = np.zeros((1, 16, 3, 3, 3)); w[0, 0, 1, 1, 1] = alpha; w[0, 1, 1, 1, 1] = -alpha
    ps.append((w, np.zeros(1)))
    return ocnn.flatten(ps)


def test_learned_start_kept_or_rejected(msf):
    cfg, geom, x0, v, y, lam = problem("c1")
    plan = msf.Plan(geom)
    xs, _ = oracle_solution("c1")
    plain, sp = plan.prox_solve(_dev(v), _dev(y), _dev(lam), cfg.sigma, tol=1e-8, max_iter=4000)
    # a network whose output layer is zero predicts x0 = v: no better than v, so rejected
    zero = msf.Cnn(np.zeros(msf.N_CNN_PARAMS, dtype=np.float32), 0.05)
    x, st = plan.prox_solve(_dev(v), _dev(y), _dev(lam), cfg.sigma, tol=1e-8, max_iter=4000, cnn=zero)
    assert st["status"] == msf.MSF_CNN_FALLBACK and not st["cnn_used"].any()
    assert (st["iters"] == sp["iters"]).all()
    # x0 = v + alpha g (a damped Jacobi step) with an alpha that lowers every frame's
    # residual (chosen with the oracle): kept, and the answer is unchanged
    H = lambda z: oracle.backproject(geom, lam * oracle.project(geom, z)) + z / cfg.sigma ** 2
    r0 = oracle.backproject(geom, lam * (y - oracle.project(geom, v)))
    d = oracle.backproject(geom, lam * oracle.project(geom, np.ones_like(v)))
    gref = np.stack([r0[f] / (d[f].mean() + 1 / cfg.sigma ** 2) for f in range(geom.n_frames)])
    alpha = next(a for a in (0.5, 0.25, 0.1, 0.05, 0.02)
                 if all(np.linalg.norm(r0[f] - a * H(gref)[f]) < 0.99 * np.linalg.norm(r0[f])
                        for f in range(geom.n_frames)))
    jac = msf.Cnn(_jacobi_net(alpha, 0.05), 0.05)
    x, st = plan.prox_solve(_dev(v), _dev(y), _dev(lam), cfg.sigma, tol=1e-8, max_iter=4000, cnn=jac)
    print("jacobi start: iters", st["iters"].tolist(), "plain", sp["iters"].tolist(), flush=True)
    assert st["status"] == msf.MSF_OK and st["cnn_used"].all()
    x = x.cpu().numpy()
    for f in range(geom.n_frames):
        assert rel_l2(x[f], xs[f]) <= 1e-4
    # the network really saw g: its prediction equals v + 0.5 g
    gfeat = plan.features(_dev(v), _dev(y), _dev(lam), cfg.sigma)
    pred = jac.infer(_dev(v), gfeat).cpu().numpy()
    assert rel_l2(pred - v, alpha * gfeat.cpu().numpy()) <= 1e-2


def test_learned_start_worse_than_v_falls_back_to_plain_cg(msf):
    """x0 = v - 5 g: finite, and its residual r_v + 5 H g is larger than r_v on
    every frame (<r_v, H g> > 0 since H is positive definite and g is r_v
    scaled), so every frame must start from v and run exactly the plain solve."""
    cfg, geom, x0, v, y, lam = problem("c1")
    plan = msf.Plan(geom)
    xs, _ = oracle_solution("c1")
    plain, sp = plan.prox_solve(_dev(v), _dev(y), _dev(lam), cfg.sigma, tol=1e-8, max_iter=4000)
    worse = msf.Cnn(_jacobi_net(-5.0, 0.05), 0.05)
    x, st = plan.prox_solve(_dev(v), _dev(y), _dev(lam), cfg.sigma, tol=1e-8, max_iter=4000, cnn=worse)
    print("worse start: iters", st["iters"].tolist(), "plain", sp["iters"].tolist(), flush=True)
    assert st["status"] == msf.MSF_CNN_FALLBACK and not st["cnn_used"].any()
    assert (st["iters"] == sp["iters"]).all()
    assert torch.equal(x, plain)
    x = x.cpu().numpy()
    for f in range(geom.n_frames):
        assert rel_l2(x[f], xs[f]) <= 1e-4


def test_features_match_oracle(msf):
    """g = (b - H v) / d with d = mean(A^T Lambda A 1) + 1/sigma^2 per frame."""
    cfg, geom, x0, v, y, lam = problem("c1")
    plan = msf.Plan(geom)
    g = plan.features(_dev(v), _dev(y), _dev(lam), cfg.sigma).cpu().numpy()
    r = oracle.backproject(geom, lam * (y - oracle.project(geom, v)))
    d = oracle.backproject(geom, lam * oracle.project(geom, np.ones_like(v)))
    for f in range(geom.n_frames):
        want = r[f] / (d[f].mean() + 1.0 / cfg.sigma ** 2)
        assert rel_l2(g[f], want) <= 1e-4
