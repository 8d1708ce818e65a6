"""The trained warm-start network (128^3 x 16 frames, 8 golden-angle views per
frame over 180 degrees) on a held-out seed: what it gains over starting from v,
and that the learned start still leads to the oracle's answer."""
import dataclasses
import json

import numpy as np
import pytest

import oracle
from paper_2008_01567_amd import synth
from paper_2008_01567_amd.calibration import FROZEN_TOL
from _problems import rel_l2

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def msf():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2008_01567_amd import msf as m
    m.lib()
    return m


def test_trained_network_gain_on_held_out_seed(msf):
    from paper_2008_01567_amd import train_cnn
    params, scales, meta = train_cnn.load("c4")
    assert meta["frames"] == 2000 and meta["config"] == "c4"
    cfg = dataclasses.replace(synth.config("c4"), cid=50010)       # held out: not a training seed
    g = synth.make_geometry(cfg)
    x0 = synth.make_phantom(cfg).astype(np.float32).astype(np.float64)
    v = synth.make_v(cfg, x0).astype(np.float32).astype(np.float64)
    y, lam = oracle.make_measurement(cfg, g, x0)
    y, lam = y.astype(np.float32).astype(np.float64), lam.astype(np.float32).astype(np.float64)
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()
    plan = msf.Plan(g)
    net = msf.Cnn(params, scales)
    tol = FROZEN_TOL["c4"]
    xp, sp = plan.prox_solve(dev(v), dev(y), dev(lam), cfg.sigma, tol=tol, max_iter=6000, check_every=16)
    xl, sl = plan.prox_solve(dev(v), dev(y), dev(lam), cfg.sigma, tol=tol, max_iter=6000, check_every=16, cnn=net)
    r0p, r0l = sp["start_rel_residual"].mean(), sl["start_rel_residual"].mean()
    print("start residual: v %.3e, network %.3e; CG iterations: v %.1f, network %.1f; seconds %.3f vs %.3f"
          % (r0p, r0l, sp["iters"].mean(), sl["iters"].mean(), sp["seconds"], sl["seconds"]), flush=True)
    # the network's start is kept on every frame and halves the residual of the start ...
    assert sl["cnn_used"].all() and sl["status"] == msf.MSF_OK
    assert r0l <= 0.7 * r0p
    # ... but the iterations to the stopping rule stay within a few percent (no speedup on this workload)
    assert sl["iters"].mean() <= 1.05 * sp["iters"].mean()
    # both starts reach the oracle's proximal map (frame 0, FP64 CG to 1e-11)
    M = oracle.FrameMatrix(g, 0)
    s = g.sino_slice(0)
    xs, _ = M.prox_cg(v[0], y[s], lam[s], cfg.sigma, tol=1e-11, max_iter=20000)
    xs = xs.reshape(v[0].shape)
    assert rel_l2(xl.cpu().numpy()[0], xs) <= 1e-4
    assert rel_l2(xp.cpu().numpy()[0], xs) <= 1e-4


def test_training_pipeline_end_to_end(msf, tmp_path):
    """The training driver on a small workload: triples from the plain solver,
    library forward/backward/Adam on crops, held-out evaluation, saved network."""
    from paper_2008_01567_amd import train_cnn
    out = str(tmp_path / "ws_c1.npz")
    train_cnn.main(["--config", "c1", "--problems", "3", "--eval", "1", "--steps", "60", "--batch", "2",
                    "--crop", "16", "--lr", "3e-3", "--out", out])
    z = np.load(out, allow_pickle=False)
    meta = json.loads(str(z["meta"]))
    assert z["params"].shape == (train_cnn.N_PARAMS,) and np.isfinite(z["params"]).all()
    assert meta["frames"] == 12 and meta["steps"] == 60
    # the trained start beats v on the training distribution's held-out problem
    ev = meta["eval"][0]
    assert ev["start_residual_learned"] < ev["start_residual_plain"]
    assert meta["final_loss"] < meta["loss_of_v"]
