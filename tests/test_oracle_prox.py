"""Pins of the FP64 proximal-map oracle (paper eq. (4) with the data term of eq. (2)).

The CG oracle is checked against the dense normal-equation solve, closed-form
special cases, linearity, the first-order small-sigma expansion and the
optimality condition of the objective.
"""
import math

import numpy as np
import pytest

import oracle
from paper_2008_01567_amd import synth


def _problem(name, frames=None):
    cfg = synth.config(name)
    g = synth.make_geometry(cfg)
    fr = list(range(g.n_frames)) if frames is None else list(frames)
    x0 = synth.make_phantom(cfg, fr)
    v = synth.make_v(cfg, x0, fr)
    y, lam = oracle.make_measurement(cfg, g, x0, fr)
    return cfg, g, x0, v, y, lam


def test_cg_matches_dense_cholesky_tiny8():
    cfg, g, x0, v, y, lam = _problem("tiny8")
    xd = oracle.prox_dense(g, v, y, lam, cfg.sigma)
    xc, st = oracle.prox_cg(g, v, y, lam, cfg.sigma, tol=1e-13)
    for f in range(g.n_frames):
        assert np.linalg.norm(xc[f] - xd[f]) <= 1e-10 * np.linalg.norm(xd[f])
        assert st[f]["true_rel_res"] < 1e-11


@pytest.mark.slow
def test_cg_matches_dense_cholesky_tiny16():
    cfg, g, x0, v, y, lam = _problem("tiny16", frames=[1])
    gs = g.subset([1])
    xd = oracle.prox_dense(gs, v, y, lam, cfg.sigma, method="siddon")
    xc, _ = oracle.prox_cg(gs, v, y, lam, cfg.sigma, tol=1e-13)
    assert np.linalg.norm(xc[0] - xd[0]) <= 1e-10 * np.linalg.norm(xd[0])


def test_zero_weights_give_identity():
    """Lambda = 0: the data term vanishes, L(v) = v and the initial residual is 0."""
    cfg, g, x0, v, y, lam = _problem("tiny8")
    x, st = oracle.prox_cg(g, v, y, np.zeros_like(lam), cfg.sigma)
    assert np.array_equal(x, v)
    assert all(s["iters"] == 0 for s in st)


def test_consistent_data_gives_identity():
    """y = A v: v already minimises both terms, so L(v) = v for any Lambda, sigma."""
    cfg, g, x0, v, y, lam = _problem("tiny8")
    yv = oracle.project(g, v)
    for sigma in (0.1, 0.5, 3.0):
        x, _ = oracle.prox_cg(g, v, yv, lam, sigma, tol=1e-14)
        assert np.abs(x - v).max() <= 1e-10 * np.abs(v).max()


def test_one_voxel_one_ray_closed_form():
    """A 1x1x1 volume and one central ray at 30 degrees: a = 1/cos(30) = 2/sqrt(3),
    x = (a Lambda y + v/sigma^2) / (a^2 Lambda + 1/sigma^2)."""
    th = math.pi / 6
    g = synth.Geometry(1, 1, 1, 1, 1, 1, 2.0, 2.0, 10.0, 20.0, np.array([0, 1], dtype=np.int64),
                       np.array([th]))
    M = oracle.FrameMatrix(g, 0)
    a = 2.0 / math.sqrt(3.0)
    assert M.nnz == 1 and abs(M.val[0] - a) < 1e-14
    for (lam, yv, v, sigma) in [(2.0, 0.7, 0.1, 0.5), (0.3, -1.0, 2.0, 1.7)]:
        x, _ = M.prox_cg(np.array([v]), np.array([yv]), np.array([lam]), sigma, tol=1e-15)
        want = (a * lam * yv + v / sigma ** 2) / (a * a * lam + 1.0 / sigma ** 2)
        assert abs(x[0] - want) <= 1e-14 * max(1.0, abs(want))


def test_joint_linearity_and_frame_permutation():
    cfg, g, x0, v, y, lam = _problem("tiny8")
    rng = np.random.default_rng(0)
    v2 = rng.standard_normal(v.shape) * 0.01
    y2 = rng.standard_normal(y.shape) * 0.1
    a, b = 0.7, -1.3
    xa, _ = oracle.prox_cg(g, v, y, lam, 0.5, tol=1e-14)
    xb, _ = oracle.prox_cg(g, v2, y2, lam, 0.5, tol=1e-14)
    xab, _ = oracle.prox_cg(g, a * v + b * v2, a * y + b * y2, lam, 0.5, tol=1e-14)
    assert np.abs(xab - (a * xa + b * xb)).max() <= 1e-10 * np.abs(xab).max()
    # permuting frames (and their sinograms/geometry) permutes the outputs
    gp = g.subset([1, 0])
    r = g.n_rays_per_view
    s0, s1 = g.sino_slice(0), g.sino_slice(1)
    yp = np.concatenate([y[s1], y[s0]])
    lp = np.concatenate([lam[s1], lam[s0]])
    xp, _ = oracle.prox_cg(gp, v[::-1].copy(), yp, lp, 0.5, tol=1e-14)
    assert np.abs(xp[::-1] - xa).max() <= 1e-12 * np.abs(xa).max()


def test_small_sigma_first_order():
    """L(v) = v + sigma^2 A^T Lambda (y - A v) + O(sigma^4)."""
    cfg, g, x0, v, y, lam = _problem("tiny8")
    # spectral radius of A^T Lambda A by power iteration; sigma^2 * rho must be small
    z = np.ones_like(v)
    for _ in range(60):
        z = oracle.backproject(g, lam * oracle.project(g, z))
        rho = np.linalg.norm(z)
        z /= rho
    errs = []
    for sigma in (math.sqrt(0.02 / rho), math.sqrt(0.005 / rho)):
        x, _ = oracle.prox_cg(g, v, y, lam, sigma, tol=1e-15)
        lin = v + sigma ** 2 * oracle.backproject(g, lam * (y - oracle.project(g, v)))
        errs.append(np.abs(x - lin).max() / np.abs(x - v).max())
    assert errs[1] < errs[0] / 3.0 and errs[1] < 0.05


def test_optimality_condition():
    """The gradient A^T Lambda (A x - y) + (x - v)/sigma^2 vanishes at the oracle's answer."""
    cfg, g, x0, v, y, lam = _problem("c1", frames=[2])
    gs = g.subset([2])
    x, st = oracle.prox_cg(gs, v, y, lam, cfg.sigma, tol=1e-12)
    grad = oracle.backproject(gs, lam * (oracle.project(gs, x) - y)) + (x - v) / cfg.sigma ** 2
    b = oracle.backproject(gs, lam * y) + v / cfg.sigma ** 2
    assert np.linalg.norm(grad) <= 1e-11 * np.linalg.norm(b)
    assert st[0]["true_rel_res"] <= 1e-11


def test_warm_start_same_answer_fewer_iterations():
    cfg, g, x0, v, y, lam = _problem("c1", frames=[0])
    gs = g.subset([0])
    xa, sa = oracle.prox_cg(gs, v, y, lam, cfg.sigma, tol=1e-10)
    near = xa + 1e-6 * np.random.default_rng(1).standard_normal(xa.shape)
    xb, sb = oracle.prox_cg(gs, v, y, lam, cfg.sigma, tol=1e-10, x0=near)
    assert np.linalg.norm(xb - xa) <= 1e-8 * np.linalg.norm(xa)
    assert sb[0]["iters"] < sa[0]["iters"]
