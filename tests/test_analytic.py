"""Pins of the analytic sinogram used as the full-size tests' measurement:
ellipsoid chords against the scalar closed form, cylinder chords against
point sampling along the ray, and both against the oracle projector of a
finely voxelised phantom (first-order convergence)."""
import dataclasses
import math

import numpy as np

import oracle
from paper_2008_01567_amd import synth
import _analytic


def _sampled_chord(S, D, shape, centre, n=20000):
    """Length inside the shape by midpoint sampling of the segment (brute force)."""
    t = (np.arange(n) + 0.5) / n
    P = S[None, :] + t[:, None] * (D - S)[None, :]
    q = (P - centre) @ shape.rot
    if shape.kind == "ellipsoid":
        inside = ((q / shape.axes) ** 2).sum(axis=1) <= 1.0
    else:
        inside = (q[:, 0] ** 2 + q[:, 1] ** 2 <= shape.axes[0] ** 2) & (np.abs(q[:, 2]) <= shape.axes[2])
    return inside.mean() * np.linalg.norm(D - S)


def test_chords_match_point_sampling():
    cfg = dataclasses.replace(synth.config("c5s"), cid=81)
    g = synth.make_geometry(cfg)
    shapes = synth.make_shapes(cfg)
    assert {s.kind for s in shapes} == {"ellipsoid", "cylinder"}
    rng = np.random.default_rng(3)
    S, D = _analytic.view_rays(g, g.angles[1])
    rows = rng.integers(0, len(D), 60)
    for s in shapes:
        c = synth.frame_centre(s, cfg, 1)
        got = _analytic._chords(S, D[rows], s, c)
        want = np.array([_sampled_chord(S, D[r], s, c) for r in rows])
        # sampling error <= 2 steps of the segment
        assert np.all(np.abs(got - want) <= 2.5 * np.linalg.norm(D[0] - S) / 20000), (s.kind, got - want)
    # the ray helper reproduces the oracle's rays
    for r in rows[:10]:
        iv, iu = divmod(int(r), g.nu)
        So, Do = oracle.ray(g, g.angles[1], iu, iv)
        assert np.allclose(So, S) and np.allclose(Do, D[r], rtol=0, atol=1e-12)


def test_bounding_boxes_lose_nothing():
    """Restricting each shape to its projected bounding box gives the same sinogram as
    evaluating every ray."""
    cfg = dataclasses.replace(synth.config("c5s"), cid=83)
    g = synth.make_geometry(cfg)
    shapes = synth.make_shapes(cfg)
    got = _analytic.sinogram(cfg, g, frames=[0, 3])
    full = []
    for f in (0, 3):
        for view in range(int(g.view_offset[f]), int(g.view_offset[f + 1])):
            S, D = _analytic.view_rays(g, g.angles[view])
            full.append(sum(s.mu * _analytic._chords(S, D, s, synth.frame_centre(s, cfg, f)) for s in shapes))
    full = np.concatenate(full)
    assert np.count_nonzero(full) > 0.05 * full.size
    assert np.array_equal(got, full)


def test_sinogram_approaches_oracle_projection_of_voxelised_phantom():
    errs = []
    for n in (16, 32):
        cfg = dataclasses.replace(synth.config("c5s"), cid=82, n=(n, n, n), det=(int(1.5 * n), int(1.5 * n)),
                                  src_iso=6.25 * n, src_det=12.5 * n, n_frames=1, views=2, supersample=4)
        g = synth.make_geometry(cfg)
        x = synth.make_phantom(cfg)
        y = oracle.FrameMatrix(g, 0).A(x[0])
        ya = _analytic.sinogram(cfg, g)
        errs.append(np.linalg.norm(y - ya) / np.linalg.norm(ya))
    # first order, frozen from the oracle: 0.117, 0.077, 0.045 at 16^3, 32^3, 64^3
    assert errs[1] < 0.75 * errs[0] and errs[1] < 0.1, errs
