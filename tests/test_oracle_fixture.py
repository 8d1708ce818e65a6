"""Pins of the FP64 oracle of the blind fixture correction (paper Appendix A):
the mask, the blur (symmetric, normalised, separable), the least-squares fit
(orthogonality of the residual), and the correction's purpose: with the true
object as the reconstruction, the smooth projection of tubes outside the field
of view is removed from the sinogram."""
import numpy as np

import oracle
from oracle import fixture
from paper_2008_01567_amd import synth
import _analytic


def test_cylinder_mask():
    x = np.ones((1, 3, 6, 8))
    m = fixture.cylinder_mask(x, 2.0)
    cx = np.arange(8) - 3.5
    cy = np.arange(6) - 2.5
    want = (cx[None, :] ** 2 + cy[:, None] ** 2 <= 4.0).astype(float)
    assert np.array_equal(m[0, 1], want)
    assert m[0, 1].sum() == 12 and m[0, 1, 2, 3] == 1.0 and m[0, 1, 0, 0] == 0.0


def test_blur_is_symmetric_normalised_and_separable():
    rng = np.random.default_rng(0)
    u, w = rng.standard_normal((2, 17, 23))
    for std in (0.7, 1.5, 3.0):
        Bu, Bw = fixture.blur_view(u, std), fixture.blur_view(w, std)
        assert abs(np.sum(Bu * w) - np.sum(u * Bw)) < 1e-12 * np.abs(u).sum()
        taps = fixture.gaussian_taps(std)
        assert abs(taps.sum() - 1.0) < 1e-15 and np.allclose(taps, taps[::-1])
        r = len(taps) // 2
        imp = np.zeros((2 * r + 5, 2 * r + 5))
        imp[r + 2, r + 2] = 1.0
        assert np.allclose(fixture.blur_view(imp, std)[2:-2, 2:-2], np.outer(taps, taps), atol=1e-15)
        const = np.ones((4 * r + 3, 4 * r + 3))
        assert np.allclose(fixture.blur_view(const, std)[r:-r, r:-r], 1.0, atol=1e-14)


def _tube_problem():
    cfg = synth.config("c1")
    g = synth.make_geometry(cfg)
    x0 = synth.make_phantom(cfg)
    y_obj = oracle.project(g, x0)
    tubes = _analytic.fixture_tubes(cfg, radius=4.0, mu=0.02)
    f_sino = _analytic.shapes_sinogram(g, tubes)
    return cfg, g, x0, y_obj, f_sino


def test_fit_is_least_squares_and_removes_smooth_fixtures():
    cfg, g, x0, y_obj, f_sino = _tube_problem()
    assert np.count_nonzero(f_sino) > 0.02 * f_sino.size      # the tubes are seen
    y = y_obj + f_sino
    y_corr, c, e, p = fixture.correct(g, x0, y, radius=16.0, std=1.0)
    for f in range(g.n_frames):
        s = g.sino_slice(f)
        # residual orthogonal to p, and c beats its neighbours
        assert abs((e[s] - c[f] * p[s]) @ p[s]) <= 1e-10 * (e[s] @ e[s])
        err = lambda cc: np.sum((e[s] - cc * p[s]) ** 2)
        assert err(c[f]) <= min(err(c[f] * 1.01), err(c[f] * 0.99))
        # with the true object, e is the fixtures' projection: the correction removes most of it
        before = np.linalg.norm(y[s] - y_obj[s])
        after = np.linalg.norm(y_corr[s] - y_obj[s])
        # (measured on the oracle: 0.15-0.16 of the fixtures' projection remains, c = 1.08)
        assert after <= 0.25 * before, (f, before, after)
        assert 0.9 < c[f] < 1.25
