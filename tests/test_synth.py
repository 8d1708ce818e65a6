"""Seeded input generator: determinism, shapes and the schedules' structure."""
import math

import numpy as np

from paper_2008_01567_amd import synth


def test_deterministic_and_seed_dependent():
    cfg = synth.config("c1")
    a = synth.make_phantom(cfg)
    b = synth.make_phantom(cfg)
    assert np.array_equal(a, b)
    assert np.array_equal(synth.make_v(cfg, a), synth.make_v(cfg, b))
    g = synth.make_geometry(cfg)
    assert np.array_equal(synth.noise_eps(cfg, g), synth.noise_eps(cfg, g))
    other = synth.make_phantom(synth.config("c2s"))
    assert other.shape != a.shape or not np.array_equal(other, a)
    # per-frame streams: a frame subset equals the slice of the whole batch
    assert np.array_equal(synth.make_v(cfg, a[2:3], [2]), synth.make_v(cfg, a)[2:3])
    assert np.array_equal(synth.noise_eps(cfg, g, [3]), synth.noise_eps(cfg, g)[g.sino_slice(3)])


def test_phantom_class_and_motion():
    cfg = synth.config("c1")
    x = synth.make_phantom(cfg)
    assert x.shape == (4, 32, 32, 32) and x.min() >= 0.0
    assert 0.01 <= x.max() <= 0.05 * (cfg.n_objects)
    # +1 voxel per frame along +z
    assert np.allclose(x[1, 1:], x[0, :-1]) and np.allclose(x[3, 1:], x[2, :-1])


def test_angle_schedules():
    g = synth.make_geometry(synth.config("c1"))
    assert g.n_views == 32 and np.allclose(np.diff(g.view_offset), 8)
    deg = np.rad2deg(g.angles)
    assert abs(deg[1] - synth.GOLDEN_DEG) < 1e-9 and (deg < 180).all()
    g2 = synth.make_geometry(synth.config("c2"))
    d2 = np.rad2deg(g2.angles).reshape(16, 16)
    assert np.allclose(d2[0], np.arange(16) * 22.5) and np.allclose(d2[1] - d2[0], 22.5 / 16)
    g3 = synth.make_geometry(synth.config("c3"))
    counts = np.diff(g3.view_offset)
    assert counts.min() >= 6 and counts.max() <= 40 and len(set(counts.tolist())) > 5
    assert abs(g2.du - 2.0) < 1e-15


def test_measurement_recipe():
    rng = np.random.default_rng(0)
    yc = np.abs(rng.standard_normal(2 * 3 * 4)) * 2
    eps = rng.standard_normal(yc.shape)
    y, lam = synth.finish_measurement(yc, eps, [1, 1], 12)
    s0 = 0.01 * yc[:12].max()
    assert np.allclose(y[:12], yc[:12] + s0 * eps[:12])
    assert np.allclose(lam[:12], 1 / np.maximum(y[:12], s0))
    assert (lam > 0).all() and np.isfinite(lam).all()
    # the paper's model: inverse variance c exp(-y_clean) with c = 1 / s^2
    yp, lp = synth.finish_measurement(yc, eps, [1, 1], 12, model="paper")
    assert np.allclose(lp[:12], np.exp(-yc[:12]) / s0 ** 2)
    assert np.allclose(yp[:12], yc[:12] + eps[:12] / np.sqrt(lp[:12]))
    # noise of a zero-attenuation ray is s; it grows with attenuation
    assert np.isclose(1 / np.sqrt(np.exp(-0.0) / s0 ** 2), s0)


def test_workload_seed_bases_are_distinct():
    """Every named workload draws from its own seed base (seed = 1000 * cid + stream), so no two
    workloads share a phantom, noise or view stream by accident."""
    from collections import Counter
    counts = Counter(cfg.cid for cfg in synth.CONFIGS.values())
    assert [cid for cid, n in counts.items() if n > 1] == []
