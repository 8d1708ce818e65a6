"""Pins of the FP64 MACE oracle (paper Sec. III): the averaging identities and
the consensus equilibrium of proximal agents, which solves the multi-regularised
MAP problem of eq. (map_multireg)."""
import numpy as np

import oracle
from oracle import mace
from paper_2008_01567_amd import synth


def test_G_is_idempotent_and_reflection_is_involution():
    rng = np.random.default_rng(0)
    W = [rng.standard_normal(50) for _ in range(4)]
    for beta in (0.3, 1.0, 2.5):
        GW = mace.G(W, beta)
        GGW = mace.G(GW, beta)
        assert all(np.allclose(a, b, rtol=0, atol=1e-14) for a, b in zip(GW, GGW))
        R = [2 * g - w for g, w in zip(GW, W)]
        RR = [2 * g - r for g, r in zip(mace.G(R, beta), R)]
        assert all(np.allclose(a, b, rtol=0, atol=1e-13) for a, b in zip(RR, W))
    # beta = 1 weighs the forward model and the mean of the priors equally
    m = mace.weighted_mean(W, 1.0)
    assert np.allclose(m, 0.5 * W[0] + 0.5 * (W[1] + W[2] + W[3]) / 3)


def test_ridge_agents_reach_map_solution():
    """Proximal agents H_k(x) = x / (1 + lam sigma^2) (prox of lam/2 ||x||^2): Algorithm 1
    converges to the solution of (A^T Lambda A + beta lam I) x = A^T Lambda y."""
    cfg = synth.config("tiny8")
    g = synth.make_geometry(cfg).subset([0])
    x0 = synth.make_phantom(cfg, [0])
    y, lw = oracle.make_measurement(cfg, g, x0, [0])
    M = oracle.FrameMatrix(g, 0)
    sigma, lam_r, beta, rho, K = 0.5, 3.0, 1.0, 0.5, 3

    def agents(W, X):
        xL, _ = M.prox_cg(W[0], y, lw, sigma, tol=1e-14)
        return [xL] + [w / (1.0 + lam_r * sigma ** 2) for w in W[1:]]
    agents.n_agents = K + 1

    xs, X, W = mace.mann_partial(agents, np.zeros(M.ncols), beta, rho, 300)
    A = M.dense()
    want = np.linalg.solve(A.T @ (lw[:, None] * A) + beta * lam_r * np.eye(M.ncols), A.T @ (lw * y))
    xbar = mace.weighted_mean(W, beta)
    assert np.linalg.norm(xbar - want) <= 1e-6 * np.linalg.norm(want)
    # at equilibrium every agent's output equals the consensus value
    assert np.linalg.norm(xs - want) <= 1e-6 * np.linalg.norm(want)


def test_plane_smoothers_are_proximal_maps():
    """Symmetric (<Hx, z> = <x, Hz>) with eigenvalues in (0, 1]: the proximal map of a
    convex quadratic (a linear map is a proximal map iff it is symmetric with spectrum in [0, 1])."""
    rng = np.random.default_rng(1)
    shape = (1, 5, 6, 7)
    n = int(np.prod(shape))
    for k in (1, 2, 3):
        H = np.zeros((n, n))
        for j in range(n):
            e = np.zeros(n)
            e[j] = 1.0
            H[:, j] = mace.plane_smoother(e.reshape(shape), k, 1.0).reshape(-1)
        assert np.allclose(H, H.T, atol=1e-15)
        ev = np.linalg.eigvalsh(H)
        assert ev.min() > 0.0 and ev.max() <= 1.0 + 1e-12
    # a constant field away from the boundary is preserved (taps sum to one)
    x = np.ones((1, 9, 9, 9))
    assert abs(mace.plane_smoother(x, 1, 1.0)[0, 4, 4, 4] - 1.0) < 1e-14


def test_slices_round_trip_and_neighbour_mean():
    rng = np.random.default_rng(3)
    W = rng.standard_normal((5, 3, 4, 6))
    for k in (1, 2, 3):
        S = mace.to_slices(W, k)
        assert np.array_equal(mace.from_slices(S, k, W.shape), W)
    # plane 2 images are (z, y) at fixed (t, x); plane 3 images are (z, x) at fixed (t, y)
    S2 = mace.to_slices(W, 2).reshape(5, 6, 3, 4)
    assert S2[1, 5, 2, 3] == W[1, 2, 3, 5]
    S3 = mace.to_slices(W, 3).reshape(5, 4, 3, 6)
    assert S3[4, 1, 0, 2] == W[4, 0, 1, 2]
    m = mace.time_neighbour_mean(W)
    assert np.allclose(m[2], (W[0] + W[1] + W[3] + W[4]) / 4)
    assert np.allclose(m[0], (W[0] + W[0] + W[1] + W[2]) / 4)       # clamped at the ends


def test_cnn_agent_with_identity_network():
    """A network whose output is zero (last layer zero) is the identity agent; a
    network that outputs its second input channel averages over time."""
    from oracle import cnn
    rng = np.random.default_rng(4)
    W = rng.uniform(0, 1, (4, 3, 5, 6))
    params = cnn.init_params(1)
    params[3] = (np.zeros_like(params[3][0]), np.zeros_like(params[3][1]))
    for k in (1, 2, 3):
        assert np.allclose(mace.cnn_agent(W, k, params, (1.0, 1.0, 1.0)), cnn.bf16_round(W) * 0 + W, atol=0)


def test_cnn_agent_centre_tap_network_closed_form():
    """A network that only passes its two channels through the centre tap and
    outputs alpha (channel 1 - channel 0) gives H(W) = W + alpha (mean_t W - W):
    the time-neighbour channel and the residual output are wired as stated."""
    from oracle import cnn
    rng = np.random.default_rng(5)
    W = rng.uniform(0.1, 1.0, (5, 3, 4, 6))
    alpha = 0.25
    params = []
    for li, (ci, co) in enumerate(zip(cnn.CHANNELS[:-1], cnn.CHANNELS[1:])):
        w = np.zeros((co, ci, 3, 3, 3))
        if li < 3:
            w[0, 0, 1, 1, 1] = 1.0
            w[1, 1, 1, 1, 1] = 1.0
        else:
            w[0, 0, 1, 1, 1] = -alpha
            w[0, 1, 1, 1, 1] = alpha
        params.append((w, np.zeros(co)))
    want = W + alpha * (mace.time_neighbour_mean(W) - W)
    for k in (1, 2, 3):
        got = mace.cnn_agent(W, k, params, (1.0, 1.0, 1.0))
        assert np.allclose(got, want, rtol=0, atol=1e-2 * alpha), k     # inputs rounded to bf16
