"""FP64 oracle of the MACE outer loop (TEST INFRASTRUCTURE ONLY).

Paper Sec. III: agents F = [L(W_0); H_1(W_1); ...; H_K(W_K)] (eq. (mace_F)),
the averaging operator G (eqs. (mace_G), (mace_avg)) with weight beta, and
Algorithm 1 (partial-update Mann iteration):  starting from X = W = copies of
x^(0), repeat  X <- F~(W; X),  Z <- G(2X - W),  W <- W + 2 rho (Z - X);
the reconstruction is X_0.
"""
from __future__ import annotations

import numpy as np


def weighted_mean(W, beta: float):
    """eq. (mace_avg): W_0/(1+beta) + beta/(1+beta) * mean_k W_k."""
    K = len(W) - 1
    return W[0] / (1.0 + beta) + (beta / (1.0 + beta)) * (sum(W[1:]) / K)


def G(W, beta: float):
    """eq. (mace_G): every component replaced by the weighted mean."""
    m = weighted_mean(W, beta)
    return [m.copy() for _ in W]


def mann_partial(agents, x_init, beta: float, rho: float, n_iter: int):
    """Algorithm 1.  ``agents(W, X)`` returns the list F~(W; X) (``agents.n_agents``
    components); the first entry may use X_0 as the warm start of the
    data-term solve."""
    K1 = agents.n_agents
    X = [x_init.copy() for _ in range(K1)]
    W = [x_init.copy() for _ in range(K1)]
    for _ in range(n_iter):
        X = agents(W, X)
        Z = G([2.0 * x - w for x, w in zip(X, W)], beta)
        W = [w + 2.0 * rho * (z - x) for w, z, x in zip(W, Z, X)]
    return X[0], X, W


def gaussian_taps(std: float, radius: int = 3) -> np.ndarray:
    """Normalised sampled Gaussian, 2 radius + 1 taps."""
    t = np.arange(-radius, radius + 1, dtype=np.float64)
    w = np.exp(-0.5 * t * t / (std * std))
    return w / w.sum()


def blur_axis(x: np.ndarray, taps: np.ndarray, axis: int) -> np.ndarray:
    """Symmetric 1D smoothing of x [frames][nz][ny][nx] along axis (0 = x,
    1 = y, 2 = z), values outside the volume taken as zero."""
    ax = 3 - axis
    r = len(taps) // 2
    pad = [(0, 0)] * x.ndim
    pad[ax] = (r, r)
    xp = np.pad(x, pad)
    out = np.zeros_like(x, dtype=np.float64)
    n = x.shape[ax]
    for k, w in enumerate(taps):
        sl = [slice(None)] * x.ndim
        sl[ax] = slice(k, k + n)
        out += w * xp[tuple(sl)]
    return out


PLANES = ((0, 1), (1, 2), (2, 0))     # xy, yz, zx


def plane_smoother(x: np.ndarray, k: int, std: float) -> np.ndarray:
    """Stand-in prior agent H_k (k = 1, 2, 3): Gaussian smoothing within the
    xy, yz or zx planes.  Symmetric with eigenvalues in (0, 1], hence the
    proximal map of a convex quadratic."""
    taps = gaussian_taps(std)
    a, b = PLANES[k - 1]
    return blur_axis(blur_axis(x, taps, a), taps, b)
