"""FP64 oracle of the MACE outer loop (TEST INFRASTRUCTURE ONLY).

Paper Sec. III: agents F = [L(W_0); H_1(W_1); ...; H_K(W_K)] (eq. (6)),
the averaging operator G (eqs. (8), (9)) with weight beta, and
Algorithm 1 (partial-update Mann iteration):  starting from X = W = copies of
x^(0), repeat  X <- F~(W; X),  Z <- G(2X - W),  W <- W + 2 rho (Z - X);
the reconstruction is X_0.
"""
from __future__ import annotations

import numpy as np


def weighted_mean(W, beta: float):
    """eq. (9): W_0/(1+beta) + beta/(1+beta) * mean_k W_k."""
    K = len(W) - 1
    return W[0] / (1.0 + beta) + (beta / (1.0 + beta)) * (sum(W[1:]) / K)


def G(W, beta: float):
    """eq. (8): every component replaced by the weighted mean."""
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


# ---------------------------------------------------------------------------
# 2.5D CNN denoiser agents (Sec. IV): one trained network applied slice by
# slice in the xy, yz and zx planes, its channels the same slice at five
# neighbouring time points, its output the denoised centre slice.
# Plane k = 1: images (y, x) per (t, z); k = 2: images (z, y) per (t, x);
# k = 3: images (z, x) per (t, y).  Reading: at the first and last two time
# points the missing neighbours repeat the end frame (indices clamped).
# ---------------------------------------------------------------------------

def to_slices(W: np.ndarray, k: int) -> np.ndarray:
    """[T][Z][Y][X] -> images [T][n_slices][h][w] of plane k."""
    if k == 1:
        return W                                # [T][Z][Y][X]: images (y, x)
    if k == 2:
        return np.transpose(W, (0, 3, 1, 2))    # [T][X][Z][Y]: images (z, y)
    return np.transpose(W, (0, 2, 1, 3))        # [T][Y][Z][X]: images (z, x)


def from_slices(S: np.ndarray, k: int) -> np.ndarray:
    """Inverse of to_slices."""
    if k == 1:
        return S
    if k == 2:
        return np.transpose(S, (0, 2, 3, 1))
    return np.transpose(S, (0, 2, 1, 3))


def time_stack(W: np.ndarray, k: int) -> np.ndarray:
    """The denoiser inputs of plane k: [T * n_slices][5][h][w], channel c of
    slice (t, s) being slice s at time clamp(t + c - 2)."""
    S = to_slices(W, k)
    T = S.shape[0]
    chans = [S[[min(max(t + d, 0), T - 1) for t in range(T)]] for d in (-2, -1, 0, 1, 2)]
    st = np.stack(chans, axis=2)                # [T][n_slices][5][h][w]
    return st.reshape(-1, 5, S.shape[2], S.shape[3])


def cnn_agent(W: np.ndarray, k: int, params2d, scales) -> np.ndarray:
    """H_k(W): the 2.5D denoiser in plane k (BF16 rounding at the GPU's points)."""
    from oracle import cnn
    W = W.astype(np.float64)
    x, _ = cnn.den_forward(params2d, time_stack(W, k), bf16=True, scale=scales)
    S = to_slices(W, k)
    return from_slices(x.reshape(S.shape), k)
