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
