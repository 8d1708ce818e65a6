"""FP64 oracle of the warm-start network (TEST INFRASTRUCTURE ONLY).

The network is not from the paper: the paper's own denoisers are 2.5D CNNs
(Sec. IV) whose weights are not available.  This is the small 3D network that
predicts a starting point for the proximal-map solve:

    input  c0 = v / c_v,  c1 = g / c_g                    (2 channels)
    h1 = relu(conv(input, W1) + b1)  2 -> 16
    h2 = relu(conv(h1, W2) + b2)    16 -> 16
    h3 = relu(conv(h2, W3) + b3)    16 -> 16
    f  = conv(h3, W4) + b4          16 -> 1
    x0 = v + c_o * f

where g is the data term's backprojected weighted residual at v (scaled to
voxel units) and c_v, c_g, c_o fixed scales stored with the network.  ``conv`` is 3x3x3 cross-correlation
with zero "same" padding.  The GPU path stores weights, layer inputs and the
gradients it feeds back into its matrix cores in bfloat16 and accumulates in
FP32; with ``bf16=True`` this oracle rounds the same tensors at the same
points (round to nearest even) and does everything else in FP64, so the two
differ only by accumulation order.

Every function is the definition written out tap by tap: forward, the input
gradient (each output tap sends its gradient back to the input voxel it
read), the weight gradient (input times output gradient summed over voxels),
mean-squared-error loss, and Adam (Kingma & Ba, ICLR 2015, Algorithm 1).
"""
from __future__ import annotations

import numpy as np

CHANNELS = (2, 16, 16, 16, 1)
TAPS = [(dz, dy, dx) for dz in range(3) for dy in range(3) for dx in range(3)]


def bf16_round(a: np.ndarray) -> np.ndarray:
    """Round to the nearest bfloat16 (ties to even), returned as float64."""
    f = np.ascontiguousarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def conv3d(x: np.ndarray, w: np.ndarray, b: np.ndarray) -> np.ndarray:
    """x [B, Ci, Z, Y, X], w [Co, Ci, 3, 3, 3], b [Co] -> [B, Co, Z, Y, X]."""
    B, Ci, Z, Y, X = x.shape
    xp = np.pad(x, ((0, 0), (0, 0), (1, 1), (1, 1), (1, 1)))
    out = np.zeros((B, w.shape[0], Z, Y, X)) + b[None, :, None, None, None]
    for dz, dy, dx in TAPS:
        if not w[:, :, dz, dy, dx].any():
            continue        # an all-zero tap adds nothing
        patch = xp[:, :, dz:dz + Z, dy:dy + Y, dx:dx + X]
        out += np.einsum("oc,bczyx->bozyx", w[:, :, dz, dy, dx], patch)
    return out


def conv3d_dgrad(dout: np.ndarray, w: np.ndarray) -> np.ndarray:
    """Gradient w.r.t. the input: output voxel p read input voxel p + tap - 1."""
    B, Co, Z, Y, X = dout.shape
    dxp = np.zeros((B, w.shape[1], Z + 2, Y + 2, X + 2))
    for dz, dy, dx in TAPS:
        dxp[:, :, dz:dz + Z, dy:dy + Y, dx:dx + X] += np.einsum("oc,bozyx->bczyx", w[:, :, dz, dy, dx], dout)
    return dxp[:, :, 1:-1, 1:-1, 1:-1]


def conv3d_wgrad(x: np.ndarray, dout: np.ndarray):
    """Gradients w.r.t. weights and bias."""
    B, Ci, Z, Y, X = x.shape
    xp = np.pad(x, ((0, 0), (0, 0), (1, 1), (1, 1), (1, 1)))
    dw = np.zeros((dout.shape[1], Ci, 3, 3, 3))
    for dz, dy, dx in TAPS:
        patch = xp[:, :, dz:dz + Z, dy:dy + Y, dx:dx + X]
        dw[:, :, dz, dy, dx] = np.einsum("bozyx,bczyx->oc", dout, patch)
    db = dout.sum(axis=(0, 2, 3, 4))
    return dw, db


def init_params(seed: int = 0, scale: float = 1.0):
    """He-normal weights, zero biases; the last layer starts small."""
    rng = np.random.default_rng(seed)
    params = []
    for li in range(4):
        ci, co = CHANNELS[li], CHANNELS[li + 1]
        std = np.sqrt(2.0 / (ci * 27)) * scale * (0.1 if li == 3 else 1.0)
        params.append((rng.standard_normal((co, ci, 3, 3, 3)) * std, np.zeros(co)))
    return params


def forward(params, inp: np.ndarray, bf16: bool = False, scale=1.0):
    """inp [B, 2, Z, Y, X] = (v, g) unscaled; scale = c or (c_v, c_g, c_o).
    Returns (x0 [B,1,Z,Y,X], cache)."""
    rnd = bf16_round if bf16 else (lambda a: a)
    cv, cg, co = (scale, scale, scale) if np.isscalar(scale) else scale
    f, cache = _layers(params, rnd(np.concatenate([inp[:, 0:1] / cv, inp[:, 1:2] / cg], axis=1)), rnd)
    return inp[:, 0:1] + co * f, {"layers": cache, "bf16": bf16, "scale": co}


def _layers(params, h, rnd):
    """The four layers on the (already scaled and rounded) input h."""
    cache = []
    for li, (w, b) in enumerate(params):
        wq = rnd(w)
        a = conv3d(h, wq, b)
        cache.append((h, wq, a))
        if li < 3:
            h = rnd(np.maximum(a, 0.0))
        else:
            h = a
    return h, cache


def backward(params, cache, dx0: np.ndarray):
    """Gradients of the loss w.r.t. every (W, b), given d loss / d x0.  With
    bf16 the gradient entering each layer is rounded to bfloat16 (after the
    ReLU mask), as the GPU feeds it to its matrix cores."""
    layers, scale = cache["layers"], cache["scale"]
    rnd = bf16_round if cache["bf16"] else (lambda a: a)
    grads = [None] * 4
    g = rnd(dx0 * scale)
    for li in range(3, -1, -1):
        h, wq, a = layers[li]
        dw, db = conv3d_wgrad(h, g)
        grads[li] = (dw, db)
        if li > 0:
            hp = layers[li - 1]
            g = rnd(conv3d_dgrad(g, wq) * (hp[2] > 0.0))
    return grads


def mse(pred: np.ndarray, target: np.ndarray):
    """loss = mean((pred - target)^2) and its gradient."""
    d = pred - target
    return float(np.mean(d * d)), 2.0 * d / d.size


def adam(params, grads, state, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step; state = {"t": int, "m": [...], "v": [...]} (updated in place)."""
    if not state:
        state["t"] = 0
        state["m"] = [(np.zeros_like(w), np.zeros_like(b)) for w, b in params]
        state["v"] = [(np.zeros_like(w), np.zeros_like(b)) for w, b in params]
    state["t"] += 1
    t = state["t"]
    out = []
    for i, ((w, b), (gw, gb)) in enumerate(zip(params, grads)):
        new = []
        for j, (p, gp) in enumerate(((w, gw), (b, gb))):
            m = b1 * state["m"][i][j] + (1 - b1) * gp
            v = b2 * state["v"][i][j] + (1 - b2) * gp * gp
            state["m"][i] = state["m"][i][:j] + (m,) + state["m"][i][j + 1:]
            state["v"][i] = state["v"][i][:j] + (v,) + state["v"][i][j + 1:]
            mh = m / (1 - b1 ** t)
            vh = v / (1 - b2 ** t)
            new.append(p - lr * mh / (np.sqrt(vh) + eps))
        out.append(tuple(new))
    return out


def flatten(params) -> np.ndarray:
    return np.concatenate([np.concatenate([w.reshape(-1), b.reshape(-1)]) for w, b in params])


def unflatten(vec: np.ndarray):
    out, o = [], 0
    for li in range(4):
        ci, co = CHANNELS[li], CHANNELS[li + 1]
        nw = co * ci * 27
        out.append((vec[o:o + nw].reshape(co, ci, 3, 3, 3).astype(np.float64), vec[o + nw:o + nw + co].astype(np.float64)))
        o += nw + co
    return out


def n_params() -> int:
    return sum(CHANNELS[i + 1] * (CHANNELS[i] * 27 + 1) for i in range(4))


# ---------------------------------------------------------------------------
# The 2.5D denoiser of the multi-slice fusion prior agents (paper Sec. IV):
# the same four layers as a 2D network, 3x3 kernels, channels 5 -> 16 -> 16
# -> 16 -> 1; its five input channels are one 2D slice at time points t-2,
# t-1, t, t+1, t+2 and its output is the denoised centre slice
#     x_t = s_t + c_o f(s_{t-2} / c_in, ..., s_{t+2} / c_in).
# A 2D cross-correlation of an image is the 3D one of the same image as a
# depth-1 volume with the 3x3 kernel as the depth-centre taps of a 3x3x3
# kernel (the other depth taps only ever see the zero padding), so the
# denoiser is evaluated with the functions above on such embedded kernels.
# ---------------------------------------------------------------------------

DENOISER_CHANNELS = (5, 16, 16, 16, 1)


def den_embed(params2d):
    """[(W [co][ci][3][3], b)] -> the equivalent 3x3x3 kernels (depth-centre taps)."""
    out = []
    for w, b in params2d:
        w3 = np.zeros(w.shape[:2] + (3, 3, 3))
        w3[:, :, 1] = w
        out.append((w3, b))
    return out


def den_forward(params2d, stack: np.ndarray, bf16: bool = False, scale=(1.0, 1.0)):
    """stack [B, 5, H, W] = one slice at t-2 .. t+2 (unscaled); scale (c_in, c_o).
    Returns (x [B, H, W], cache)."""
    rnd = bf16_round if bf16 else (lambda a: a)
    c_in, c_o = scale
    f, cache = _layers(den_embed(params2d), rnd(stack[:, :, None] / c_in), rnd)
    return stack[:, 2] + c_o * f[:, 0, 0], {"layers": cache, "bf16": bf16, "scale": c_o}


def den_backward(params2d, cache, dx: np.ndarray):
    """Gradients w.r.t. every (W [co][ci][3][3], b) given d loss / d x [B, H, W]."""
    grads = backward(den_embed(params2d), cache, dx[:, None, None])
    return [(gw[:, :, 1], gb) for gw, gb in grads]


def den_init_params(seed: int = 0, scale: float = 1.0):
    """He-normal 3x3 weights, zero biases; the last layer starts small."""
    rng = np.random.default_rng(seed)
    params = []
    for li in range(4):
        ci, co = DENOISER_CHANNELS[li], DENOISER_CHANNELS[li + 1]
        std = np.sqrt(2.0 / (ci * 9)) * scale * (0.1 if li == 3 else 1.0)
        params.append((rng.standard_normal((co, ci, 3, 3)) * std, np.zeros(co)))
    return params


def den_unflatten(vec: np.ndarray):
    out, o = [], 0
    for li in range(4):
        ci, co = DENOISER_CHANNELS[li], DENOISER_CHANNELS[li + 1]
        nw = co * ci * 9
        out.append((vec[o:o + nw].reshape(co, ci, 3, 3).astype(np.float64), vec[o + nw:o + nw + co].astype(np.float64)))
        o += nw + co
    return out


def den_n_params() -> int:
    return sum(DENOISER_CHANNELS[i + 1] * (DENOISER_CHANNELS[i] * 9 + 1) for i in range(4))
