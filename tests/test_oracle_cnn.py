"""Pins of the FP64 warm-start network oracle: central finite differences,
special kernels, and cross-checks against a library conv3d / autograd / Adam
(torch on the CPU in float64, an independent implementation)."""
import numpy as np
import pytest
import torch

from oracle import cnn


def _rand_params(seed, scale=0.3):
    rng = np.random.default_rng(seed)
    out = []
    for li in range(4):
        ci, co = cnn.CHANNELS[li], cnn.CHANNELS[li + 1]
        out.append((rng.standard_normal((co, ci, 3, 3, 3)) * scale / np.sqrt(ci * 27) * 3,
                    rng.standard_normal(co) * 0.05))
    return out


def test_identity_kernel_and_zero_weights():
    rng = np.random.default_rng(0)
    x = rng.standard_normal((2, 3, 5, 6, 7))
    w = np.zeros((3, 3, 3, 3, 3))
    for c in range(3):
        w[c, c, 1, 1, 1] = 1.0
    assert np.array_equal(cnn.conv3d(x, w, np.zeros(3)), x)
    b = np.array([0.5, -1.0])
    out = cnn.conv3d(x, np.zeros((2, 3, 3, 3, 3)), b)
    assert np.array_equal(out, np.broadcast_to(b[None, :, None, None, None], out.shape))
    # a pure shift kernel moves the volume by one voxel (zero padding at the edge)
    w = np.zeros((1, 1, 3, 3, 3))
    w[0, 0, 1, 1, 2] = 1.0          # reads x[..., i + 1]
    out = cnn.conv3d(x[:, :1], w, np.zeros(1))
    assert np.array_equal(out[..., :-1], x[:, :1, ..., 1:]) and (out[..., -1] == 0).all()


def test_conv3d_matches_library_conv():
    rng = np.random.default_rng(1)
    x = rng.standard_normal((2, 4, 6, 5, 7))
    w = rng.standard_normal((3, 4, 3, 3, 3))
    b = rng.standard_normal(3)
    ref = torch.nn.functional.conv3d(torch.from_numpy(x), torch.from_numpy(w), torch.from_numpy(b), padding=1)
    assert np.allclose(cnn.conv3d(x, w, b), ref.numpy(), rtol=1e-12, atol=1e-12)


def test_network_gradients_match_autograd():
    rng = np.random.default_rng(2)
    params = _rand_params(3)
    inp = rng.standard_normal((2, 2, 6, 7, 5))
    target = rng.standard_normal((2, 1, 6, 7, 5))
    out, cache = cnn.forward(params, inp)
    loss, dout = cnn.mse(out, target)
    grads = cnn.backward(params, cache, dout)
    tp = [(torch.tensor(w, requires_grad=True), torch.tensor(b, requires_grad=True)) for w, b in params]
    h = torch.from_numpy(inp)
    for li, (w, b) in enumerate(tp):
        h = torch.nn.functional.conv3d(h, w, b, padding=1)
        if li < 3:
            h = torch.relu(h)
    pred = torch.from_numpy(inp[:, 0:1]) + h
    tl = ((pred - torch.from_numpy(target)) ** 2).mean()
    tl.backward()
    assert abs(tl.item() - loss) <= 1e-12 * abs(loss)
    for (gw, gb), (w, b) in zip(grads, tp):
        assert np.allclose(gw, w.grad.numpy(), rtol=1e-10, atol=1e-12)
        assert np.allclose(gb, b.grad.numpy(), rtol=1e-10, atol=1e-12)


def test_scaled_network_matches_unscaled_definition():
    """x0 = v + c_o f(v/c_v, g/c_g): the scales only rescale the inputs and the output."""
    rng = np.random.default_rng(8)
    params = _rand_params(9)
    inp = rng.standard_normal((1, 2, 4, 5, 6))
    cv, cg, co = 0.05, 0.002, 0.01
    a, _ = cnn.forward(params, inp, scale=(cv, cg, co))
    scaled = np.concatenate([inp[:, 0:1] / cv, inp[:, 1:2] / cg], axis=1)
    b, _ = cnn.forward(params, scaled)
    assert np.allclose(a, inp[:, 0:1] + co * (b - scaled[:, 0:1]), rtol=1e-12, atol=1e-14)


def test_bf16_backward_rounds_at_the_documented_points():
    rng = np.random.default_rng(10)
    params = _rand_params(11)
    inp = rng.standard_normal((1, 2, 4, 4, 4))
    target = rng.standard_normal((1, 1, 4, 4, 4))
    out, cache = cnn.forward(params, inp, bf16=True, scale=0.5)
    grads = cnn.backward(params, cache, cnn.mse(out, target)[1])
    out64, cache64 = cnn.forward(params, inp, scale=0.5)
    grads64 = cnn.backward(params, cache64, cnn.mse(out64, target)[1])
    # bf16 storage changes the result at the bf16 level, not more
    for (gw, gb), (hw, hb) in zip(grads, grads64):
        assert np.linalg.norm(gw - hw) <= 0.05 * np.linalg.norm(hw)
    # the layer inputs of the bf16 path are bf16 numbers
    for h, wq, a in cache["layers"]:
        assert np.array_equal(h, cnn.bf16_round(h)) and np.array_equal(wq, cnn.bf16_round(wq))


def test_network_gradients_central_differences():
    rng = np.random.default_rng(4)
    params = _rand_params(5)
    inp = rng.standard_normal((1, 2, 4, 5, 4))
    target = rng.standard_normal((1, 1, 4, 5, 4))

    def loss_of(p):
        return cnn.mse(cnn.forward(p, inp)[0], target)[0]

    out, cache = cnn.forward(params, inp)
    grads = cnn.backward(params, cache, cnn.mse(out, target)[1])
    vec = cnn.flatten(params)
    gvec = cnn.flatten(grads)
    h = 1e-6
    for k in rng.choice(len(vec), size=40, replace=False):
        e = np.zeros_like(vec)
        e[k] = h
        fd = (loss_of(cnn.unflatten(vec + e)) - loss_of(cnn.unflatten(vec - e))) / (2 * h)
        assert abs(fd - gvec[k]) <= 1e-7 * max(1.0, abs(fd)), (k, fd, gvec[k])


def test_adam_matches_library_adam():
    rng = np.random.default_rng(6)
    params = _rand_params(7)
    tp = [torch.tensor(a) for wb in params for a in wb]
    opt = torch.optim.Adam(tp, lr=1e-3, betas=(0.9, 0.999), eps=1e-8)
    state = {}
    p = params
    for step in range(3):
        grads = [(rng.standard_normal(w.shape), rng.standard_normal(b.shape)) for w, b in params]
        for t, g in zip(tp, [a for wb in grads for a in wb]):
            t.grad = torch.from_numpy(g.copy())
        opt.step()
        p = cnn.adam(p, grads, state)
    for a, t in zip([a for wb in p for a in wb], tp):
        assert np.allclose(a, t.numpy(), rtol=1e-12, atol=1e-14)


def test_bf16_rounding():
    vals = np.array([1.0, 1.00390625, 1.005859375, 1.0 + 2 ** -9, -3.0e-5, 0.0])
    r = cnn.bf16_round(vals)
    # spacing at 1 is 2^-7: 1 + 2^-8 is a tie and goes to the even 1.0; 1 + 1.5*2^-8 rounds up
    # to 1 + 2^-7; 1 + 2^-9 rounds down
    assert r[0] == 1.0 and r[1] == 1.0 and r[2] == 1.0078125 and r[3] == 1.0
    t = torch.tensor(vals, dtype=torch.float32).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(r, t)
    assert cnn.n_params() == 15169


# ---- the 2.5D denoiser (five time points as channels, 3x3 kernels)

def _den_params(seed):
    rng = np.random.default_rng(seed)
    out = []
    for li in range(4):
        ci, co = cnn.DENOISER_CHANNELS[li], cnn.DENOISER_CHANNELS[li + 1]
        out.append((rng.standard_normal((co, ci, 3, 3)) / np.sqrt(ci * 9) * 1.5, rng.standard_normal(co) * 0.05))
    return out


def _torch_denoiser(params, stack, c_in, c_o):
    """The denoiser with torch's conv2d (float64): x = s_2 + c_o f(stack / c_in)."""
    tp = [(torch.tensor(w, requires_grad=True), torch.tensor(b, requires_grad=True)) for w, b in params]
    h = torch.from_numpy(stack) / c_in
    for li, (w, b) in enumerate(tp):
        h = torch.nn.functional.conv2d(h, w, b, padding=1)
        if li < 3:
            h = torch.relu(h)
    return torch.from_numpy(stack[:, 2]) + c_o * h[:, 0], tp


def test_denoiser_matches_library_conv2d_and_autograd():
    """The depth-1 embedding used for the 2D network equals torch's conv2d
    network, values and parameter gradients (an independent implementation)."""
    rng = np.random.default_rng(20)
    params = _den_params(21)
    stack = rng.standard_normal((3, 5, 7, 9))
    target = rng.standard_normal((3, 7, 9))
    c_in, c_o = 0.7, 0.3
    x, cache = cnn.den_forward(params, stack, scale=(c_in, c_o))
    loss, dx = cnn.mse(x, target)
    grads = cnn.den_backward(params, cache, dx)
    ref, tp = _torch_denoiser(params, stack, c_in, c_o)
    assert np.allclose(x, ref.detach().numpy(), rtol=1e-12, atol=1e-12)
    tl = ((ref - torch.from_numpy(target)) ** 2).mean()
    tl.backward()
    assert abs(tl.item() - loss) <= 1e-12 * abs(loss)
    for (gw, gb), (w, b) in zip(grads, tp):
        assert gw.shape == w.shape
        assert np.allclose(gw, w.grad.numpy(), rtol=1e-10, atol=1e-12)
        assert np.allclose(gb, b.grad.numpy(), rtol=1e-10, atol=1e-12)


def test_denoiser_parameter_layout():
    assert cnn.den_n_params() == 5521
    p = _den_params(22)
    vec = cnn.flatten(p)
    assert vec.size == 5521
    back = cnn.den_unflatten(vec)
    assert all(np.array_equal(a, c) and np.array_equal(b, d) for (a, b), (c, d) in zip(p, back))
    # W_1[o][i][ky][kx] sits at (o * 5 + i) * 9 + 3 ky + kx, then b_1 after 16 * 5 * 9 weights
    assert vec[(3 * 5 + 4) * 9 + 3 * 2 + 1] == p[0][0][3, 4, 2, 1]
    assert vec[16 * 5 * 9 + 7] == p[0][1][7]
