"""Pins of the learned-denoiser oracle (forward, backward, Adam)."""
import numpy as np
import pytest

from oracle import cnn


def test_param_count():
    # 2*9*64+64 + 6*(64*9*64+64) + 64*9+1
    assert cnn.param_count() == 1216 + 6 * 36928 + 577 == 223361


def test_zero_last_layer_is_identity():
    blob = cnn.init_params(0)
    layers = cnn.unpack(blob)
    layers[-1][0][:] = 0.0
    layers[-1][1][:] = 0.0
    v = np.random.default_rng(1).uniform(0, 255, size=(2, 5, 7))
    assert np.array_equal(cnn.forward(cnn.pack(layers), v, [10.0, 300.0]), v)


def test_single_pixel_convolution_by_hand():
    # one 3x3 image: the centre output sees all nine taps, the corner four
    rng = np.random.default_rng(2)
    x = rng.normal(size=(1, 3, 3, 2))
    w = rng.normal(size=(4, 3, 3, 2))
    b = rng.normal(size=4)
    out = cnn.conv3x3(x, w, b)
    centre = b + sum(w[:, dy, dx, :] @ x[0, dy, dx, :] for dy in range(3) for dx in range(3))
    assert np.allclose(out[0, 1, 1], centre)
    corner = b + sum(w[:, dy, dx, :] @ x[0, dy - 1, dx - 1, :] for dy in (1, 2) for dx in (1, 2))
    assert np.allclose(out[0, 0, 0], corner)


def test_network_input_channels():
    v = np.full((1, 2, 2), 51.0)
    inp = cnn.network_input(v, [510.0])
    assert np.allclose(inp[..., 0], 0.2) and np.allclose(inp[..., 1], 1.0)


def test_gradient_matches_finite_differences():
    rng = np.random.default_rng(3)
    blob = cnn.init_params(4)
    layers = cnn.unpack(blob)
    layers[-1][0][:] *= 10.0                  # a last layer big enough to matter
    blob = cnn.pack(layers)
    v = rng.uniform(0, 255, size=(2, 5, 6))
    tgt = v + rng.normal(0, 20, size=v.shape)
    sig = np.array([25.0, 40.0])
    loss, grad = cnn.loss_and_grad(blob, v, sig, tgt)
    sizes = [int(np.prod(w)) + b[0] for w, b in cnn.layer_shapes()]
    starts = np.concatenate([[0], np.cumsum(sizes)[:-1]])
    idx = []
    for s, n in zip(starts, sizes):
        idx += list(rng.choice(np.arange(s, s + n), size=3, replace=False))
        idx.append(s + n - 1)                 # a bias
    h = 1e-6
    for i in idx:
        bp, bm = blob.copy(), blob.copy()
        bp[i] += h
        bm[i] -= h
        fd = (cnn.loss_and_grad(bp, v, sig, tgt)[0] - cnn.loss_and_grad(bm, v, sig, tgt)[0]) / (2 * h)
        assert abs(fd - grad[i]) <= 1e-6 * max(1e-3, abs(grad[i])) + 1e-10, (i, fd, grad[i])


def test_adam_first_step_is_signed_lr():
    g = np.array([0.5, -2.0, 1e-3])
    p, m, v = cnn.adam_step(np.zeros(3), np.zeros(3), np.zeros(3), g, 1, 0.01)
    # m_hat = g, v_hat = g^2 on the first step
    assert np.allclose(p, -0.01 * g / (np.abs(g) + 1e-8))


def test_overfits_a_tiny_batch():
    rng = np.random.default_rng(5)
    v = rng.uniform(0, 255, size=(1, 6, 6))
    tgt = np.clip(v + 30.0, 0, 255)
    blob = cnn.init_params(6)
    m = np.zeros_like(blob)
    s = np.zeros_like(blob)
    l0 = cnn.loss_and_grad(blob, v, [20.0], tgt)[0]
    for t in range(1, 61):
        loss, g = cnn.loss_and_grad(blob, v, [20.0], tgt)
        blob, m, s = cnn.adam_step(blob, m, s, g, t, 1e-3)
    assert loss < 0.2 * l0
