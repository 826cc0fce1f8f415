"""Pins of the DnCNN-17 oracle (Section VI-4): gradients by central finite
differences, the normalisation's invariants, inference with running
statistics, and the folded inference network."""
import numpy as np
import pytest

from oracle import dncnn


@pytest.fixture(scope="module")
def batch():
    rng = np.random.default_rng(7)
    v = rng.uniform(0, 255, size=(2, 8, 8))
    target = np.clip(v + rng.normal(0, 10, size=v.shape), 0, 255)
    sigma = np.array([30.0, 400.0])
    blob = dncnn.init_params(3)
    w1, b1, mids, w17, b17 = dncnn.unpack(blob)
    w17 *= 10.0                                   # make the residual matter
    for _, g, b in mids:
        g[:] = rng.uniform(0.5, 1.5, size=g.shape)
        b[:] = rng.normal(0, 0.1, size=b.shape)
    return v, sigma, target, blob


def test_layout():
    w1, b1, mid0, w17, b17, total = dncnn.offsets()
    assert (w1, b1, mid0) == (0, 1152, 1216) and total == 1216 + 15 * (36864 + 128) + 577
    assert dncnn.param_count() == dncnn.init_params(0).size


def test_gradients_by_finite_differences(batch):
    v, sigma, target, blob = batch
    loss, grad, _ = dncnn.loss_and_grad(blob, v, sigma, target)
    _, b1, mid0, w17, b17, _ = dncnn.offsets()
    idx = [5, b1 + 3, mid0 + 17, mid0 + 36864 + 2, mid0 + 36864 + 64 + 9, mid0 + 7 * dncnn.MID_STRIDE + 1000,
           mid0 + 14 * dncnn.MID_STRIDE + 36864 + 63, w17 + 100, b17]
    h = 1e-5
    for i in idx:
        bp, bm = blob.copy(), blob.copy()
        bp[i] += h
        bm[i] -= h
        lp = dncnn.loss_and_grad(bp, v, sigma, target)[0]
        lm = dncnn.loss_and_grad(bm, v, sigma, target)[0]
        fd = (lp - lm) / (2 * h)
        assert grad[i] == pytest.approx(fd, rel=2e-4, abs=1e-9), f"parameter {i}"


def test_normalisation_invariants(batch):
    v, sigma, target, blob = batch
    _, c = dncnn.forward(blob, v, sigma, train=True, keep=True)
    for zhat, (mu, var) in zip(c["zhat"], c["stats"]):
        assert np.allclose(zhat.mean(axis=(0, 1, 2)), 0.0, atol=1e-12)
        assert np.allclose(zhat.var(axis=(0, 1, 2)), var / (var + dncnn.BN_EPS), rtol=1e-10)


def test_running_statistics_and_inference(batch):
    v, sigma, target, blob = batch
    out_train, c = dncnn.forward(blob, v, sigma, train=True, keep=True)
    run = np.concatenate([np.concatenate([mu, var]) for mu, var in c["stats"]])
    out_eval = dncnn.forward(blob, v, sigma, running=run, train=False)
    assert np.max(np.abs(out_eval - out_train)) < 1e-9
    r0 = dncnn.init_running()
    r1 = dncnn.update_running(r0, c["stats"]).reshape(15, 2, 64)
    mu0, var0 = c["stats"][0]
    assert np.allclose(r1[0, 0], 0.1 * mu0) and np.allclose(r1[0, 1], 0.9 + 0.1 * var0)


def test_folded_network_equals_inference(batch):
    v, sigma, target, blob = batch
    rng = np.random.default_rng(4)
    run = np.concatenate([np.concatenate([rng.normal(0, 0.3, 64), rng.uniform(0.2, 2.0, 64)]) for _ in range(15)])
    a = dncnn.forward(blob, v, sigma, running=run, train=False)
    b = dncnn.forward_folded(dncnn.fold(blob, run), v, sigma)
    assert np.max(np.abs(a - b)) < 1e-9


def test_backward_from_a_stored_cache(batch):
    # the gradient formed from stored activations and pre-normalisation
    # values (statistics re-derived from z) equals the one of the forward
    # pass that produced them; a changed activation changes it
    v, sigma, target, blob = batch
    out, c = dncnn.forward(blob, v, sigma, train=True, keep=True)
    loss, grad, stats = dncnn.loss_and_grad(blob, v, sigma, target)
    c2 = dncnn.cache_from_stored(c["x0"], c["a"], c["z"])
    loss2, grad2, stats2 = dncnn.backward(blob, c2, out, target)
    assert loss2 == loss and np.array_equal(grad2, grad)
    for (m1, v1), (m2, v2) in zip(stats, stats2):
        assert np.array_equal(m1, m2) and np.array_equal(v1, v2)
    a = [t.copy() for t in c["a"]]
    a[3][0, 2, 2, :] += 0.5
    _, grad3, _ = dncnn.backward(blob, dncnn.cache_from_stored(c["x0"], a, c["z"]), out, target)
    assert not np.array_equal(grad3, grad)
