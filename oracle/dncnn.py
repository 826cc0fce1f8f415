"""FP64 oracle of DnCNN-17 with batch normalisation as an IDA denoiser:
forward (training and inference mode), backward, loss, running statistics,
and the folding of normalisation into the convolutions.

TEST INFRASTRUCTURE ONLY: nothing in the product path imports this module.

The network of Section VI-4 (Zhang et al.'s DnCNN with 17 layers):

  layer 1      3x3 conv -> 64, bias, ReLU
  layers 2-16  3x3 conv 64 -> 64 (no bias), batch normalisation (per-channel
               gamma, beta), ReLU
  layer 17     3x3 conv 64 -> 1, bias
  output       D(v) = v - 255 f          (the network predicts the residual)

Readings where the paper is silent: the input has the same two channels as
the smaller learned denoiser, v / 255 and the constant map
min(sigma, 255) / 255 (IDA's sigma spans several hundred grey levels, more
than one blind network covers); normalisation uses the batch mean and the
biased batch variance with eps = 1e-5 in training, and running estimates
(momentum 0.1, biased variance, starting at mean 0 and variance 1) at
inference; convolutions are 'same' with zero padding.

Parameter blob (float32 on the device, float64 here): W1 [64][3][3][2], b1
[64]; then for each of the 15 middle layers W [64][3][3][64], gamma [64],
beta [64]; then W17 [1][3][3][64], b17 [1].  Running statistics: for each
middle layer mean [64] then variance [64].

Every value is float64.  `backward` takes the forward cache as an argument,
so that the gradient can also be formed from activations and
pre-normalisation values that another evaluation of the network stored
(`cache_from_stored` derives the batch statistics and the normalised values
from the stored pre-normalisation values, as the forward pass does).

Parity: pinned by tests/test_oracle_dncnn.py: central finite differences of
the loss (weights, gamma, beta), the normalised values' zero mean and unit
variance per channel, inference with running statistics equal to the batch
statistics reproducing training mode, and the folded network reproducing
inference mode.
"""

import math

import numpy as np

from . import cnn as ocnn

CH = 64
N_MID = 15
BN_EPS = 1e-5
MOMENTUM = 0.1
MID_STRIDE = CH * 9 * CH + 2 * CH


def offsets():
    """(w1, b1, mid0, w17, b17, total) offsets in the blob."""
    w1 = 0
    b1 = w1 + CH * 9 * 2
    mid0 = b1 + CH
    w17 = mid0 + N_MID * MID_STRIDE
    b17 = w17 + 9 * CH
    return w1, b1, mid0, w17, b17, b17 + 1


def param_count():
    return offsets()[-1]


def running_count():
    return N_MID * 2 * CH


def unpack(blob):
    """-> (W1, b1, [(W, gamma, beta)] * 15, W17, b17) as float64 views."""
    blob = np.asarray(blob, dtype=np.float64)
    w1, b1, mid0, w17, b17, _ = offsets()
    mids = []
    for l in range(N_MID):
        o = mid0 + l * MID_STRIDE
        mids.append((blob[o:o + CH * 9 * CH].reshape(CH, 3, 3, CH), blob[o + CH * 9 * CH:o + CH * 9 * CH + CH],
                     blob[o + CH * 9 * CH + CH:o + MID_STRIDE]))
    return (blob[w1:b1].reshape(CH, 3, 3, 2), blob[b1:mid0], mids, blob[w17:b17].reshape(1, 3, 3, CH),
            blob[b17:b17 + 1])


def pack(w1, b1, mids, w17, b17):
    parts = [w1.reshape(-1), b1]
    for w, g, b in mids:
        parts += [w.reshape(-1), g, b]
    parts += [w17.reshape(-1), b17]
    return np.concatenate(parts)


def init_params(seed):
    """He-normal weights, zero biases, gamma 1, beta 0; the last layer scaled
    by 0.1 so that the untrained network starts near the identity."""
    rng = np.random.default_rng(seed)
    w1 = rng.normal(0.0, math.sqrt(2.0 / 18.0), size=(CH, 3, 3, 2))
    mids = [(rng.normal(0.0, math.sqrt(2.0 / (9 * CH)), size=(CH, 3, 3, CH)), np.ones(CH), np.zeros(CH))
            for _ in range(N_MID)]
    w17 = 0.1 * rng.normal(0.0, math.sqrt(2.0 / (9 * CH)), size=(1, 3, 3, CH))
    return pack(w1, np.zeros(CH), mids, w17, np.zeros(1))


def init_running():
    r = np.zeros((N_MID, 2, CH))
    r[:, 1, :] = 1.0
    return r.reshape(-1)


def _normalise(z):
    """Batch statistics of one normalisation (mean and biased variance per
    channel over every pixel of the batch) and the normalised values."""
    mu = z.mean(axis=(0, 1, 2))
    var = ((z - mu) ** 2).mean(axis=(0, 1, 2))
    return (mu, var), (z - mu) / np.sqrt(var + BN_EPS)


def forward(blob, v, sigma, running=None, train=True, keep=False):
    """D(v) for a batch v [N,H,W], sigma [N].  train=True normalises with the
    batch statistics (returned in the cache as (mean, var) per layer);
    train=False uses `running`."""
    w1, b1, mids, w17, b17 = unpack(blob)
    run = None if running is None else np.asarray(running, dtype=np.float64).reshape(N_MID, 2, CH)
    x0 = ocnn.network_input(v, sigma)
    a = np.maximum(ocnn.conv3x3(x0, w1, b1), 0.0)
    cache = {"x0": x0, "a": [a], "z": [], "zhat": [], "stats": []}
    for l, (w, g, b) in enumerate(mids):
        z = ocnn.conv3x3(a, w, np.zeros(CH))
        if train:
            (mu, var), zhat = _normalise(z)
        else:
            mu, var = run[l, 0], run[l, 1]
            zhat = (z - mu) / np.sqrt(var + BN_EPS)
        a = np.maximum(g * zhat + b, 0.0)
        cache["z"].append(z)
        cache["zhat"].append(zhat)
        cache["stats"].append((mu, var))
        cache["a"].append(a)
    f = ocnn.conv3x3(a, w17, b17)[..., 0]
    out = np.asarray(v, dtype=np.float64) - 255.0 * f
    return (out, cache) if keep else out


def cache_from_stored(x0, a, z):
    """Training-mode forward cache from stored values: the network input x0,
    the 16 activations a_1 .. a_16 (after each ReLU) and the 15
    pre-normalisation values; the batch statistics and normalised values are
    derived from z as in `forward`."""
    cache = {"x0": np.asarray(x0, dtype=np.float64), "a": [np.asarray(t, dtype=np.float64) for t in a],
             "z": [np.asarray(t, dtype=np.float64) for t in z], "zhat": [], "stats": []}
    for zl in cache["z"]:
        st, zhat = _normalise(zl)
        cache["stats"].append(st)
        cache["zhat"].append(zhat)
    return cache


def backward(blob, cache, out, target):
    """Training mode: MSE of out/255 against target/255 (out = D(v)), its
    gradient blob, and the batch statistics [(mean, var)] of the 15
    normalisations, from the forward cache."""
    w1, b1, mids, w17, b17 = unpack(blob)
    c = cache
    out = np.asarray(out, dtype=np.float64)
    n = out.size
    diff = (out - np.asarray(target, dtype=np.float64)) / 255.0
    loss = float(np.sum(diff * diff) / n)
    g = (-2.0 * diff / n)[..., None]                      # dL/df
    gw17, gb17 = ocnn.conv3x3_weight_grad(c["a"][-1], g)
    ga = ocnn.conv3x3_input_grad(g, w17)                  # dL/da_16
    gmids = [None] * N_MID
    for l in range(N_MID - 1, -1, -1):
        w, gam, _ = mids[l]
        gy = ga * (c["a"][l + 1] > 0.0)                   # through the ReLU
        zhat = c["zhat"][l]
        _, var = c["stats"][l]
        cnt = gy.shape[0] * gy.shape[1] * gy.shape[2]
        ggam = (gy * zhat).sum(axis=(0, 1, 2))
        gbet = gy.sum(axis=(0, 1, 2))
        gzh = gy * gam
        gz = ((gzh - gzh.sum(axis=(0, 1, 2)) / cnt - zhat * (gzh * zhat).sum(axis=(0, 1, 2)) / cnt)
              / np.sqrt(var + BN_EPS))
        gw, _ = ocnn.conv3x3_weight_grad(c["a"][l], gz)
        gmids[l] = (gw, ggam, gbet)
        ga = ocnn.conv3x3_input_grad(gz, w)               # dL/da_l
    g1 = ga * (c["a"][0] > 0.0)
    gw1, gb1 = ocnn.conv3x3_weight_grad(c["x0"], g1)
    return loss, pack(gw1, gb1, gmids, gw17, gb17), c["stats"]


def loss_and_grad(blob, v, sigma, target):
    """Training mode: MSE of D(v)/255 against target/255, its gradient blob,
    and the batch statistics [(mean, var)] of the 15 normalisations."""
    out, c = forward(blob, v, sigma, train=True, keep=True)
    return backward(blob, c, out, target)


def update_running(running, stats):
    """Exponential moving average of the batch statistics (momentum 0.1)."""
    r = np.asarray(running, dtype=np.float64).reshape(N_MID, 2, CH).copy()
    for l, (mu, var) in enumerate(stats):
        r[l, 0] = (1.0 - MOMENTUM) * r[l, 0] + MOMENTUM * mu
        r[l, 1] = (1.0 - MOMENTUM) * r[l, 1] + MOMENTUM * var
    return r.reshape(-1)


def fold(blob, running):
    """Inference network without normalisation: middle layer l becomes a
    convolution with weights W s_c and bias beta_c - mean_c s_c per output
    channel c, s = gamma / sqrt(var + eps).  Returns (w1, b1, [(W', b')], w17,
    b17)."""
    w1, b1, mids, w17, b17 = unpack(blob)
    run = np.asarray(running, dtype=np.float64).reshape(N_MID, 2, CH)
    out = []
    for l, (w, g, b) in enumerate(mids):
        s = g / np.sqrt(run[l, 1] + BN_EPS)
        out.append((w * s[:, None, None, None], b - run[l, 0] * s))
    return w1, b1, out, w17, b17


def forward_folded(folded, v, sigma):
    w1, b1, mids, w17, b17 = folded
    a = np.maximum(ocnn.conv3x3(ocnn.network_input(v, sigma), w1, b1), 0.0)
    for w, b in mids:
        a = np.maximum(ocnn.conv3x3(a, w, b), 0.0)
    return np.asarray(v, dtype=np.float64) - 255.0 * ocnn.conv3x3(a, w17, b17)[..., 0]


def adam_step(blob, m, v, grad, step, lr):
    return ocnn.adam_step(blob, m, v, grad, step, lr)
