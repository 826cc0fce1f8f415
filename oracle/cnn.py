"""FP64 oracle of the learned IDA denoiser: forward, backward, loss, Adam.

TEST INFRASTRUCTURE ONLY: nothing in the product path imports this module.

The paper's learned denoiser is DnCNN (Section VI-4: 17 layers of 3x3
convolutions with 64 channels, batch normalisation and ReLU), whose trained
weights are not available.  The stand-in is smaller and trained here:

  input    2 channels: v / 255 and a constant map min(sigma, 255) / 255
  layer 1  3x3 conv 2 -> 64, bias, ReLU
  2 .. 7   3x3 conv 64 -> 64, bias, ReLU
  layer 8  3x3 conv 64 -> 1, bias
  output   D(v) = v - 255 * f(v, sigma)   (the network predicts the residual)

Convolutions are 'same' with zero padding; no batch normalisation (a
documented departure from DnCNN).  Loss: mean squared error between D(v)/255
and the target/255 over all pixels of the batch.  Optimiser: Adam with the
usual bias correction (beta1 0.9, beta2 0.999, eps 1e-8).

Parameter blob (float32 on the device, float64 here), layer after layer:
weights [C_out][3][3][C_in] (tap = 3 dy + dx, dy, dx in 0..2 for offsets
-1..1), then bias [C_out].

Parity: pinned by tests/test_oracle_cnn.py with central finite differences of
the loss in float64, a zero last layer giving the identity, and an explicit
single-pixel convolution.
"""

import math

import numpy as np

CH = 64
LAYERS = [(2, CH)] + [(CH, CH)] * 6 + [(CH, 1)]
BETA1, BETA2, EPS = 0.9, 0.999, 1e-8


def layer_shapes():
    return [((co, 3, 3, ci), (co,)) for ci, co in LAYERS]


def param_count():
    return sum(int(np.prod(w)) + b[0] for w, b in layer_shapes())


def unpack(blob):
    """Flat blob -> list of (W[co,3,3,ci], b[co]) views."""
    blob = np.asarray(blob, dtype=np.float64)
    out, o = [], 0
    for ws, bs in layer_shapes():
        nw = int(np.prod(ws))
        out.append((blob[o:o + nw].reshape(ws), blob[o + nw:o + nw + bs[0]]))
        o += nw + bs[0]
    return out


def pack(layers):
    return np.concatenate([np.concatenate([w.reshape(-1), b]) for w, b in layers])


def init_params(seed):
    """He-normal weights (std sqrt(2 / (9 C_in))), zero biases; last layer
    scaled by 0.1 so the untrained network starts near the identity."""
    rng = np.random.default_rng(seed)
    layers = []
    for i, (ci, co) in enumerate(LAYERS):
        w = rng.normal(0.0, math.sqrt(2.0 / (9 * ci)), size=(co, 3, 3, ci))
        if i == len(LAYERS) - 1:
            w *= 0.1
        layers.append((w, np.zeros(co)))
    return pack(layers)


def conv3x3(x, w, b):
    """x [N,H,W,ci], w [co,3,3,ci], b [co] -> [N,H,W,co]; zero padding."""
    N, H, W, ci = x.shape
    xp = np.pad(x, ((0, 0), (1, 1), (1, 1), (0, 0)))
    out = np.zeros((N, H, W, w.shape[0])) + b
    for dy in range(3):
        for dx in range(3):
            out += xp[:, dy:dy + H, dx:dx + W, :] @ w[:, dy, dx, :].T
    return out


def conv3x3_input_grad(g, w):
    """Gradient of conv3x3 w.r.t. its input: g [N,H,W,co] -> [N,H,W,ci]."""
    N, H, W, co = g.shape
    gp = np.pad(g, ((0, 0), (1, 1), (1, 1), (0, 0)))
    out = np.zeros((N, H, W, w.shape[3]))
    for dy in range(3):
        for dx in range(3):
            # output pixel p used input p + (dy-1, dx-1); so input q receives
            # from output q - (dy-1, dx-1)
            out += gp[:, 2 - dy:2 - dy + H, 2 - dx:2 - dx + W, :] @ w[:, dy, dx, :]
    return out


def conv3x3_weight_grad(x, g):
    """dL/dW [co,3,3,ci] and dL/db [co] from input x and output gradient g."""
    N, H, W, ci = x.shape
    co = g.shape[3]
    xp = np.pad(x, ((0, 0), (1, 1), (1, 1), (0, 0)))
    gw = np.zeros((co, 3, 3, ci))
    gf = g.reshape(-1, co)
    for dy in range(3):
        for dx in range(3):
            gw[:, dy, dx, :] = gf.T @ xp[:, dy:dy + H, dx:dx + W, :].reshape(-1, ci)
    return gw, gf.sum(axis=0)


def network_input(v, sigma):
    """v [N,H,W] pixels, sigma [N] -> [N,H,W,2]."""
    v = np.asarray(v, dtype=np.float64)
    s = np.minimum(np.asarray(sigma, dtype=np.float64), 255.0) / 255.0
    return np.stack([v / 255.0, np.broadcast_to(s[:, None, None], v.shape)], axis=-1)


def forward(blob, v, sigma, keep=False):
    """D(v) for a batch; with keep=True also the layer inputs for backward."""
    layers = unpack(blob)
    a = network_input(v, sigma)
    acts = [a]
    for i, (w, b) in enumerate(layers):
        a = conv3x3(a, w, b)
        if i < len(layers) - 1:
            a = np.maximum(a, 0.0)
        acts.append(a)
    out = np.asarray(v, dtype=np.float64) - 255.0 * a[..., 0]
    return (out, acts) if keep else out


def backward(blob, acts, out, target):
    """MSE loss of out/255 against target/255 and its gradient blob, given
    the forward cache: acts[0] the network input, acts[i] (i = 1..7) the
    output of layer i after its ReLU (its sign gives the ReLU's derivative),
    and `out` = v - 255 f.  The cache may come from another evaluation of the
    same network (for example the values a device stored), so that each
    layer's gradient can be checked from the same inputs."""
    layers = unpack(blob)
    out = np.asarray(out, dtype=np.float64)
    n = out.size
    diff = (out - np.asarray(target, dtype=np.float64)) / 255.0
    loss = float(np.sum(diff * diff) / n)
    # d loss / d out = 2 diff / (255 n); out = v - 255 f  ->  d/df = -2 diff / n
    g = (-2.0 * diff / n)[..., None]
    grads = [None] * len(layers)
    for i in range(len(layers) - 1, -1, -1):
        w, _ = layers[i]
        if i < len(layers) - 1:
            g = g * (np.asarray(acts[i + 1]) > 0.0)
        grads[i] = conv3x3_weight_grad(np.asarray(acts[i], dtype=np.float64), g)
        if i > 0:
            g = conv3x3_input_grad(g, w)
    return loss, pack(grads)


def loss_and_grad(blob, v, sigma, target):
    """MSE loss of D(v)/255 against target/255 and its gradient blob."""
    out, acts = forward(blob, v, sigma, keep=True)
    return backward(blob, acts, out, target)


def adam_step(blob, m, v, grad, step, lr):
    """One Adam update (step counts from 1); returns new (blob, m, v)."""
    m = BETA1 * m + (1.0 - BETA1) * grad
    v = BETA2 * v + (1.0 - BETA2) * grad * grad
    mh = m / (1.0 - BETA1 ** step)
    vh = v / (1.0 - BETA2 ** step)
    return blob - lr * mh / (np.sqrt(vh) + EPS), m, v
