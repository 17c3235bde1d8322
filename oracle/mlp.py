"""FP64 twin of the learned Zernike surrogate (not in the paper).

A multilayer perceptron maps (tile x, tile y, 32 spectral-overlap features)
to the twelve Noll coefficients c_4..c_15:

    X  = bf16((inputs - mean) / std), zero-padded to 64 columns
    H1 = bf16(relu(X W1^T + b1))        W1: 128 x 64   (columns >= 34 unused)
    H2 = bf16(relu(H1 W2^T + b2))       W2: 128 x 128
    Y  = H2 W3^T + b3                   W3: 16 x 128   (rows >= 12 unused)

The GPU keeps bfloat16 copies of the weights and of every matrix-multiply
operand, and accumulates in FP32.  This twin rounds to bfloat16 at the same
points and accumulates in FP64, so both sides compute the same function up to
accumulation order.  Loss: mean squared error over samples and the twelve
outputs.  Backward (same quantisation points):

    dY  = bf16(2 (Y - T) / (n * 12)),  padded to 16 columns
    dW3 = dY^T H2,  db3 = sum dY,  dZ2 = bf16((dY W3) * [H2 > 0])
    dW2 = dZ2^T H1, db2 = sum dZ2, dZ1 = bf16((dZ2 W2) * [H1 > 0])
    dW1 = dZ1^T X,  db1 = sum dZ1

Adam (Kingma & Ba 2015) with bias correction updates FP32 master weights.
"""

import numpy as np

N_IN = 34
N_IN_PAD = 64
N_HID = 128
N_OUT = 12
N_OUT_PAD = 16
SHAPES = [("W1", (N_HID, N_IN_PAD)), ("b1", (N_HID,)), ("W2", (N_HID, N_HID)), ("b2", (N_HID,)),
          ("W3", (N_OUT_PAD, N_HID)), ("b3", (N_OUT_PAD,))]
N_PARAMS = sum(int(np.prod(s)) for _, s in SHAPES)


def bf16(x):
    """Round float values to the nearest bfloat16 (ties to even), returned as float64.

    bfloat16 keeps the sign, the 8 exponent bits and the top 7 mantissa bits of an
    IEEE float32; rounding adds half an ulp of the kept part, with ties going to the
    even kept pattern."""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = (u + 0x7FFF + lsb) >> 16
    out = (r << 16).astype(np.uint32).view(np.float32).astype(np.float64)
    return np.where(np.isnan(f), np.nan, out)


def unpack(theta):
    """Split a flat parameter vector into named arrays (views)."""
    theta = np.asarray(theta, dtype=np.float64)
    out, o = {}, 0
    for name, shape in SHAPES:
        size = int(np.prod(shape))
        out[name] = theta[o:o + size].reshape(shape)
        o += size
    return out


def init_params(seed=0):
    """He-style uniform initialisation; padded rows/columns are zero."""
    rng = np.random.default_rng(seed)
    p = {}
    w1 = np.zeros((N_HID, N_IN_PAD))
    w1[:, :N_IN] = rng.uniform(-1, 1, (N_HID, N_IN)) * np.sqrt(6.0 / N_IN)
    p["W1"], p["b1"] = w1, np.zeros(N_HID)
    p["W2"], p["b2"] = rng.uniform(-1, 1, (N_HID, N_HID)) * np.sqrt(6.0 / N_HID), np.zeros(N_HID)
    w3 = np.zeros((N_OUT_PAD, N_HID))
    w3[:N_OUT] = rng.uniform(-1, 1, (N_OUT, N_HID)) * np.sqrt(3.0 / N_HID)
    p["W3"], p["b3"] = w3, np.zeros(N_OUT_PAD)
    return np.concatenate([p[name].ravel() for name, _ in SHAPES]).astype(np.float32)


def _inputs(inputs, mean, std):
    x = np.zeros((len(inputs), N_IN_PAD))
    x[:, :N_IN] = (np.asarray(inputs, np.float64) - mean) / std
    return x


def forward(theta, inputs, mean, std, quantize=True):
    """Returns (Y (n, 12), cache)."""
    q = bf16 if quantize else (lambda a: np.asarray(a, np.float64))
    p = unpack(theta)
    w1, w2, w3 = q(p["W1"]), q(p["W2"]), q(p["W3"])
    x = q(_inputs(inputs, mean, std).astype(np.float32)) if quantize else _inputs(inputs, mean, std)
    h1 = q(np.maximum(x @ w1.T + p["b1"], 0.0))
    h2 = q(np.maximum(h1 @ w2.T + p["b2"], 0.0))
    y = h2 @ w3.T + p["b3"]
    return y[:, :N_OUT], {"x": x, "h1": h1, "h2": h2, "w1": w1, "w2": w2, "w3": w3}


def loss_and_grad(theta, inputs, targets, mean, std, quantize=True):
    """Mean squared error and its gradient with respect to the flat parameters."""
    q = bf16 if quantize else (lambda a: np.asarray(a, np.float64))
    n = len(inputs)
    y, c = forward(theta, inputs, mean, std, quantize)
    diff = y - np.asarray(targets, np.float64)
    loss = float(np.sum(diff ** 2) / (n * N_OUT))
    dy = np.zeros((n, N_OUT_PAD))
    dy[:, :N_OUT] = 2.0 * diff / (n * N_OUT)
    dy = q(dy)
    g = {"W3": dy.T @ c["h2"], "b3": dy.sum(0)}
    dz2 = q((dy @ c["w3"]) * (c["h2"] > 0))
    g["W2"], g["b2"] = dz2.T @ c["h1"], dz2.sum(0)
    dz1 = q((dz2 @ c["w2"]) * (c["h1"] > 0))
    g["W1"], g["b1"] = dz1.T @ c["x"], dz1.sum(0)
    return loss, np.concatenate([g[name].ravel() for name, _ in SHAPES])


def adam_step(theta, m, v, grad, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update at step t (1-based); returns new (theta, m, v)."""
    m = b1 * m + (1 - b1) * grad
    v = b2 * v + (1 - b2) * grad * grad
    mh = m / (1 - b1 ** t)
    vh = v / (1 - b2 ** t)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v
