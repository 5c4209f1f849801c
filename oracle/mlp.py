"""FP64 oracle of the learned active-set gate's network (test infrastructure only).

Network 8-32-32-1: h1 = relu(W1 x + b1), h2 = relu(W2 h1 + b2),
z = W3 h2 + b3, p = sigmoid(z).  Loss: mean binary cross-entropy with a
positive-class weight pw, l = -(pw y log p + (1 - y) log(1 - p)).
Optimiser: Adam (Kingma and Ba, ICLR 2015) with bias correction.

Parameters are one flat vector of 1377 values in the order
W1[32][8], b1[32], W2[32][32], b2[32], W3[1][32], b3[1] (row-major).  The
GPU keeps FP32 master weights and computes with their BF16 rounding
(round to nearest, ties to even); ``bf16_round`` gives the same values so
the oracle evaluates the identical network in FP64.
"""
import numpy as np

SHAPES = [("W1", (32, 8)), ("b1", (32,)), ("W2", (32, 32)), ("b2", (32,)), ("W3", (1, 32)), ("b3", (1,))]
NPARAMS = sum(int(np.prod(s)) for _, s in SHAPES)  # 1377


def unpack(theta):
    theta = np.asarray(theta, dtype=np.float64)
    out, o = {}, 0
    for name, shape in SHAPES:
        k = int(np.prod(shape))
        out[name] = theta[o:o + k].reshape(shape)
        o += k
    return out


def pack(d):
    return np.concatenate([np.asarray(d[name], dtype=np.float64).reshape(-1) for name, _ in SHAPES])


def bf16_round(x32):
    """fp32 -> nearest bf16 (ties to even), returned as float64; NaN kept quiet."""
    a = np.ascontiguousarray(x32, dtype=np.float32)
    u = a.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16) << 16
    nan = np.isnan(a)
    r = np.where(nan, (u | 0x400000) & 0xFFFF0000, r)
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def _sigmoid(z):
    return np.where(z >= 0, 1.0 / (1.0 + np.exp(-np.abs(z))), np.exp(-np.abs(z)) / (1.0 + np.exp(-np.abs(z))))


def forward(theta, x):
    """Returns (p, cache).  x: [B, 8]."""
    P = unpack(theta)
    x = np.asarray(x, dtype=np.float64)
    a1 = x @ P["W1"].T + P["b1"]
    h1 = np.maximum(a1, 0.0)
    a2 = h1 @ P["W2"].T + P["b2"]
    h2 = np.maximum(a2, 0.0)
    z = (h2 @ P["W3"].T)[:, 0] + P["b3"][0]
    p = _sigmoid(z)
    return p, dict(x=x, a1=a1, h1=h1, a2=a2, h2=h2, z=z, P=P)


def loss(theta, x, y, pos_weight=1.0):
    p, c = forward(theta, x)
    y = np.asarray(y, dtype=np.float64)
    z = c["z"]
    # log p = -softplus(-z), log(1 - p) = -softplus(z), evaluated stably
    sp_neg = np.logaddexp(0.0, -z)
    sp_pos = np.logaddexp(0.0, z)
    return float(np.mean(pos_weight * y * sp_neg + (1.0 - y) * sp_pos))


def backward(theta, x, y, pos_weight=1.0):
    """Gradient of the mean weighted BCE with respect to the flat parameters."""
    p, c = forward(theta, x)
    y = np.asarray(y, dtype=np.float64)
    B = x.shape[0]
    dz = (pos_weight * y * (p - 1.0) + (1.0 - y) * p) / B
    P = c["P"]
    g = {}
    g["W3"] = dz[None, :] @ c["h2"]
    g["b3"] = np.array([dz.sum()])
    dh2 = dz[:, None] * P["W3"][0][None, :]
    da2 = dh2 * (c["a2"] > 0)
    g["W2"] = da2.T @ c["h1"]
    g["b2"] = da2.sum(0)
    dh1 = da2 @ P["W2"]
    da1 = dh1 * (c["a1"] > 0)
    g["W1"] = da1.T @ c["x"]
    g["b1"] = da1.sum(0)
    return pack(g)


def adam_step(theta, grad, m, v, t, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update at step t (1-based).  Returns (theta, m, v)."""
    m = beta1 * m + (1.0 - beta1) * grad
    v = beta2 * v + (1.0 - beta2) * grad * grad
    mh = m / (1.0 - beta1 ** t)
    vh = v / (1.0 - beta2 ** t)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v
