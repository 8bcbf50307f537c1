"""FP64 reference of the variant picker's cost model (test infrastructure).

A multilayer perceptron 13 -> 64 -> 64 -> 1 with ReLU hidden units predicts
the log run time of one (problem, record) pair from its 13 features; it is
trained by mean squared error with Adam, and the pick is the candidate with
the smallest prediction (ties: lowest index).  The paper leaves every choice
of transformation to the user (its sec. 1: instructions, loop bounds and
transformations fix the code); this model is how the build chooses records
for shapes it has not timed.

Parameters are one flat vector in this order (the layout the GPU kernels
use): W1[64][13], b1[64], W2[64][64], b2[64], w3[64], b3.

Only tests and the benchmark's CPU leg import this module.
"""
import numpy as np

NF, NH = 13, 64
SIZES = (("W1", NH * NF), ("b1", NH), ("W2", NH * NH), ("b2", NH), ("w3", NH), ("b3", 1))
NPARAMS = sum(n for _, n in SIZES)  # 5121


def unpack(p):
    """Views of the flat parameter vector as (W1, b1, W2, b2, w3, b3)."""
    p = np.asarray(p, dtype=np.float64)
    out, o = [], 0
    for name, n in SIZES:
        v = p[o:o + n]
        if name == "W1":
            v = v.reshape(NH, NF)
        elif name == "W2":
            v = v.reshape(NH, NH)
        out.append(v)
        o += n
    return out


def forward(p, X):
    """Returns (y, cache): y[b] = w3 . relu(W2 relu(W1 x_b + b1) + b2) + b3."""
    W1, b1, W2, b2, w3, b3 = unpack(p)
    X = np.asarray(X, dtype=np.float64)
    z1 = X @ W1.T + b1
    h1 = np.maximum(z1, 0.0)
    z2 = h1 @ W2.T + b2
    h2 = np.maximum(z2, 0.0)
    y = h2 @ w3 + b3[0]
    return y, (X, z1, h1, z2, h2)


def mse(y, t):
    """L = mean((y - t)^2) and dL/dy = 2 (y - t) / n."""
    y = np.asarray(y, dtype=np.float64)
    t = np.asarray(t, dtype=np.float64)
    d = y - t
    return float(np.mean(d * d)), 2.0 * d / len(d)


def backward(p, cache, dy):
    """Gradient of sum_b dy[b] * y[b] with respect to the flat parameters,
    by the chain rule through the two ReLU layers (ReLU'(0) = 0)."""
    W1, b1, W2, b2, w3, b3 = unpack(p)
    X, z1, h1, z2, h2 = cache
    dy = np.asarray(dy, dtype=np.float64)
    g_w3 = h2.T @ dy
    g_b3 = np.array([dy.sum()])
    dz2 = np.outer(dy, w3) * (z2 > 0)
    g_W2 = dz2.T @ h1
    g_b2 = dz2.sum(axis=0)
    dz1 = (dz2 @ W2) * (z1 > 0)
    g_W1 = dz1.T @ X
    g_b1 = dz1.sum(axis=0)
    return np.concatenate([g_W1.ravel(), g_b1, g_W2.ravel(), g_b2, g_w3, g_b3])


def adam(p, g, m, v, step, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (bias-corrected moments); returns new (p, m, v).
    `step` counts from 1."""
    m = beta1 * m + (1 - beta1) * g
    v = beta2 * v + (1 - beta2) * g * g
    mh = m / (1 - beta1 ** step)
    vh = v / (1 - beta2 ** step)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v


def pick(p, feats, mean, std):
    """Index of the candidate with the smallest predicted log time after
    standardising the features (std = 0 counts as 1); ties: lowest index."""
    std = np.where(np.asarray(std) == 0, 1.0, std)
    y, _ = forward(p, (np.asarray(feats, np.float64) - mean) / std)
    return int(np.argmin(y))
