"""FP64 CPU oracle of the surrogate ensemble (TEST INFRASTRUCTURE ONLY: only
the test suite, the smoke check and the benchmark's CPU leg may use it; it
shares no code with the HIP library).

One member is an MLP 4 -> H -> H -> 2 with tanh hidden activations and a
linear output.  Its parameters form one vector in the order
W1 [H][4], b1 [H], W2 [H][H] (row i feeds hidden unit i), b2 [H],
W3 [2][H], b3 [2].  The loss of n samples is the mean squared error over
samples and outputs, L = sum (y - Y)^2 / (2 n).  Training is Adam
(Kingma & Ba 2015) with bias-corrected moments, beta1 = 0.9,
beta2 = 0.999, eps = 1e-8.  Inference in BF16 rounds W2 and the layer-1
activations to BF16 (round to nearest even) before the layer-2 product and
accumulates exactly; everything else stays in full precision.
"""
from __future__ import annotations

import numpy as np

NIN, NOUT = 4, 2


def sizes(H: int):
    return [("W1", (H, NIN)), ("b1", (H,)), ("W2", (H, H)), ("b2", (H,)), ("W3", (NOUT, H)), ("b3", (NOUT,))]


def n_params(H: int) -> int:
    return sum(int(np.prod(s)) for _, s in sizes(H))


def unpack(theta, H: int):
    out, o = {}, 0
    for name, s in sizes(H):
        k = int(np.prod(s))
        out[name] = np.asarray(theta[o:o + k], dtype=np.float64).reshape(s)
        o += k
    return out


def pack(p, H: int):
    return np.concatenate([p[name].reshape(-1) for name, _ in sizes(H)])


def forward(theta, X, H: int):
    """Return (y, cache) for inputs X [n][4]."""
    p = unpack(theta, H)
    X = np.asarray(X, dtype=np.float64)
    h1 = np.tanh(X @ p["W1"].T + p["b1"])
    h2 = np.tanh(h1 @ p["W2"].T + p["b2"])
    y = h2 @ p["W3"].T + p["b3"]
    return y, (X, h1, h2, p)


def loss(theta, X, Y, H: int) -> float:
    y, _ = forward(theta, X, H)
    return float(((y - np.asarray(Y, np.float64)) ** 2).sum() / (NOUT * len(X)))


def grad(theta, X, Y, H: int):
    """Gradient of loss() by the chain rule, layer by layer."""
    y, (X, h1, h2, p) = forward(theta, X, H)
    n = len(X)
    dy = 2.0 * (y - np.asarray(Y, np.float64)) / (NOUT * n)
    g = {"W3": dy.T @ h2, "b3": dy.sum(0)}
    dz2 = (dy @ p["W3"]) * (1.0 - h2 ** 2)
    g["W2"] = dz2.T @ h1
    g["b2"] = dz2.sum(0)
    dz1 = (dz2 @ p["W2"]) * (1.0 - h1 ** 2)
    g["W1"] = dz1.T @ X
    g["b1"] = dz1.sum(0)
    return pack(g, H)


def adam(theta, m, v, g, t: int, lr: float, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update at step t (1-based); returns (theta, m, v)."""
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mhat = m / (1 - b1 ** t)
    vhat = v / (1 - b2 ** t)
    return theta - lr * mhat / (np.sqrt(vhat) + eps), m, v


def bf16(a):
    """Round to the nearest BF16 value (ties to even), as float64."""
    a = np.asarray(a, dtype=np.float32)
    u = a.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def forward_bf16(theta, X, H: int):
    """Inference with W2 and the layer-1 activations in BF16."""
    p = unpack(theta, H)
    X = np.asarray(X, dtype=np.float64)
    h1 = bf16(np.tanh(X @ p["W1"].T + p["b1"]))
    h2 = np.tanh(h1 @ bf16(p["W2"]).T + p["b2"])
    return h2 @ p["W3"].T + p["b3"]


def ensemble(thetas, X, H: int, threshold: float, bf16_inference=True, out_scale=None, out_shift=None):
    """Mean, (population) standard deviation over members, fallback flags.

    Each member's outputs are first mapped to the caller's units,
    y * out_scale + out_shift per output (identity by default: a network
    trained on normalised targets gives physical values this way), and the
    statistics and the fallback test (std > threshold * |mean| for some
    output) are taken in those units."""
    f = forward_bf16 if bf16_inference else (lambda t, x, h: forward(t, x, h)[0])
    ys = np.stack([f(t, X, H) for t in thetas])
    if out_scale is not None:
        ys = ys * np.asarray(out_scale, np.float64)
    if out_shift is not None:
        ys = ys + np.asarray(out_shift, np.float64)
    mu = ys.mean(0)
    sd = ys.std(0)
    fb = (sd > threshold * np.abs(mu)).any(axis=1)
    return mu, sd, fb
