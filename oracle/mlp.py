"""CPU ORACLE (test infrastructure only): the monotone CDF network in float64.

The learned-splitter sort needs a model F(x) of the cumulative distribution of
normalized keys x in [0, 1] that is nondecreasing, so that the bucket it
predicts never reorders keys.  The network is 1 -> 32 -> 32 -> 1 with
nonnegative weights and the ramp activation r(z) = min(max(z, 0), 1):

    h1 = r(W1 * x + b1)            W1: [32],     b1: [32]
    h2 = r(W2 @ h1 + b2)           W2: [32, 32], b2: [32]
    f  = W3 . h2 + b3              W3: [32],     b3: scalar

Nonnegative weights and a nondecreasing activation make f nondecreasing in x.
The ramp (a ReLU capped at 1) is used because a nonnegative-weight ReLU network
is convex in x and cannot follow a concave CDF; sums of ramps can follow any
nondecreasing shape.  Loss: mean squared error against rank/n.  Optimizer:
Adam (Kingma & Ba, 2015) followed by projection of the weights onto >= 0.

Parameters travel as one flat vector of 1153 values in the order
[W1, b1, W2 (row-major, W2[o, i]), b2, W3, b3].  The ramp's derivative is 1 on
the open interval (0, 1) and 0 elsewhere.
"""
from __future__ import annotations

import numpy as np

H = 32
N_PARAMS = H + H + H * H + H + H + 1  # 1153


def unpack(p):
    p = np.asarray(p, dtype=np.float64)
    o = 0
    W1 = p[o:o + H]; o += H
    b1 = p[o:o + H]; o += H
    W2 = p[o:o + H * H].reshape(H, H); o += H * H
    b2 = p[o:o + H]; o += H
    W3 = p[o:o + H]; o += H
    b3 = p[o]
    return W1, b1, W2, b2, W3, b3


def pack(W1, b1, W2, b2, W3, b3):
    return np.concatenate([W1, b1, W2.reshape(-1), b2, W3, [b3]]).astype(np.float64)


def ramp(z):
    return np.minimum(np.maximum(z, 0.0), 1.0)


def ramp_grad(z):
    return ((z > 0.0) & (z < 1.0)).astype(np.float64)


def forward(p, x):
    """f(x) for a batch x of shape [m]; returns f, and the pre-activations."""
    W1, b1, W2, b2, W3, b3 = unpack(p)
    x = np.asarray(x, dtype=np.float64)
    z1 = x[:, None] * W1[None, :] + b1[None, :]          # [m, H]
    h1 = ramp(z1)
    z2 = h1 @ W2.T + b2[None, :]                         # [m, H]
    h2 = ramp(z2)
    f = h2 @ W3 + b3                                     # [m]
    return f, (z1, h1, z2, h2)


def loss_grad(p, x, y):
    """Mean squared error and its exact gradient with respect to p."""
    W1, b1, W2, b2, W3, b3 = unpack(p)
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    m = x.shape[0]
    f, (z1, h1, z2, h2) = forward(p, x)
    r = f - y
    loss = float(np.mean(r * r))
    df = 2.0 * r / m                                     # dL/df, [m]
    gW3 = h2.T @ df
    gb3 = df.sum()
    dh2 = df[:, None] * W3[None, :]
    dz2 = dh2 * ramp_grad(z2)
    gW2 = dz2.T @ h1                                     # [H_out, H_in]
    gb2 = dz2.sum(axis=0)
    dh1 = dz2 @ W2
    dz1 = dh1 * ramp_grad(z1)
    gW1 = (dz1 * x[:, None]).sum(axis=0)
    gb1 = dz1.sum(axis=0)
    return loss, pack(gW1, gb1, gW2, gb2, gW3, gb3)


def weight_mask():
    """1.0 at positions holding weights (projected to >= 0), 0.0 at biases."""
    return pack(np.ones(H), np.zeros(H), np.ones((H, H)), np.zeros(H), np.ones(H), 0.0)


def adam_step(p, g, m, v, t, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (step number t >= 1) then projection of weights to >= 0."""
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    mhat = m / (1.0 - beta1 ** t)
    vhat = v / (1.0 - beta2 ** t)
    p = p - lr * mhat / (np.sqrt(vhat) + eps)
    w = weight_mask() > 0
    p = np.where(w, np.maximum(p, 0.0), p)
    return p, m, v


def to_pwl(p, n_knots=1025):
    """Knots of the network's CDF at the grid x_j = j/(n_knots-1): clamp to
    [0, 1] and take the running maximum so the knots never decrease."""
    x = np.arange(n_knots, dtype=np.float64) / (n_knots - 1)
    f, _ = forward(p, x)
    return np.maximum.accumulate(np.clip(f, 0.0, 1.0))


def init_params(u):
    """Initial parameters from caller-supplied uniforms u in [0,1) of length
    N_PARAMS: hidden ramps of layer 1 spread their breakpoints over [0, 1];
    layer 2 starts as a scaled average; the output starts near identity."""
    u = np.asarray(u, dtype=np.float64)
    W1 = 4.0 + 4.0 * u[0:H]                               # slopes in [4, 8)
    centers = (np.arange(H) + u[H:2 * H]) / H             # breakpoints over [0,1)
    b1 = -W1 * centers
    W2 = (0.5 + u[2 * H:2 * H + H * H].reshape(H, H)) / H
    b2 = -0.25 + 0.5 * u[2 * H + H * H:3 * H + H * H] - 0.0
    W3 = (0.5 + u[3 * H + H * H:4 * H + H * H]) / H
    b3 = 0.0
    return pack(W1, b1, W2, b2, W3, b3)
