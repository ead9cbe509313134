"""Plain FP64 reference of the learned inverse CDF's network (test infrastructure only: loaded
by the tests, never by the product path).

The network maps normalized inputs x = (u, v, c) to y through four hidden layers of 64 SiLU
units and a linear output:
    z1 = x W1 + b1, h_l = silu(z_l), z_{l+1} = h_l W_{l+1} + b_{l+1} (l = 1..3), y = h4 W5 + b5,
silu(z) = z / (1 + exp(-z)).  Parameters are one flat vector in the order W1 (3x64, row = input),
b1, W2 (64x64, row = input unit), b2, W3, b3, W4, b4, W5 (64), b5 (1): 12801 numbers.
The loss of a batch is sum_i (y_i - t_i)^2; its gradient is the textbook back-propagation.
"""
from __future__ import annotations

import numpy as np

H = 64
SHAPES = [("W1", (3, H)), ("b1", (H,)), ("W2", (H, H)), ("b2", (H,)), ("W3", (H, H)), ("b3", (H,)),
          ("W4", (H, H)), ("b4", (H,)), ("W5", (H,)), ("b5", (1,))]
N_PARAMS = sum(int(np.prod(s)) for _, s in SHAPES)


def unpack(theta):
    out, o = {}, 0
    for name, shp in SHAPES:
        n = int(np.prod(shp))
        out[name] = np.asarray(theta[o:o + n], dtype=np.float64).reshape(shp)
        o += n
    return out


def pack(d):
    return np.concatenate([np.asarray(d[name], dtype=np.float64).ravel() for name, _ in SHAPES])


def silu(z):
    return z / (1.0 + np.exp(-z))


def dsilu(z):
    s = 1.0 / (1.0 + np.exp(-z))
    return s * (1.0 + z * (1.0 - s))


def forward(theta, x):
    """y for inputs x (n, 3); also the pre-activations of the four hidden layers."""
    p = unpack(theta)
    zs = []
    z = x @ p["W1"] + p["b1"]
    zs.append(z)
    for l in (2, 3, 4):
        z = silu(z) @ p[f"W{l}"] + p[f"b{l}"]
        zs.append(z)
    y = silu(z) @ p["W5"] + p["b5"][0]
    return y, zs


def loss_and_grad(theta, x, t):
    """sum_i (y_i - t_i)^2 and its gradient with respect to theta (flat, same order)."""
    p = unpack(theta)
    y, zs = forward(theta, x)
    e = y - t
    dy = 2.0 * e
    g = {}
    h4 = silu(zs[3])
    g["W5"] = h4.T @ dy
    g["b5"] = np.array([dy.sum()])
    dz = np.outer(dy, p["W5"]) * dsilu(zs[3])
    for l in (4, 3, 2):
        h = silu(zs[l - 2])
        g[f"W{l}"] = h.T @ dz
        g[f"b{l}"] = dz.sum(axis=0)
        dz = (dz @ p[f"W{l}"].T) * dsilu(zs[l - 2])
    g["W1"] = x.T @ dz
    g["b1"] = dz.sum(axis=0)
    return float(e @ e), pack(g)
