"""FP64 NumPy reference of the learned W-kernel network.  Test infrastructure only:
nothing in the product path imports this module.

The network maps a tap's coordinates to its complex value.  It has no
counterpart in the paper: it replaces the precomputed, oversampled GCF table
(Section 2.2) by a function of the same coordinates.  A tap of the 2-D W kernel
depends on its phase s and index k only through the offset
d = k - S/2 + 1 - s/O (the argument at which the GCF is sampled), so the
network takes (w_hat, d_u, d_v):

    x0 = w_hat / w_hat_range,  x1 = d_u / (S/2),  x2 = d_v / (S/2)

(w_hat_range is chosen by the trainer as twice the largest |w_hat|, so that
x0 stays in [-1/2, 1/2]: the encoding below has period 2 in each input, and
on that interval it is one-to-one.  x1 = 1 lies outside the support, where
the tap is zero by rule.)

Encoding (64 features): for input i < 3 and frequency k < 6,
    e[12 i + 2 k] = sin(pi 2^k x_i),  e[12 i + 2 k + 1] = cos(pi 2^k x_i);  e[36:64] = 0.
Layers: h1 = relu(e W1 + b1), h2 = relu(h1 W2 + b2), h3 = relu(h2 W3 + b3),
        y = h3 W4 + b4 (2 outputs).
Tap = out_scale * (y0 + i y1) where |d_u| < S/2 and |d_v| < S/2, else 0 (the
support rule of the tables).
Loss over a batch of n samples: (1/n) sum over samples and (Re, Im) of (y - t)^2,
targets t = tap / out_scale.

Pins (tests/test_oracle_mlp.py): backward against central finite differences,
the encoding at points with known sines, Adam's first step against its closed
form (lr * sign(g)), and the tap layout against the 2-D table's index order.
"""
from __future__ import annotations

import math
from typing import Dict

import numpy as np

N_INPUT = 3
N_FREQ = 6
D_IN = 64
HIDDEN = 64


def init_params(seed: int = 0) -> Dict[str, np.ndarray]:
    """He-uniform weights, zero biases (FP64), from a seeded generator."""
    rng = np.random.default_rng(seed)
    fan_in = {"W1": 2 * N_INPUT * N_FREQ, "W2": HIDDEN, "W3": HIDDEN, "W4": HIDDEN}
    shapes = {"W1": (D_IN, HIDDEN), "W2": (HIDDEN, HIDDEN), "W3": (HIDDEN, HIDDEN), "W4": (HIDDEN, 2)}
    p = {}
    for k, shp in shapes.items():
        lim = math.sqrt(6.0 / fan_in[k]) if k != "W4" else math.sqrt(3.0 / fan_in[k])
        p[k] = rng.uniform(-lim, lim, size=shp)
    p["W1"][2 * N_INPUT * N_FREQ:] = 0.0          # rows of the always-zero features
    for k, n in (("b1", HIDDEN), ("b2", HIDDEN), ("b3", HIDDEN), ("b4", 2)):
        p[k] = np.zeros(n)
    return p


def tap_inputs(w_hat_norm, d_u, d_v, support: int) -> np.ndarray:
    """[n, 3] network inputs (w_hat_norm is w_hat / w_hat_range)."""
    h = support / 2.0
    cols = np.broadcast_arrays(np.asarray(w_hat_norm, float), np.asarray(d_u, float) / h,
                               np.asarray(d_v, float) / h)
    return np.stack([c.ravel() for c in cols], axis=1)


def table_offsets(support: int, oversample: int) -> np.ndarray:
    """[O][S] offsets d = k - S/2 + 1 - s/O (the GCF argument of tap k at phase s)."""
    k = np.arange(support, dtype=np.float64)
    s = np.arange(oversample, dtype=np.float64)
    return k[None, :] - support / 2.0 + 1.0 - s[:, None] / oversample


def table_inputs(w_hat_norm_planes, support: int, oversample: int) -> np.ndarray:
    """Inputs of every entry of a [planes][O][O][S][S] table indexed
    [plane][s_v][s_u][k_v][k_u], in that (row-major) order: [planes*O*O*S*S, 3]."""
    wn = np.asarray(w_hat_norm_planes, float).reshape(-1)
    d = table_offsets(support, oversample)
    P, O, S = wn.size, oversample, support
    w_ = np.broadcast_to(wn[:, None, None, None, None], (P, O, O, S, S))
    du = np.broadcast_to(d[None, None, :, None, :], (P, O, O, S, S))
    dv = np.broadcast_to(d[None, :, None, :, None], (P, O, O, S, S))
    return tap_inputs(w_, du, dv, support)


def encode(x: np.ndarray) -> np.ndarray:
    """[n, 3] -> [n, 64] sinusoidal features."""
    n = x.shape[0]
    e = np.zeros((n, D_IN))
    for i in range(N_INPUT):
        for k in range(N_FREQ):
            a = math.pi * (2.0 ** k) * x[:, i]
            e[:, 12 * i + 2 * k] = np.sin(a)
            e[:, 12 * i + 2 * k + 1] = np.cos(a)
    return e


def forward(params: Dict[str, np.ndarray], e: np.ndarray):
    """Returns (y [n, 2], cache) in FP64."""
    z1 = e @ params["W1"] + params["b1"]
    h1 = np.maximum(z1, 0.0)
    z2 = h1 @ params["W2"] + params["b2"]
    h2 = np.maximum(z2, 0.0)
    z3 = h2 @ params["W3"] + params["b3"]
    h3 = np.maximum(z3, 0.0)
    y = h3 @ params["W4"] + params["b4"]
    return y, (e, z1, h1, z2, h2, z3, h3)


def taps(params: Dict[str, np.ndarray], out_scale: float, x: np.ndarray, support: int) -> np.ndarray:
    """Complex taps at inputs x [n, 3], zero where |d_u| or |d_v| >= S/2."""
    y, _ = forward(params, encode(x))
    inside = (np.abs(x[:, 1]) < 1.0) & (np.abs(x[:, 2]) < 1.0)
    return np.where(inside, out_scale * (y[:, 0] + 1j * y[:, 1]), 0.0)


def tap_table(params: Dict[str, np.ndarray], out_scale: float, w_hat_norm_planes, support: int,
              oversample: int) -> np.ndarray:
    """The network's taps laid out as a complex [planes][O][O][S][S] table."""
    x = table_inputs(w_hat_norm_planes, support, oversample)
    P = np.asarray(w_hat_norm_planes).size
    return taps(params, out_scale, x, support).reshape(P, oversample, oversample, support, support)


def loss(y: np.ndarray, t: np.ndarray) -> float:
    return float(np.sum((y - t) ** 2) / y.shape[0])


def backward(params: Dict[str, np.ndarray], cache, y: np.ndarray, t: np.ndarray) -> Dict[str, np.ndarray]:
    """Gradients of loss(y, t) with respect to every parameter (chain rule)."""
    e, z1, h1, z2, h2, z3, h3 = cache
    n = y.shape[0]
    dy = 2.0 * (y - t) / n
    g = {"W4": h3.T @ dy, "b4": dy.sum(axis=0)}
    d3 = (dy @ params["W4"].T) * (z3 > 0)
    g["W3"], g["b3"] = h2.T @ d3, d3.sum(axis=0)
    d2 = (d3 @ params["W3"].T) * (z2 > 0)
    g["W2"], g["b2"] = h1.T @ d2, d2.sum(axis=0)
    d1 = (d2 @ params["W2"].T) * (z1 > 0)
    g["W1"], g["b1"] = e.T @ d1, d1.sum(axis=0)
    return g


def adam_step(params, grads, m, v, step: int, lr: float, beta1: float = 0.9, beta2: float = 0.999,
              eps: float = 1e-8):
    """One Adam update (Kingma & Ba 2015), in place; step counts from 1."""
    for k in params:
        m[k] = beta1 * m[k] + (1 - beta1) * grads[k]
        v[k] = beta2 * v[k] + (1 - beta2) * grads[k] ** 2
        mh = m[k] / (1 - beta1 ** step)
        vh = v[k] / (1 - beta2 ** step)
        params[k] = params[k] - lr * mh / (np.sqrt(vh) + eps)


def grid_network(vis: np.ndarray, uvw: np.ndarray, weights, params: Dict[str, np.ndarray],
                 out_scale: float, x0_planes, inv_cell_u: float, inv_cell_v: float, oversample: int,
                 support: int, height: int, width: int, n_planes: int, w_min: float, inv_dw: float,
                 chunk: int = 256):
    """FP64 grid with the network's taps evaluated per visibility (no table):
    the visibility at plane p and phases (s_u, s_v) adds tap(x0_planes[p],
    d_u[k_u], d_v[k_v]) V to footprint cell (y0 + k_v, x0 + k_u), with
    d = k - S/2 + 1 - s/O.  Index conversion and drops as the table gridders
    (oracle.gridding.pixel_coords)."""
    from . import gridding as G
    n_pol = vis.shape[1]
    pc = G.pixel_coords(uvw, inv_cell_u, inv_cell_v, oversample, support, height, width,
                        n_planes, w_min, inv_dw)
    valid = pc["valid"] & G.finite_values(vis, weights)
    wv = G.weighted_vis(vis, weights)
    x0_planes = np.asarray(x0_planes, np.float64)
    out = np.zeros((n_pol, height, width), np.complex128)
    flat = out.reshape(n_pol, -1)
    idx = np.nonzero(valid)[0]
    k = np.arange(support, dtype=np.float64)
    S = support
    for c0 in range(0, idx.size, chunk):
        sel = idx[c0:c0 + chunk]
        du = k[None, :] - S / 2.0 + 1.0 - pc["sx"][sel][:, None] / oversample        # [n, S]
        dv = k[None, :] - S / 2.0 + 1.0 - pc["sy"][sel][:, None] / oversample
        wn = x0_planes[pc["plane"][sel]]
        x = tap_inputs(wn[:, None, None], du[:, None, :], dv[:, :, None], S)          # [n*S*S, 3]
        kern = taps(params, out_scale, x, S).reshape(sel.size, S, S)                   # [n, kv, ku]
        rows = pc["y0"][sel][:, None] + np.arange(S)[None, :]
        cols = pc["x0"][sel][:, None] + np.arange(S)[None, :]
        cell = (rows[:, :, None] * width + cols[:, None, :]).ravel()
        for p in range(n_pol):
            contrib = (kern * wv[sel, p][:, None, None]).ravel()
            flat[p] += np.bincount(cell, weights=contrib.real, minlength=height * width) \
                + 1j * np.bincount(cell, weights=contrib.imag, minlength=height * width)
    return out, int(np.count_nonzero(~valid))
