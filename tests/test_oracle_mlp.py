"""Pins for the FP64 network reference (oracle/mlp.py)."""
import math

import numpy as np

from oracle import gridding as G
from oracle import mlp as M


def _params(rng, scale=0.3):
    p = {}
    for i, (a, b) in enumerate([(64, 64), (64, 64), (64, 64), (64, 2)], 1):
        p[f"W{i}"] = rng.uniform(-scale, scale, (a, b))
        p[f"b{i}"] = rng.uniform(-0.1, 0.1, b)
    return p


def test_encoding_identities():
    """Each (sin, cos) pair lies on the unit circle and consecutive frequencies
    obey the double-angle formula, so the k-th feature is at 2^k pi x."""
    x = np.random.default_rng(0).uniform(-1, 1, (50, 3))
    e = M.encode(x)
    assert e.shape == (50, 64) and np.all(e[:, 36:] == 0)
    for i in range(3):
        for k in range(6):
            s, c = e[:, 12 * i + 2 * k], e[:, 12 * i + 2 * k + 1]
            np.testing.assert_allclose(s * s + c * c, 1.0, atol=1e-14)
            if k == 0:
                np.testing.assert_allclose(s, np.sin(math.pi * x[:, i]), atol=1e-14)
            else:
                ps, pc = e[:, 12 * i + 2 * k - 2], e[:, 12 * i + 2 * k - 1]
                np.testing.assert_allclose(s, 2 * ps * pc, atol=1e-12)
    e = M.encode(np.array([[0.5, -0.5, 0.25]]))
    assert abs(e[0, 0] - 1) < 1e-15 and abs(e[0, 12] + 1) < 1e-15          # sin(pi/2), sin(-pi/2)
    assert abs(e[0, 24 + 2] - 1) < 1e-15                                     # sin(2 pi / 4)


def test_forward_of_constructed_network():
    """Weights that route one feature through the three ReLU layers: y0 is that
    feature plus a known constant, y1 the negated cosine feature."""
    p = {k: np.zeros(s) for k, s in (("W1", (64, 64)), ("W2", (64, 64)), ("W3", (64, 64)),
                                     ("W4", (64, 2)))}
    for k in ("b1", "b2", "b3"):
        p[k] = np.zeros(64)
    p["b4"] = np.array([-3.0, 0.0])
    p["W1"][12, 0] = 1.0          # sin(pi x1) -> unit 0
    p["W1"][13, 1] = 1.0          # cos(pi x1) -> unit 1
    p["b1"][0] = p["b1"][1] = 1.5 # keeps both units above zero
    p["W2"][0, 0] = p["W3"][0, 0] = 1.0
    p["W2"][1, 1] = p["W3"][1, 1] = 1.0
    p["W4"][0, 0] = 2.0
    p["W4"][1, 1] = -1.0
    x = np.random.default_rng(3).uniform(-1, 1, (20, 3))
    y, _ = M.forward(p, M.encode(x))
    np.testing.assert_allclose(y[:, 0], 2 * (np.sin(math.pi * x[:, 1]) + 1.5) - 3.0, atol=1e-14)
    np.testing.assert_allclose(y[:, 1], -(np.cos(math.pi * x[:, 1]) + 1.5), atol=1e-14)
    # a negative pre-activation is cut by the ReLU
    p["b1"][0] = -5.0
    y, _ = M.forward(p, M.encode(x))
    np.testing.assert_allclose(y[:, 0], -3.0, atol=0)


def test_backward_matches_central_differences():
    rng = np.random.default_rng(1)
    p = _params(rng)
    x = rng.uniform(-1, 1, (40, 3))
    e = M.encode(x)
    t = rng.standard_normal((40, 2))
    y, cache = M.forward(p, e)
    g = M.backward(p, cache, y, t)
    h = 1e-6
    for name in p:
        flat = p[name].ravel()
        idx = rng.choice(flat.size, size=min(12, flat.size), replace=False)
        if name == "W1":
            idx = np.concatenate([idx, [5 * 64 + 7, 30 * 64 + 1]])   # rows of live features
        for j in idx:
            old = flat[j]
            flat[j] = old + h
            lp = M.loss(M.forward(p, e)[0], t)
            flat[j] = old - h
            lm = M.loss(M.forward(p, e)[0], t)
            flat[j] = old
            num = (lp - lm) / (2 * h)
            ana = g[name].ravel()[j]
            assert abs(num - ana) <= 1e-6 * max(1.0, abs(num)), (name, j, num, ana)


def test_adam_first_step_is_signed_learning_rate():
    """With bias correction, Adam's first update is -lr * g / (|g| + eps)."""
    p = {"a": np.array([1.0, -2.0, 0.5])}
    g = {"a": np.array([0.3, -4.0, 1e-3])}
    m = {"a": np.zeros(3)}
    v = {"a": np.zeros(3)}
    M.adam_step(p, g, m, v, 1, lr=0.01)
    np.testing.assert_allclose(p["a"], np.array([1.0, -2.0, 0.5]) - 0.01 * g["a"] / (np.abs(g["a"]) + 1e-8),
                               rtol=1e-12)


def test_table_inputs_follow_the_table_layout():
    """Row (p, s_v, s_u, k_v, k_u) of table_inputs carries the offsets of the
    2-D table entry at that index: d = k - S/2 + 1 - s/O on each axis."""
    S, O = 8, 4
    wn = np.array([-0.5, 0.25])
    x = M.table_inputs(wn, S, O).reshape(2, O, O, S, S, 3)
    d = G.tap_offsets(S, O)
    for (p, sv, su, kv, ku) in [(0, 0, 0, 0, 0), (1, 3, 1, 7, 2), (0, 2, 3, 5, 6), (1, 0, 2, 0, 7)]:
        np.testing.assert_array_equal(x[p, sv, su, kv, ku], [wn[p], d[su, ku] / (S / 2), d[sv, kv] / (S / 2)])
    assert x[..., 1].max() == 1.0 and x[..., 1].min() > -1.0


def test_taps_zero_outside_support():
    rng = np.random.default_rng(2)
    p = _params(rng)
    t = M.tap_table(p, 2.0, [0.1], 8, 2)
    # k = S-1 at phase 0 sits at d = S/2: outside the support
    assert np.all(t[0, :, 0, :, 7] == 0) and np.all(t[0, 0, :, 7, :] == 0)
    assert np.all(t[0, 1, 1] != 0)


def test_grid_network_equals_table_route():
    """Per-visibility network taps and the network's tap table fed to the
    2-D table gridder give the same grid."""
    from synth import random_point_workload
    rng = np.random.default_rng(5)
    p = _params(rng)
    wl = random_point_workload(300, 4, 48, 40, 8, 4, seed=3, n_planes=3, margin=3, weights=True,
                               kernel="w2d")
    x0 = np.array([-0.4, 0.05, 0.3])
    table = M.tap_table(p, 1.3, x0, 8, 4)
    ref, d1 = G.grid_table2d(wl.vis, wl.uvw, wl.weights, table, 1.0, 1.0, 4, 48, 40, 3, wl.w_min,
                             wl.inv_dw)
    got, d2 = M.grid_network(wl.vis, wl.uvw, wl.weights, p, 1.3, x0, 1.0, 1.0, 4, 8, 48, 40, 3,
                             wl.w_min, wl.inv_dw, chunk=37)
    assert d1 == d2 and d1 > 0
    np.testing.assert_allclose(got, ref, atol=1e-12 * np.abs(ref).max(), rtol=0)
