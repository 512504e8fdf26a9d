"""Pins of the oracle's W-stacking split (Section 5: the data is split into
slices by w, each gridded as its own problem with a GCF for the offset from
the slice's centre).  Hand-computed slice indices, brute-force partitions, a
delta table that shows which plane each slice picks, and the w-independent
case where the slices' grids must add up to the grid of the whole stream."""
import math

import numpy as np
import pytest

from oracle import gridding as G


def _uvw_w(ws):
    out = np.zeros((len(ws), 3))
    out[:, 2] = ws
    return out


def test_wslice_index_hand_values():
    # slices of width 2 from -3: [-3, -1), [-1, 1), [1, 3)
    ws = [-3.0, -1.0000001, -1.0, 0.0, 0.999999, 1.0, 2.9999, 3.0, -3.0000001, np.nan, np.inf, -np.inf, 1e300]
    want = [0, 0, 1, 1, 1, 2, 2, 3, 3, 3, 3, 3, 3]
    got = G.wslice_index(_uvw_w(ws), -3.0, 0.5, 3)
    assert got.tolist() == want


def test_wslice_partition_brute_force():
    rng = np.random.default_rng(3)
    n, n_slices, w_first, inv_width = 3000, 5, -7.0, 0.4
    ws = rng.uniform(-9.0, 9.0, n)
    ws[rng.choice(n, 20, replace=False)] = np.nan
    order, offsets = G.wslice_partition(_uvw_w(ws), w_first, inv_width, n_slices)
    # brute force: walk the stream once per slice, in input order
    want = []
    starts = []
    for s in range(n_slices + 1):
        starts.append(len(want))
        for i, w in enumerate(ws):
            t = (w - w_first) * inv_width
            inside = (not math.isnan(t)) and 0.0 <= t < n_slices
            if (math.floor(t) if inside else n_slices) == s:
                want.append(i)
    assert order.tolist() == want
    assert offsets.tolist() == starts
    assert sorted(order.tolist()) == list(range(n))


def _delta_table(n_planes, support):
    """Real taps: plane j has the single value (j + 1) at the centre tap S/2 - 1."""
    t = np.zeros((n_planes, 1, support))
    for j in range(n_planes):
        t[j, 0, support // 2 - 1] = j + 1.0
    return t


def test_grid_wstack_picks_the_plane_relative_to_the_slice_centre():
    S, H, W, n_planes = 8, 32, 32, 5
    w_first, inv_width, n_slices = 100.0, 0.1, 4           # slices of width 10 from w = 100
    w_min_rel, inv_dw = -5.0, 0.4                          # planes at -5, -2.5, 0, 2.5, 5 about the centre
    cases = [(0, 2), (1, 0), (3, 4), (2, 3)]               # (slice, plane): one visibility each
    ws = [w_first + 10.0 * s + 5.0 + (w_min_rel + j / inv_dw) * 0.999 for s, j in cases]
    uvw = _uvw_w(ws)                                       # u = v = 0: the centre tap lands on (H/2, W/2)
    vis = (np.arange(1, len(cases) + 1) * (1 + 2j)).reshape(-1, 1).astype(np.complex64)
    grids, dropped, outside = G.grid_wstack(vis, uvw, None, _delta_table(n_planes, S), 1.0, 1.0, 1, H, W,
                                            n_planes, w_min_rel, inv_dw, w_first, inv_width, n_slices)
    assert dropped == 0 and outside == 0
    want = np.zeros_like(grids)
    for n, (s, j) in enumerate(cases):
        want[s, 0, H // 2, W // 2] += (j + 1) ** 2 * complex(vis[n, 0])
    np.testing.assert_array_equal(grids, want)


def test_grid_wstack_sums_to_the_whole_for_a_w_independent_kernel():
    rng = np.random.default_rng(11)
    n, S, O, H, W = 600, 8, 8, 64, 64
    uvw = np.stack([rng.uniform(-20, 20, n), rng.uniform(-20, 20, n), rng.uniform(-50, 50, n)], axis=1)
    vis = (rng.standard_normal((n, 4)) + 1j * rng.standard_normal((n, 4))).astype(np.complex64)
    wts = rng.uniform(0.5, 2.0, (n, 4)).astype(np.float32)
    taps = G.kb_table(S, O, 8.6)
    w_first, inv_width, n_slices = -40.0, 0.1, 7           # [-40, 30): some visibilities in no slice
    grids, dropped, outside = G.grid_wstack(vis, uvw, wts, taps, 1.0, 1.0, O, H, W, 1, 0.0, 0.0,
                                            w_first, inv_width, n_slices)
    inside = (uvw[:, 2] >= -40.0) & (uvw[:, 2] < 30.0)
    whole, d_whole = G.grid_separable(vis[inside], uvw[inside], wts[inside], taps, 1.0, 1.0, O, H, W)
    assert outside == int(np.count_nonzero(~inside)) and outside > 0
    assert dropped == d_whole
    np.testing.assert_allclose(grids.sum(axis=0), whole, rtol=0, atol=1e-12)


def test_slice_w_min_agrees_with_the_library():
    """The w_min of each slice's kernel descriptor, formed by the library's
    gr_wslice_kernel (a host-only C entry point), equals the oracle's bit for
    bit, so both sides pick the same planes; the rest of the descriptor is
    copied unchanged."""
    from paper_1605_07023_amd import binding as B
    rng = np.random.default_rng(17)
    for _ in range(2000):
        w_first = float(rng.uniform(-5e3, 5e3))
        inv_width = float(10.0 ** rng.uniform(-4, 1))
        w_min_rel = float(rng.uniform(-1e3, 0.0))
        s = int(rng.integers(0, 255))
        table = B.GrKernel(B.GR_SEPARABLE, B.GR_F32, 1, 16, 8, 32, w_min_rel, 0.25, 1 << 20)
        k = B.gr_wslice_kernel(table, w_first, inv_width, s)
        assert k.w_min == G.wslice_w_min(w_first, inv_width, s, w_min_rel)
        assert (k.kind, k.tap_dtype, k.taps_complex, k.support, k.oversample, k.n_planes, k.inv_dw, k.taps) == \
            (table.kind, table.tap_dtype, table.taps_complex, table.support, table.oversample, table.n_planes,
             table.inv_dw, table.taps)


def test_slice_kernel_rejects_bad_arguments():
    from paper_1605_07023_amd import binding as B
    table = B.GrKernel(B.GR_SEPARABLE, B.GR_F32, 1, 16, 8, 32, -10.0, 0.25, 1 << 20)
    for args in [(0.0, 0.0, 0), (0.0, -1.0, 0), (float("nan"), 1.0, 0), (0.0, 1.0, -1), (0.0, 1.0, 255)]:
        with pytest.raises(B.GridderError):
            B.gr_wslice_kernel(table, *args)
