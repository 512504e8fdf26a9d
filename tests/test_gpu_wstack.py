"""GPU tests of W-stacking (Section 5: the stream split by w into slices, each
gridded as its own problem) through the C ABI.

Bars: gr_wslice_partition's output (slice offsets, order, and every moved
uvw, visibility and weight value) equals the oracle's partition bit for bit,
at small ragged sizes, with empty, full and non-finite cases, and on the
whole 7,257,600-visibility track set; each slice's grid, gridded by one
gr_grid_batch over the slices or by one gr_grid per slice, within 1e-5
relative L2 of the oracle's FP64 grid of that slice, and empty slices zero.
"""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import gridding as G  # noqa: E402
from synth import wstack_workload  # noqa: E402

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _say(msg):
    print(msg, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def R():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1605_07023_amd import binding, runner
    binding.load_library()
    return runner


def _partition(uvw, vis, wts, w_first, inv_width, n_slices):
    """gr_wslice_partition on host arrays; returns host (uvw, vis, weights, offsets)."""
    from paper_1605_07023_amd import binding as B
    n, P = vis.shape
    d_uvw = torch.from_numpy(np.ascontiguousarray(uvw)).to(DEV) if n else torch.zeros((1, 3), dtype=torch.float64, device=DEV)
    d_vis = torch.from_numpy(np.ascontiguousarray(vis)).to(DEV) if n else torch.zeros((1, P), dtype=torch.complex64, device=DEV)
    d_w = None
    if wts is not None:
        d_w = torch.from_numpy(np.ascontiguousarray(wts)).to(DEV) if n else torch.zeros((1, P), dtype=torch.float32, device=DEV)
    o_uvw = torch.full_like(d_uvw, 7.0)
    o_vis = torch.full_like(d_vis, 7.0)
    o_w = None if d_w is None else torch.full_like(d_w, 7.0)
    offs = torch.full((n_slices + 1,), -1, dtype=torch.int64, device=DEV)
    nw = B.gr_wslice_partition_workspace_bytes(n, n_slices)
    ws = torch.empty(nw, dtype=torch.uint8, device=DEV)
    B.gr_wslice_partition(d_uvw, d_vis, d_w, n, P, w_first, inv_width, n_slices, o_uvw, o_vis, o_w, offs, ws, nw)
    torch.cuda.synchronize()
    return (o_uvw.cpu().numpy()[:n], o_vis.cpu().numpy()[:n], None if o_w is None else o_w.cpu().numpy()[:n],
            offs.cpu().numpy())


def _check_partition(uvw, vis, wts, w_first, inv_width, n_slices):
    got_uvw, got_vis, got_w, got_off = _partition(uvw, vis, wts, w_first, inv_width, n_slices)
    order, offsets = G.wslice_partition(uvw, w_first, inv_width, n_slices)
    np.testing.assert_array_equal(got_off, offsets)
    # bit for bit (NaNs included): compare the raw words
    np.testing.assert_array_equal(got_uvw.view(np.uint64), np.ascontiguousarray(uvw[order]).view(np.uint64))
    np.testing.assert_array_equal(got_vis.view(np.uint32), np.ascontiguousarray(vis[order]).view(np.uint32))
    if wts is not None:
        np.testing.assert_array_equal(got_w.view(np.uint32), np.ascontiguousarray(wts[order]).view(np.uint32))
    return offsets


@pytest.mark.parametrize("P,with_w,n,n_slices", [
    (4, True, 5000, 7), (1, False, 257, 3), (4, False, 1, 1), (1, True, 0, 5), (4, True, 70001, 255),
    (1, True, 4096, 64)])
def test_partition_bit_exact(R, P, with_w, n, n_slices):
    _say(f"w-slice partition P={P} weights={with_w} n={n} slices={n_slices}")
    rng = np.random.default_rng(100 + n + n_slices)
    uvw = rng.uniform(-100.0, 100.0, (n, 3))
    # slowly varying w in runs, as along tracks, plus values outside the slices
    uvw[:, 2] = np.repeat(rng.uniform(-60.0, 60.0, max(n // 16 + 1, 1)), 16)[:n]
    if n > 20:
        uvw[rng.choice(n, 8, replace=False), 2] = np.nan
        uvw[rng.choice(n, 3, replace=False), 2] = np.inf
    vis = (rng.standard_normal((n, P)) + 1j * rng.standard_normal((n, P))).astype(np.complex64)
    wts = rng.uniform(0.5, 2.0, (n, P)).astype(np.float32) if with_w else None
    w_first, inv_width = -50.0, n_slices / 100.0            # [-50, 50): the rest in no slice
    _check_partition(uvw, vis, wts, w_first, inv_width, n_slices)


def test_partition_edges(R):
    """Every visibility outside the slices; w on slice edges; one slice holding all."""
    _say("w-slice partition edges")
    rng = np.random.default_rng(7)
    n = 3000
    vis = (rng.standard_normal((n, 1)) + 1j * rng.standard_normal((n, 1))).astype(np.complex64)
    uvw = np.zeros((n, 3))
    uvw[:, 2] = rng.uniform(100.0, 200.0, n)
    off = _check_partition(uvw, vis, None, -50.0, 0.07, 7)
    assert off.tolist() == [0] * 8
    uvw[:, 2] = rng.integers(-3, 4, n) * 2.0 - 1.0        # exactly on the edges of width-2 slices from -7
    off = _check_partition(uvw, vis, None, -7.0, 0.5, 7)
    assert off[-1] == n - np.count_nonzero(uvw[:, 2] >= 7.0)
    off = _check_partition(uvw, vis, None, -1e9, 1e-10, 1)
    assert off.tolist() == [0, n]


def test_partition_full_track_set(R):
    """The whole 2 h, 2 s-dump set (7,257,600 visibilities, 4 polarisations), 7 slices."""
    _say("w-slice partition, 7,257,600 visibilities, 7 slices")
    wl = wstack_workload(n_pol=4, grid=2048, support=16)
    m = wl.meta
    off = _check_partition(wl.uvw, wl.vis, None, m["w_first"], m["inv_width"], m["n_slices"])
    _say(f"  slice sizes {np.diff(np.append(off, wl.n_vis)).tolist()}")
    assert off[-1] == wl.n_vis                              # every w inside the padded range


@pytest.mark.parametrize("mode,P", [("batch", 4), ("per_slice", 4), ("batch", 1)])
def test_grid_wstack_matches_oracle(R, mode, P):
    from paper_1605_07023_amd import binding as B
    _say(f"W-stacked gridding ({mode}), P={P}, 7 slices, 16 residual planes, S=16, 512^2")
    wl = wstack_workload(n_baselines=30, n_pol=P, grid=512, support=16, planes_per_slice=16)
    rng = np.random.default_rng(21)
    wl.weights = rng.uniform(0.5, 2.0, (wl.n_vis, P)).astype(np.float32)
    taps = (rng.standard_normal((16, 8, 16)) + 1j * rng.standard_normal((16, 8, 16))).astype(np.complex64)
    t = torch.from_numpy(np.ascontiguousarray(taps).view(np.float32).reshape(16, 8, 16, 2)).to(DEV)
    dw = R.upload(wl, DEV, taps=t)
    dw.kernel = B.make_kernel(t, 16, 8, 16, taps_complex=True, w_min=wl.w_min, inv_dw=wl.inv_dw)
    m = wl.meta
    grids, off = R.grid_wstack(dw, m["w_first"], m["inv_width"], m["n_slices"], mode=mode)
    got = grids.cpu().numpy().astype(np.complex128)
    want, dropped, outside = G.grid_wstack(wl.vis, wl.uvw, wl.weights, taps.astype(np.complex128),
                                           wl.inv_cell_u, wl.inv_cell_v, 8, 512, 512, 16, wl.w_min, wl.inv_dw,
                                           m["w_first"], m["inv_width"], m["n_slices"])
    _, offsets = G.wslice_partition(wl.uvw, m["w_first"], m["inv_width"], m["n_slices"])
    assert off.tolist() == offsets.tolist()
    sizes = np.diff(np.append(offsets, wl.n_vis))[:m["n_slices"]]
    _say(f"  slice sizes {sizes.tolist()}, dropped {dropped}, outside {outside}")
    assert (sizes == 0).any() and (sizes > 0).sum() >= 4   # empty slices are part of the case
    for s in range(m["n_slices"]):
        if sizes[s] == 0:
            assert not np.any(got[s]), s
            continue
        e = float(np.linalg.norm(got[s] - want[s]) / np.linalg.norm(want[s]))
        _say(f"  slice {s}: {sizes[s]} visibilities, rel L2 {e:.2e}")
        assert e <= 1e-5, (s, e)
