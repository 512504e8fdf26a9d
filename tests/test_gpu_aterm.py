"""GPU tests of gr_grid_aterm (Section 6: non-separable GCFs that change per
visibility and per polarisation, as A-projection's do) through the C ABI.

Bars: against the FP64 oracle's grid within 1e-5 relative L2 (FP32, FP16 and
BF16 taps, the oracle fed the same rounded taps), P = 1 and 4, S = 8 to 32, with
weights, a non-finite coordinate and ids out of range, the statistics
{kept, dropped} equal to the oracle's; integer taps and visibilities bit for
bit; an empty stream and a stream of only bad ids leave the grid untouched.
"""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import gridding as G  # noqa: E402
from synth import aterm_taps, aterm_workload  # noqa: E402

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


def _run(R, wl, ids, n_ids, taps_dev, tap_dtype):
    from paper_1605_07023_amd import binding as B
    dw = R.upload(wl, DEV, taps=taps_dev)
    dw.kernel = B.make_kernel(taps_dev, wl.support, wl.oversample, wl.n_planes, taps_complex=True,
                              tap_dtype=tap_dtype, w_min=wl.w_min, inv_dw=wl.inv_dw, kind=B.GR_TABLE2D)
    d_ids = torch.from_numpy(np.ascontiguousarray(ids)).to(DEV) if wl.n_vis else torch.zeros(1, dtype=torch.int32,
                                                                                            device=DEV)
    stats = torch.zeros(2, dtype=torch.int64, device=DEV)
    g = R.grid_aterm(dw, d_ids, n_ids, stats=stats)
    torch.cuda.synchronize()
    return g.cpu().numpy().astype(np.complex128), stats.cpu().numpy()


@pytest.mark.parametrize("P,S,tdt", [(4, 16, "f32"), (1, 32, "f32"), (4, 8, "f32"), (4, 16, "f16"), (1, 40, "f32"),
                                     (4, 16, "bf16")])
def test_aterm_matches_oracle(R, P, S, tdt):
    from paper_1605_07023_amd import binding as B
    _say(f"A-term gridding P={P} S={S} taps {tdt}")
    wl = aterm_workload(S, n_baselines=3, grid=512, n_pol=P)
    rng = np.random.default_rng(S + P)
    wl.weights = rng.uniform(0.5, 2.0, (wl.n_vis, P)).astype(np.float32)
    wl.uvw = wl.uvw.copy()
    wl.uvw[17, 1] = np.nan                                   # dropped by the coordinate rule
    ids = wl.meta["kernel_id"].copy()
    n_ids = wl.meta["n_ids"]
    ids[rng.choice(wl.n_vis, 40, replace=False)] = n_ids     # dropped by the id rule
    ids[rng.choice(wl.n_vis, 40, replace=False)] = -3
    taps = aterm_taps(5, n_ids, wl.n_planes, wl.oversample, P, S)
    if tdt == "f16":
        t16 = np.ascontiguousarray(taps).view(np.float32).astype(np.float16)
        taps_ref = t16.astype(np.float32).view(np.complex64).reshape(taps.shape)
        taps_dev = torch.from_numpy(t16).to(DEV)
        code = B.GR_F16
    elif tdt == "bf16":
        tb = torch.from_numpy(np.ascontiguousarray(taps).view(np.float32)).to(torch.bfloat16)   # RNE on the host
        taps_ref = np.ascontiguousarray(tb.to(torch.float32).numpy()).view(np.complex64).reshape(taps.shape)
        taps_dev = tb.to(DEV)
        code = B.GR_BF16
    else:
        taps_ref = taps
        taps_dev = torch.from_numpy(np.ascontiguousarray(taps).view(np.float32)).to(DEV)
        code = B.GR_F32
    got, stats = _run(R, wl, ids, n_ids, taps_dev, code)
    want, dropped = G.grid_aterm(wl.vis, wl.uvw, wl.weights, ids, taps_ref.astype(np.complex128), wl.inv_cell_u,
                                 wl.inv_cell_v, wl.oversample, wl.height, wl.width, wl.n_planes, wl.w_min, wl.inv_dw)
    e = float(np.linalg.norm(got - want) / np.linalg.norm(want))
    _say(f"  {wl.n_vis} visibilities, {dropped} dropped, rel L2 {e:.2e}")
    assert stats.tolist() == [wl.n_vis - dropped, dropped]
    assert dropped >= 41
    assert e <= 1e-5


def test_aterm_integer_values_exact(R):
    from paper_1605_07023_amd import binding as B
    _say("A-term gridding, integer taps and visibilities, exact")
    P, S = 4, 16
    wl = aterm_workload(S, n_baselines=2, grid=512, n_pol=P)
    rng = np.random.default_rng(8)
    wl.vis = (rng.integers(-3, 4, (wl.n_vis, P)) + 1j * rng.integers(-3, 4, (wl.n_vis, P))).astype(np.complex64)
    n_ids = wl.meta["n_ids"]
    shape = (n_ids, wl.n_planes, wl.oversample, wl.oversample, P, S, S)
    taps = (rng.integers(-1, 2, shape) + 1j * rng.integers(-1, 2, shape)).astype(np.complex64)
    taps_dev = torch.from_numpy(np.ascontiguousarray(taps).view(np.float32)).to(DEV)
    got, stats = _run(R, wl, wl.meta["kernel_id"], n_ids, taps_dev, B.GR_F32)
    want, dropped = G.grid_aterm(wl.vis, wl.uvw, None, wl.meta["kernel_id"], taps.astype(np.complex128),
                                 wl.inv_cell_u, wl.inv_cell_v, wl.oversample, wl.height, wl.width, wl.n_planes,
                                 wl.w_min, wl.inv_dw)
    np.testing.assert_array_equal(got, want)
    assert stats.tolist() == [wl.n_vis - dropped, dropped]


def test_aterm_edge_cases(R):
    """Empty stream; only bad ids: the grid keeps its contents and every visibility is counted dropped."""
    from paper_1605_07023_amd import binding as B
    _say("A-term gridding edge cases")
    P, S = 1, 8
    wl = aterm_workload(S, n_baselines=1, grid=256, n_pol=P)
    n_ids = wl.meta["n_ids"]
    taps = aterm_taps(1, n_ids, wl.n_planes, wl.oversample, P, S)
    taps_dev = torch.from_numpy(np.ascontiguousarray(taps).view(np.float32)).to(DEV)
    bad = np.full(wl.n_vis, n_ids, np.int32)
    got, stats = _run(R, wl, bad, n_ids, taps_dev, B.GR_F32)
    assert not np.any(got) and stats.tolist() == [0, wl.n_vis]
    import dataclasses
    empty = dataclasses.replace(wl, uvw=wl.uvw[:0], vis=wl.vis[:0])
    dw = R.upload(empty, DEV, taps=taps_dev)
    dw.kernel = B.make_kernel(taps_dev, S, wl.oversample, wl.n_planes, taps_complex=True, w_min=wl.w_min,
                              inv_dw=wl.inv_dw, kind=B.GR_TABLE2D)
    g = torch.full((P, wl.height, wl.width), 2.0 + 1.0j, dtype=torch.complex64, device=DEV)
    R.grid_aterm(dw, torch.zeros(1, dtype=torch.int32, device=DEV), n_ids, grid_out=g)
    torch.cuda.synchronize()
    assert bool(torch.all(g == (2.0 + 1.0j)))


def test_aterm_largest_id_space(R):
    """n_ids x n_planes = 32767, the most the record's 15-bit plane field holds: the largest id
    and plane grid correctly, ids past the end are dropped."""
    import dataclasses
    from paper_1605_07023_amd import binding as B
    from synth import random_point_workload
    _say("A-term gridding, 32767 GCF ids")
    P, S, n_ids = 1, 2, 32767
    wl = random_point_workload(20000, P, 64, 64, S, 1, seed=4, n_planes=1, margin=2)
    wl = dataclasses.replace(wl, kernel="aterm")
    rng = np.random.default_rng(6)
    ids = rng.integers(0, n_ids, wl.n_vis).astype(np.int32)
    ids[:50] = n_ids - 1                                     # the largest id
    ids[50:60] = n_ids                                       # one past the end: dropped
    taps = (rng.standard_normal((n_ids, 1, 1, 1, P, S, S))
            + 1j * rng.standard_normal((n_ids, 1, 1, 1, P, S, S))).astype(np.complex64)
    taps_dev = torch.from_numpy(np.ascontiguousarray(taps).view(np.float32)).to(DEV)
    got, stats = _run(R, wl, ids, n_ids, taps_dev, B.GR_F32)
    want, dropped = G.grid_aterm(wl.vis, wl.uvw, None, ids, taps.astype(np.complex128), wl.inv_cell_u,
                                 wl.inv_cell_v, 1, wl.height, wl.width, 1, wl.w_min, wl.inv_dw)
    e = float(np.linalg.norm(got - want) / np.linalg.norm(want))
    _say(f"  {wl.n_vis} visibilities, {dropped} dropped, rel L2 {e:.2e}")
    assert stats.tolist() == [wl.n_vis - dropped, dropped] and dropped >= 10
    assert e <= 1e-5
