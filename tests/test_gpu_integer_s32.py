"""Bit-exact integer checks of the support-32 gridders.

Small-integer visibilities and small-integer complex taps keep every partial
sum an exact FP32 integer, so the grid must equal the FP64 oracle bit for bit
whatever order the matrix-core products and the atomic window additions take.
A lost, doubled or misplaced flush of one part-window (the S = 32 wave form
splits each 48-cell window into 4 row parts at P = 4) changes some cell by a
whole integer and fails here, where a relative-L2 bound could miss it.

Cases: the wave-form MFMA gridder at P = 4 and P = 1 in the default launch
(the 32-plane, oversampling-8 table of the full-shape configuration), the
paper's VALU kernel with 4 x 2 coarsening (and two other coarsenings), and the
full 33M-visibility, 4096^2 shape with integer values on 7 sampled rows
against the C oracle.
"""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import gridding as G  # noqa: E402
from synth import full_shape_workload, random_point_workload  # noqa: E402

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


def _int_taps(rng, planes, O, S):
    """Complex taps with real and imaginary parts in {-1, 0, 1}; [planes][O][S]."""
    return (rng.integers(-1, 2, (planes, O, S)) + 1j * rng.integers(-1, 2, (planes, O, S))).astype(np.complex128)


def _int_vis(rng, n, P, lo=-2, hi=2):
    return (rng.integers(lo, hi + 1, (n, P)) + 1j * rng.integers(lo, hi + 1, (n, P))).astype(np.complex64)


def _upload_int(R, wl, taps):
    from paper_1605_07023_amd import binding as B
    t = torch.from_numpy(np.ascontiguousarray(np.stack([taps.real, taps.imag], -1), dtype=np.float32)).to(DEV)
    dw = R.upload(wl, DEV, taps=t)
    dw.kernel = B.make_kernel(t, wl.support, wl.oversample, wl.n_planes, taps_complex=True,
                              w_min=wl.w_min, inv_dw=wl.inv_dw)
    return dw


def _bound_ok(wl, taps_abs_max=1, vis_abs_max=2):
    """Every partial sum stays below 2^24 in magnitude: a complex contribution
    has |Re|, |Im| <= 4 |V| |T|^2 component bounds, times the largest number of
    footprints on one cell (counted from the oracle's coordinates)."""
    c = G.pixel_coords(wl.uvw, wl.inv_cell_u, wl.inv_cell_v, wl.oversample, wl.support, wl.height,
                       wl.width, wl.n_planes, wl.w_min, wl.inv_dw)
    ok = c["valid"]
    cover = np.zeros((wl.height + 1, wl.width + 1), np.int64)
    x0, y0, S = c["x0"][ok], c["y0"][ok], wl.support
    np.add.at(cover, (y0, x0), 1)
    np.add.at(cover, (y0 + S, x0), -1)
    np.add.at(cover, (y0, x0 + S), -1)
    np.add.at(cover, (y0 + S, x0 + S), 1)
    per_cell = cover.cumsum(0).cumsum(1)
    worst = int(per_cell.max()) * 4 * vis_abs_max * taps_abs_max * taps_abs_max
    return worst < 2 ** 24, int(per_cell.max())


@pytest.mark.parametrize("P,N,seg", [(4, 20000, 0), (4, 9000, 1024), (1, 24000, 0), (1, 7000, 333)])
def test_wave_form_s32_integer_bit_exact(R, P, N, seg):
    """The S = 32 wave form (48-cell windows; 4 row parts at P = 4), default
    launch, with the full-shape table size (32 planes, oversampling 8)."""
    _say(f"S=32 wave form integer bit-exact P={P} N={N} seg_len={seg}")
    rng = np.random.default_rng(100 + P + seg)
    wl = random_point_workload(N, P, 200, 232, 32, 8, seed=200 + P + seg, n_planes=32, margin=4,
                               weights=False, kernel="wsep")
    wl.vis = _int_vis(rng, N, P)
    ok, worst = _bound_ok(wl)
    assert ok, worst
    taps = _int_taps(rng, 32, 8, 32)
    dw = _upload_int(R, wl, taps)
    stats = torch.zeros(2, dtype=torch.int64, device=DEV)
    g = R.grid(dw, tune=R.tuning(vis_per_wg=seg) if seg else None, stats=stats)
    torch.cuda.synchronize()
    ref, dropped = G.grid_separable(wl.vis, wl.uvw, None, taps, 1.0, 1.0, 8, 200, 232, 32, wl.w_min, wl.inv_dw)
    assert stats.cpu().tolist() == [N - dropped, dropped] and dropped > 0
    np.testing.assert_array_equal(g.cpu().numpy().astype(np.complex128), ref)


@pytest.mark.parametrize("cu,cv", [(4, 2), (8, 1), (2, 4)])
def test_romein_valu_s32_integer_bit_exact(R, cu, cv):
    """The paper's VALU kernel (Romein distribution, thread coarsening, flush on
    leaving the bounding box) at S = 32, quad polarisation."""
    _say(f"S=32 VALU kernel integer bit-exact cu={cu} cv={cv}")
    rng = np.random.default_rng(300 + 10 * cu + cv)
    N = 6000
    wl = random_point_workload(N, 4, 144, 176, 32, 8, seed=301 + cu, n_planes=32, margin=3,
                               weights=False, kernel="wsep")
    wl.vis = _int_vis(rng, N, 4)
    ok, worst = _bound_ok(wl)
    assert ok, worst
    taps = _int_taps(rng, 32, 8, 32)
    dw = _upload_int(R, wl, taps)
    g = R.grid(dw, tune=R.tuning(cu, cv, vis_per_wg=512, variant=1))
    torch.cuda.synchronize()
    ref, _ = G.grid_separable(wl.vis, wl.uvw, None, taps, 1.0, 1.0, 8, 144, 176, 32, wl.w_min, wl.inv_dw)
    np.testing.assert_array_equal(g.cpu().numpy().astype(np.complex128), ref)


def test_full_shape_s32_integer_sampled_rows_bit_exact(R, c_oracle):
    """All 33,030,144 quad-pol visibilities of the full shape (64 antennas, 16
    channels, 1024 dumps, 4096^2) with values in {-1, 0, 1} + i{-1, 0, 1} and
    integer taps, gridded in the default launch: 7 sampled rows equal the C
    FP64 oracle's bit for bit."""
    wl = full_shape_workload(32)
    _say(f"full shape S=32 integer values: N={wl.n_vis}")
    rng = np.random.default_rng(32032)
    wl.vis = _int_vis(rng, wl.n_vis, 4, -1, 1)
    ok, worst = _bound_ok(wl, vis_abs_max=1)
    _say(f"    largest footprint count on one cell: {worst}")
    assert ok, worst
    taps = _int_taps(rng, 32, 8, 32)
    dw = _upload_int(R, wl, taps)
    stats = torch.zeros(2, dtype=torch.int64, device=DEV)
    g = R.grid(dw, stats=stats)
    torch.cuda.synchronize()
    assert stats.cpu().tolist() == [wl.n_vis, 0]
    rows = [64, 1100, 2047, 2048, 2049, 2900, 3990]
    got = g[:, rows].cpu().numpy().astype(np.complex128)
    del g, dw
    torch.cuda.empty_cache()
    ref, dropped = c_oracle.grid_separable(wl.vis, wl.uvw, None, taps, wl.inv_cell_u, wl.inv_cell_v, 8,
                                           wl.height, wl.width, wl.n_planes, wl.w_min, wl.inv_dw, rows=rows)
    assert dropped == 0
    assert np.abs(ref).max() > 0
    np.testing.assert_array_equal(got, ref)
