"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle.

Bars: index/record work bit-exact; FP64 table generation within 1e-12;
FP32 gridding within 1e-5 relative L2 of the FP64 grid; integer-valued inputs
(every partial sum exact in FP32) bit-exact regardless of atomic order.
"""
import copy
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import gridding as G  # noqa: E402
from synth import full_shape_workload, random_point_workload, tiny_kb_workload  # noqa: E402

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


def _rel_l2(got, ref):
    return float(np.linalg.norm(got - ref) / max(np.linalg.norm(ref), 1e-300))


def _oracle_grid(wl, taps):
    return G.grid_separable(wl.vis, wl.uvw, wl.weights, taps, wl.inv_cell_u, wl.inv_cell_v,
                            wl.oversample, wl.height, wl.width, wl.n_planes, wl.w_min, wl.inv_dw)


def _oracle_taps(wl):
    if wl.kernel == "kb":
        return G.kb_table(wl.support, wl.oversample, wl.beta)
    if wl.kernel == "w2d":
        return G.wkernel_2d_table(wl.support, wl.oversample, wl.plane_w_hat(), wl.fov,
                                  wl.support_aa, wl.beta)
    return G.wkernel_table(wl.support, wl.oversample, wl.plane_w_hat(), wl.support_aa, wl.beta)


# ------------------------------------------------------------------ tables

@pytest.mark.parametrize("S,O,beta", [(8, 8, 8.6), (16, 4, 10.0), (6, 16, 0.0)])
def test_kb_table_fp64_matches_oracle(R, S, O, beta):
    from paper_1605_07023_amd import binding as B
    _say(f"kb table S={S} O={O} beta={beta}")
    out = torch.empty((O, S), dtype=torch.float64, device=DEV)
    B.gr_make_kb_table(beta, S, O, B.GR_F64, out)
    ref = G.kb_table(S, O, beta)[0]
    np.testing.assert_allclose(out.cpu().numpy(), ref, rtol=0, atol=1e-13)


@pytest.mark.parametrize("S,O,planes", [(16, 8, 5), (32, 8, 3), (8, 4, 2)])
def test_wkernel_table_fp64_matches_oracle(R, S, O, planes):
    from paper_1605_07023_amd import binding as B
    _say(f"wkernel table S={S} O={O} planes={planes}")
    w0, dw = -float(S - 8), 2.0 * (S - 8) / max(planes - 1, 1)
    out = torch.empty((planes, O, S, 2), dtype=torch.float64, device=DEV)
    B.gr_make_wkernel_table(S, O, planes, w0, dw, 8, 8.6, 0, B.GR_F64, out)
    got = out.cpu().numpy()
    got = got[..., 0] + 1j * got[..., 1]
    ref = G.wkernel_table(S, O, w0 + dw * np.arange(planes), 8, 8.6)
    assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()


# ------------------------------------------------------------------ preprocess

def test_preprocess_records_exact(R):
    _say("preprocess records: random points with drops and non-finite values")
    wl = random_point_workload(5000, 4, 96, 128, 16, 8, seed=3, n_planes=9, margin=12,
                               weights=True, kernel="wsep")
    wl.uvw[5, 0] = np.nan
    wl.uvw[6, 2] = np.inf
    wl.uvw[7, 2] = 1e6                  # plane out of range
    wl.vis[8, 2] = np.complex64(complex(np.nan, 0))
    wl.weights[9, 1] = np.inf
    dw = R.upload(wl, DEV)
    stats = torch.zeros(2, dtype=torch.int64, device=DEV)
    rec, _ = R.preprocess(dw, stats)
    got = R.decode_records(rec.cpu().numpy())
    ref = G.pixel_coords(wl.uvw, 1.0, 1.0, 8, 16, 96, 128, 9, wl.w_min, wl.inv_dw)
    valid = ref["valid"] & G.finite_values(wl.vis, wl.weights)
    np.testing.assert_array_equal(got["valid"].astype(bool), valid)
    for k in ("x0", "y0", "sx", "sy", "plane"):
        np.testing.assert_array_equal(got[k][valid], ref[k][valid], err_msg=k)
    assert stats.cpu().tolist() == [int(valid.sum()), int((~valid).sum())]
    assert 0 < (~valid).sum() < wl.n_vis


def test_preprocess_tiny_config_exact(R):
    _say("preprocess records: tiny KB config")
    wl = tiny_kb_workload()
    dw = R.upload(wl, DEV)
    rec, wv = R.preprocess(dw)
    got = R.decode_records(rec.cpu().numpy())
    ref = G.pixel_coords(wl.uvw, wl.inv_cell_u, wl.inv_cell_v, 8, 8, 512, 512)
    assert ref["valid"].all() and got["valid"].all()
    for k in ("x0", "y0", "sx", "sy"):
        np.testing.assert_array_equal(got[k], ref[k], err_msg=k)
    np.testing.assert_array_equal(wv.cpu().numpy(), wl.vis)


# ------------------------------------------------------------------ gridding

TUNINGS_P1 = [(1, 1), (2, 2), (4, 4), (8, 2), (2, 8), (8, 8), (4, 1)]
TUNINGS_P4 = [(1, 1), (2, 2), (4, 2), (2, 4), (4, 4), (8, 2), (8, 1)]


@pytest.mark.parametrize("cu,cv", TUNINGS_P1)
def test_grid_tiny_config(R, cu, cv):
    _say(f"grid tiny KB config VALU cu={cu} cv={cv}")
    wl = tiny_kb_workload()
    dw = R.upload(wl, DEV)
    g = R.grid(dw, tune=R.tuning(cu, cv, variant=1)).cpu().numpy()
    ref, _ = _oracle_grid(wl, _oracle_taps(wl))
    assert _rel_l2(g, ref) <= 1e-5


@pytest.mark.parametrize("seg", [0, 1, 7, 64])
def test_grid_tiny_config_mfma(R, seg):
    _say(f"grid tiny KB config MFMA seg_len={seg}")
    wl = tiny_kb_workload()
    dw = R.upload(wl, DEV)
    g = R.grid(dw, tune=R.tuning(vis_per_wg=seg, variant=2)).cpu().numpy()
    ref, _ = _oracle_grid(wl, _oracle_taps(wl))
    assert _rel_l2(g, ref) <= 1e-5


@pytest.mark.parametrize("S,P,seg", [(8, 4, 0), (16, 4, 33), (32, 4, 4096), (16, 1, 5), (32, 1, 0),
                                     (56, 4, 100), (2, 1, 3)])
def test_grid_points_mfma(R, S, P, seg):
    _say(f"grid random points MFMA S={S} P={P} seg_len={seg}")
    wl = random_point_workload(4001, P, 200, 136, S, 8, seed=S + P, n_planes=5, margin=6,
                               weights=True, kernel="wsep" if S >= 8 else "kb")
    if S < 8:
        wl.beta = 2.0
    dw = R.upload(wl, DEV)
    stats = torch.zeros(2, dtype=torch.int64, device=DEV)
    g = R.grid(dw, tune=R.tuning(vis_per_wg=seg, variant=2), stats=stats).cpu().numpy()
    ref, dropped = _oracle_grid(wl, _oracle_taps(wl))
    assert _rel_l2(g, ref) <= 1e-5
    assert stats.cpu().tolist() == [wl.n_vis - dropped, dropped] and dropped > 0


# The single-problem MFMA gridder has four forms, chosen by the LDS its tap
# table needs (complex W taps, O = 8; 160 KiB of LDS):
#   wave form, gapped table (rows of W entries, W = 48 at S = 32, 32 at S = 16, plus
#   a lead of W - S), triple entries (12 B) or (Re, Im) pairs (8 B), + one slice of
#   32 pair records per wave (16 waves at S = 32, 12 at S = 16; P = 4: 2944 B with
#   triples, 3968 B with pairs; P = 1: 1408 B / 1664 B);
#   block form, rows of S + 2 entries, triple: table + 12,800 B (P = 4) / 6,656 B (P = 1);
#   block form, (Re, Im) pairs: pair table + 12,288 B (P = 4).
# At S = 32, 40 planes (320 rows) at P = 4 take the triple block form, 60 planes (480
# rows) the pair block form, 48 planes (384 rows) at P = 1 the triple block form.
# Wave form table kinds: at S = 32, P = 4, 5 planes fit triple entries, 32 planes
# (256 rows, the full-shape table) only pairs; at P = 1, 36 planes (288 rows) take
# pairs; at S = 16, P = 4, 48 planes (384 rows) take pairs.  A pair table whose
# planes are conjugate pairs (plane n - 1 - p the conjugate of plane p, as a W
# kernel's at w symmetric about 0) is read through the mirror plane; `mirror`
# builds such a table.  Integer visibilities and taps keep every sum exact, so
# each kind must equal the FP64 oracle bit for bit.
@pytest.mark.parametrize("S,P,planes,rg,mirror", [(32, 4, 5, 0, False), (32, 4, 32, 0, False),
                                                  (32, 4, 32, 4, False), (32, 1, 36, 0, False),
                                                  (16, 4, 5, 0, False), (16, 4, 48, 0, False),
                                                  (16, 4, 48, 4, False), (32, 4, 32, 0, True),
                                                  (32, 4, 31, 3, True), (32, 1, 36, 0, True),
                                                  (16, 4, 48, 0, True)])
def test_wave_form_table_kinds_bit_exact(R, S, P, planes, rg, mirror):
    _say(f"wave form table kinds, integer inputs, S={S} P={P} planes={planes} row groups={rg} mirror={mirror}")
    rng = np.random.default_rng(S * 100 + planes + P)
    wl = random_point_workload(3000, P, 120, 104, S, 8, seed=planes + S, n_planes=planes, margin=4,
                               weights=False, kernel="wsep")
    wl.vis = (rng.integers(-2, 3, (wl.n_vis, P)) + 1j * rng.integers(-2, 3, (wl.n_vis, P))).astype(np.complex64)
    taps = rng.integers(-1, 2, (planes, 8, S)) + 1j * rng.integers(-1, 2, (planes, 8, S))
    if mirror:
        half = planes // 2
        taps[planes - half:] = np.conj(taps[:half][::-1])
        if planes & 1:
            taps[half] = taps[half].real
        assert np.array_equal(taps, np.conj(taps[::-1]))
    taps_np = np.stack([taps.real, taps.imag], axis=-1)
    g = _custom_taps_run(R, wl, taps_np, R.tuning(0, 0, 0, rg, 0, variant=2))
    ref, dropped = _oracle_grid(wl, taps)
    assert wl.n_vis - dropped > 2000
    assert np.abs(ref).max() < 2 ** 20
    np.testing.assert_array_equal(g.astype(np.complex128), ref)


@pytest.mark.parametrize("S,planes,dt", [(32, 32, "f32"), (16, 32, "f32"), (16, 7, "f64"), (8, 1, "f32")])
def test_wkernel_table_planes_conjugate(R, S, planes, dt):
    """gr_make_wkernel_table at w values symmetric about 0 gives mirror planes
    that are exact complex conjugates (the table form the gridder reads through
    the mirror plane), and stays within 1e-12 of the FP64 oracle's taps."""
    from paper_1605_07023_amd import binding as B
    _say(f"W table conjugate planes S={S} planes={planes} dtype={dt}")
    wh = np.linspace(-1.5 * S, 1.5 * S, planes) if planes > 1 else np.zeros(1)
    step = float(wh[1] - wh[0]) if planes > 1 else 0.0
    tdt, code = {"f32": (torch.float32, B.GR_F32), "f64": (torch.float64, B.GR_F64)}[dt]
    out = torch.empty((planes, 8, S, 2), dtype=tdt, device=DEV)
    B.gr_make_wkernel_table(S, 8, planes, float(wh[0]), step, max(S - 2, 1), 2.0 * S / 4, 0, code, out, None)
    t = out.cpu().numpy().astype(np.float64)
    z = t[..., 0] + 1j * t[..., 1]
    np.testing.assert_array_equal(z, np.conj(z[::-1]))
    assert np.abs(z).max() > 0.01
    if dt == "f64":
        ref = G.wkernel_table(S, 8, float(wh[0]) + step * np.arange(planes), max(S - 2, 1), 2.0 * S / 4)
        assert np.abs(z - ref).max() <= 1e-12 * np.abs(ref).max()


@pytest.mark.parametrize("P,planes,seg", [(4, 40, 0), (4, 40, 77), (4, 60, 0), (1, 48, 9)])
def test_grid_points_mfma_block_forms(R, P, planes, seg):
    _say(f"grid random points MFMA block forms P={P} planes={planes} seg_len={seg}")
    wl = random_point_workload(3001, P, 160, 144, 32, 8, seed=planes + P, n_planes=planes, margin=6,
                               weights=True, kernel="wsep")
    dw = R.upload(wl, DEV)
    g = R.grid(dw, tune=R.tuning(vis_per_wg=seg, variant=2)).cpu().numpy()
    ref, _ = _oracle_grid(wl, _oracle_taps(wl))
    assert _rel_l2(g, ref) <= 1e-5


@pytest.mark.parametrize("n,P", [(3000, 1), (1537, 4)])
def test_fused_binning_many_tiles_per_block_bit_exact(R, n, P):
    """The fused binning's scatter groups each block of 512 visibilities by
    tile in a 512-slot table: on a 2048^2 grid of 16-cell tiles nearly every
    visibility of a block has a tile of its own (the table nearly full), and a
    ragged last block.  Integer values and taps: the grid of gr_grid (fused
    binning, MFMA gridder) equals the FP64 oracle's bit for bit, statistics too."""
    from paper_1605_07023_amd import binding as B
    _say(f"fused binning, many tiles per block, n={n} P={P}")
    rng = np.random.default_rng(n + P)
    S, H, W = 16, 2048, 2048
    wl = random_point_workload(n, P, H, W, S, 8, seed=n + 3 * P, n_planes=2, margin=4, weights=False,
                               kernel="wsep")
    wl.vis = (rng.integers(-2, 3, (wl.n_vis, P)) + 1j * rng.integers(-2, 3, (wl.n_vis, P))).astype(np.complex64)
    taps = rng.integers(-1, 2, (2, 8, S)) + 1j * rng.integers(-1, 2, (2, 8, S))
    t = torch.from_numpy(np.ascontiguousarray(np.stack([taps.real, taps.imag], axis=-1), dtype=np.float32)).to(DEV)
    dw = R.upload(wl, DEV, taps=t)
    dw.kernel = B.make_kernel(t, S, 8, 2, taps_complex=True, w_min=wl.w_min, inv_dw=wl.inv_dw)
    stats = torch.zeros(2, dtype=torch.int64, device=DEV)
    g = R.grid(dw, tune=R.tuning(vis_per_wg=64, variant=2), stats=stats).cpu().numpy()
    ref, dropped = _oracle_grid(wl, taps)
    assert stats.cpu().tolist() == [wl.n_vis - dropped, dropped]
    assert wl.n_vis - dropped > n // 2
    np.testing.assert_array_equal(g.astype(np.complex128), ref)


@pytest.mark.parametrize("P,seg", [(4, 0), (1, 45)])
def test_preprocess_bin_equals_separate_calls(R, P, seg):
    """gr_preprocess_bin (fused) + gr_grid_binned against gr_preprocess + gr_bin +
    gr_grid_binned and the FP64 oracle, with coordinate drops and non-finite
    visibilities and weights: integer values and taps, so every grid is exact;
    statistics equal; the fused binned stream holds the same kept entries plus
    one zero-valued entry per visibility dropped for its values."""
    from paper_1605_07023_amd import binding as B
    _say(f"fused preprocess+bin vs separate calls P={P} seg_len={seg}")
    rng = np.random.default_rng(40 + P)
    wl = random_point_workload(3000, P, 80, 72, 16, 4, seed=41 + P, n_planes=3, margin=5, weights=True,
                               kernel="wsep")
    wl.vis = (rng.integers(-2, 3, (wl.n_vis, P)) + 1j * rng.integers(-2, 3, (wl.n_vis, P))).astype(np.complex64)
    wl.weights = rng.integers(1, 3, (wl.n_vis, P)).astype(np.float32)
    wl.uvw[3, 1] = np.nan
    wl.uvw[4, 2] = np.inf
    wl.vis[10, P - 1] = np.complex64(complex(0, np.inf))
    wl.vis[11, 0] = np.complex64(complex(np.nan, 1))
    wl.weights[12, 0] = np.nan
    taps = rng.integers(-1, 2, (3, 4, 16)) + 1j * rng.integers(-1, 2, (3, 4, 16))
    t = torch.from_numpy(np.ascontiguousarray(np.stack([taps.real, taps.imag], axis=-1), dtype=np.float32)).to(DEV)
    dw = R.upload(wl, DEV, taps=t)
    k = B.make_kernel(t, 16, 4, 3, taps_complex=True, w_min=wl.w_min, inv_dw=wl.inv_dw)
    N, H, W = wl.n_vis, wl.height, wl.width
    # separate calls
    st_a = torch.zeros(2, dtype=torch.int64, device=DEV)
    rec = torch.empty((N, 2), dtype=torch.int32, device=DEV)
    wv = torch.empty((N, P), dtype=torch.complex64, device=DEV)
    B.gr_preprocess(dw.uvw, dw.vis, B.GR_F32, None, dw.weights, N, P, k, 1.0, 1.0, H, W, rec, wv, st_a)
    nb_a = B.gr_bin_bytes(N, P, 16, H, W, seg)
    bins_a = torch.empty(nb_a, dtype=torch.uint8, device=DEV)
    B.gr_bin(rec, wv, N, P, 16, H, W, seg, bins_a, nb_a)
    g_a = torch.zeros((P, H, W), dtype=torch.complex64, device=DEV)
    B.gr_grid_binned(bins_a, N, P, k, seg, g_a, H, W)
    # fused
    st_b = torch.zeros(2, dtype=torch.int64, device=DEV)
    nb_b = B.gr_preprocess_bin_bytes(N, P, 16, H, W, seg)
    assert nb_b >= nb_a + 8 * N
    bins_b = torch.empty(nb_b, dtype=torch.uint8, device=DEV)
    B.gr_preprocess_bin(dw.uvw, dw.vis, B.GR_F32, None, dw.weights, N, P, k, 1.0, 1.0, H, W, seg, bins_b, nb_b,
                        st_b)
    g_b = torch.zeros((P, H, W), dtype=torch.complex64, device=DEV)
    B.gr_grid_binned(bins_b, N, P, k, seg, g_b, H, W)
    torch.cuda.synchronize()
    ref, dropped = _oracle_grid(wl, taps)
    np.testing.assert_array_equal(g_a.cpu().numpy().astype(np.complex128), ref)
    np.testing.assert_array_equal(g_b.cpu().numpy().astype(np.complex128), ref)
    assert st_a.cpu().tolist() == st_b.cpu().tolist() == [N - dropped, dropped]
    # binned streams: kept entries as a multiset of (record, values)
    coord_ok = G.pixel_coords(wl.uvw, 1.0, 1.0, 4, 16, H, W, 3, wl.w_min, wl.inv_dw)["valid"]
    value_drops = int((coord_ok & ~G.finite_values(wl.vis, wl.weights)).sum())
    assert value_drops == 3

    def entries(raw, n_kept):
        b = raw.cpu().numpy()
        recs = b[:8 * N].view(np.uint32).reshape(N, 2)[:n_kept]
        off = (8 * N + 255) // 256 * 256
        vals = b[off:off + 8 * P * N].view(np.float32).reshape(N, 2 * P)[:n_kept]
        return sorted(zip(map(tuple, recs.tolist()), map(tuple, vals.tolist())))

    ea, eb = entries(bins_a, N - dropped), entries(bins_b, N - dropped + value_drops)
    zero = tuple([0.0] * (2 * P))
    extra = list(eb)
    for e in ea:
        extra.remove(e)
    assert len(extra) == value_drops and all(v == zero for _, v in extra)


def test_bin_is_a_grouping_of_the_valid_stream(R):
    """gr_bin output: every valid record exactly once, each segment inside its
    tile, segment lengths <= seg_len, input order kept within runs."""
    from paper_1605_07023_amd import binding as B
    _say("gr_bin grouping")
    S, seg = 16, 50
    wl = random_point_workload(3000, 4, 256, 192, S, 8, seed=1, n_planes=3, margin=4,
                               weights=False, kernel="wsep")
    dw = R.upload(wl, DEV)
    rec, wv = R.preprocess(dw)
    nb = B.gr_bin_bytes(wl.n_vis, 4, S, 256, 192, seg)
    bins = torch.zeros(nb, dtype=torch.uint8, device=DEV)
    B.gr_bin(rec, wv, wl.n_vis, 4, S, 256, 192, seg, bins, nb)
    torch.cuda.synchronize()
    raw = bins.cpu().numpy()
    r_in = rec.cpu().numpy().view(np.uint64).ravel()
    valid = (r_in >> np.uint64(63)) == 1
    nv = int(valid.sum())
    r_out = raw[:8 * nv].view(np.uint64)
    np.testing.assert_array_equal(np.sort(r_out), np.sort(r_in[valid]))
    # weighted visibilities travel with their records
    off_w = (8 * wl.n_vis + 255) // 256 * 256
    w_out = raw[off_w:off_w + 32 * nv].view(np.complex64).reshape(nv, 4)
    w_in = wv.cpu().numpy()[valid]
    order = {int(k): i for i, k in enumerate(r_in[valid])}
    # records can repeat in principle; this draw has unique records
    assert len(order) == nv
    np.testing.assert_array_equal(w_out, w_in[[order[int(k)] for k in r_out]])
    T = (32 if S <= 16 else 48 if S <= 32 else 64) - S      # the binning tile documented for gr_bin
    n_tx, n_ty = -(-192 // T), -(-256 // T)
    off = off_w + (32 * wl.n_vis + 255) // 256 * 256
    off += 2 * ((4 * n_tx * n_ty + 255) // 256 * 256)
    max_segs = n_tx * n_ty + -(-wl.n_vis // seg)
    segs = raw[off:off + 16 * max_segs].view(np.int32).reshape(-1, 4)
    n_segs = int(raw[off + (16 * max_segs + 255) // 256 * 256:][:4].view(np.int32)[0])
    segs = segs[:n_segs]
    assert segs[:, 1].sum() == nv and segs[:, 1].max() <= seg and segs[:, 1].min() >= 1
    x0 = (r_out & np.uint64(0xFFFF)).astype(np.int64)
    y0 = ((r_out >> np.uint64(16)) & np.uint64(0xFFFF)).astype(np.int64)
    for b, ln, t, _ in segs:
        assert np.all(x0[b:b + ln] // T == t % n_tx) and np.all(y0[b:b + ln] // T == t // n_tx)


def _box_class(xr, yr, S, rg, tile):
    """The pairing class of a footprint at (xr, yr) in its window: first row
    group, first column group of 8, and whether it reaches one more of each."""
    nc = (tile - 1) // 8 + 1
    dc = ((xr % 8) + S - 1) // 8 - (S - 1) // 8
    dg = ((yr % rg) + S - 1) // rg - (S - 1) // rg
    return (((yr // rg) * nc + xr // 8) * 2 + dc) * 2 + dg


@pytest.mark.parametrize("S,P,seg", [(32, 4, 300), (16, 4, 4096), (32, 1, 77), (8, 4, 1000), (32, 4, 32768),
                                     (16, 4, 40000)])
def test_pairing_order_is_a_class_sort_of_each_segment(R, S, P, seg):
    """gr_grid_binned's pairing order (the last region of the bins buffer): per
    segment a permutation of the segment's entries, their D-tile classes
    non-decreasing (entries of one class may come in any order); and the grid
    equals the FP64 oracle's.  Segment lengths up to 32768 keep the classes in
    LDS between the ordering's two passes, longer ones read the records again."""
    from paper_1605_07023_amd import binding as B
    _say(f"pairing order S={S} P={P} seg_len={seg}")
    rng = np.random.default_rng(S + P + seg)
    H, W = 200, 168
    wl = random_point_workload(4000, P, H, W, S, 8, seed=S * 7 + P, n_planes=3, margin=4,
                               weights=False, kernel="wsep")
    wl.vis = (rng.integers(-2, 3, (wl.n_vis, P)) + 1j * rng.integers(-2, 3, (wl.n_vis, P))).astype(np.complex64)
    taps = rng.integers(-1, 2, (3, 8, S)) + 1j * rng.integers(-1, 2, (3, 8, S))
    t = torch.from_numpy(np.ascontiguousarray(np.stack([taps.real, taps.imag], axis=-1), dtype=np.float32)).to(DEV)
    dw = R.upload(wl, DEV, taps=t)
    k = B.make_kernel(t, S, 8, 3, taps_complex=True, w_min=wl.w_min, inv_dw=wl.inv_dw)
    rec, wv = R.preprocess(dw)
    N = wl.n_vis
    nb = B.gr_bin_bytes(N, P, S, H, W, seg)
    bins = torch.zeros(nb, dtype=torch.uint8, device=DEV)
    B.gr_bin(rec, wv, N, P, S, H, W, seg, bins, nb)
    g = torch.zeros((P, H, W), dtype=torch.complex64, device=DEV)
    B.gr_grid_binned(bins, N, P, k, seg, g, H, W)
    torch.cuda.synchronize()
    ref, _ = _oracle_grid(wl, taps)
    np.testing.assert_array_equal(g.cpu().numpy().astype(np.complex128), ref)
    raw = bins.cpu().numpy()
    r_all = raw[:8 * N].view(np.uint64)
    order = raw[nb - (4 * N + 255) // 256 * 256:][:4 * N].view(np.int32)
    T = (32 if S <= 16 else 48 if S <= 32 else 64) - S
    rg = 16 // P
    n_tx, n_ty = -(-W // T), -(-H // T)
    off = (8 * N + 255) // 256 * 256 + (8 * P * N + 255) // 256 * 256
    off += 2 * ((4 * n_tx * n_ty + 255) // 256 * 256)
    max_segs = n_tx * n_ty + -(-N // seg)
    segs = raw[off:off + 16 * max_segs].view(np.int32).reshape(-1, 4)
    n_segs = int(raw[off + (16 * max_segs + 255) // 256 * 256:][:4].view(np.int32)[0])
    assert n_segs > 1
    multi = 0
    for b, ln, tid, _ in segs[:n_segs]:
        o = order[b:b + ln].astype(np.int64)
        np.testing.assert_array_equal(np.sort(o), np.arange(b, b + ln))
        r = r_all[o]
        xr = (r & np.uint64(0xFFFF)).astype(np.int64) - (tid % n_tx) * T
        yr = ((r >> np.uint64(16)) & np.uint64(0xFFFF)).astype(np.int64) - (tid // n_tx) * T
        c = _box_class(xr, yr, S, rg, T)
        assert np.all(np.diff(c) >= 0)
        multi += len(np.unique(c)) > 1
    assert multi > 0


@pytest.mark.parametrize("cu,cv", TUNINGS_P4)
@pytest.mark.parametrize("S", [8, 16])
def test_grid_points_wkernel_p4(R, cu, cv, S):
    _say(f"grid random points W kernel S={S} P=4 cu={cu} cv={cv}")
    wl = random_point_workload(3001, 4, 80, 112, S, 8, seed=S + cu, n_planes=7, margin=6,
                               weights=True, kernel="wsep")
    dw = R.upload(wl, DEV)
    stats = torch.zeros(2, dtype=torch.int64, device=DEV)
    g = R.grid(dw, tune=R.tuning(cu, cv, vis_per_wg=256), stats=stats).cpu().numpy()
    ref, dropped = _oracle_grid(wl, _oracle_taps(wl))
    assert _rel_l2(g, ref) <= 1e-5
    assert stats.cpu().tolist() == [wl.n_vis - dropped, dropped] and dropped > 0


@pytest.mark.parametrize("variant", [0, 1])
@pytest.mark.parametrize("wg_u,wg_v,vpw", [(3, 5, 7), (16, 4, 1), (1, 1, 100000), (5, 1, 33), (64, 64, 64)])
def test_grid_tile_shapes_and_ragged_chunks(R, wg_u, wg_v, vpw, variant):
    """Variant 1: the VALU kernel with its blocks taken in tiles of wg_u x wg_v
    and chunks of vpw visibilities (ragged); variant 0: the library's choice
    (the binned MFMA path, which ignores the tile fields and takes vpw as its
    segment length)."""
    _say(f"grid tile shape {wg_u}x{wg_v} vis_per_wg={vpw} variant={variant}")
    wl = random_point_workload(777, 1, 64, 48, 16, 8, seed=5, n_planes=3, margin=2,
                               weights=False, kernel="wsep")
    dw = R.upload(wl, DEV)
    g = R.grid(dw, tune=R.tuning(2, 4, wg_u, wg_v, vpw, variant=variant)).cpu().numpy()
    ref, _ = _oracle_grid(wl, _oracle_taps(wl))
    assert _rel_l2(g, ref) <= 1e-5


@pytest.mark.parametrize("P,S", [(4, 16), (4, 32), (1, 16), (1, 32), (4, 56)])
def test_mfma_row_groups_per_wave(R, P, S):
    """Every row-group count the autotuner offers for the MFMA wave form grids
    the same points as the oracle (the work-group shape dimension of the sweep)."""
    from paper_1605_07023_amd import autotune as A
    wl = random_point_workload(2500, P, 160, 144, S, 8, seed=40 + S + P, n_planes=5, margin=3,
                               weights=True, kernel="wsep")
    ref, _ = _oracle_grid(wl, _oracle_taps(wl))
    dw = R.upload(wl, DEV)
    for rg in A.row_group_options(P, S):
        _say(f"mfma P={P} S={S} row groups per wave {rg}")
        g = R.grid(dw, tune=R.tuning(0, 0, 0, rg, 512, variant=2)).cpu().numpy()
        assert _rel_l2(g, ref) <= 1e-5, rg


def _custom_taps_run(R, wl, taps_np, tune):
    from paper_1605_07023_amd import binding as B
    t = torch.from_numpy(np.ascontiguousarray(taps_np.astype(np.float32))).to(DEV)
    dw = R.upload(wl, DEV, taps=t)
    dw.kernel = B.make_kernel(t, wl.support, wl.oversample, wl.n_planes,
                              taps_complex=(taps_np.ndim == 4), w_min=wl.w_min, inv_dw=wl.inv_dw)
    return R.grid(dw, tune=tune).cpu().numpy()


@pytest.mark.parametrize("cu,cv,variant", [(1, 1, 1), (4, 2, 1), (8, 8, 1), (0, 0, 2)])
def test_delta_table_and_integer_inputs_bit_exact(R, cu, cv, variant):
    """Integer visibilities with integer taps: every partial sum is an exact
    FP32 integer, so the grid must equal the FP64 oracle bit for bit whatever
    order the atomics land in (a lost or duplicated flush would show)."""
    _say(f"integer-valued inputs bit-exact cu={cu} cv={cv} variant={variant}")
    rng = np.random.default_rng(cu * 10 + cv)
    wl = random_point_workload(4000, 1, 64, 64, 8, 8, seed=11, weights=False)
    wl.vis = (rng.integers(-3, 4, (wl.n_vis, 1)) + 1j * rng.integers(-3, 4, (wl.n_vis, 1))).astype(np.complex64)
    # delta table: every visibility lands on its own cell
    delta = np.zeros((1, 8, 8))
    delta[:, :, 3] = 1.0
    g = _custom_taps_run(R, wl, delta, R.tuning(cu, cv, vis_per_wg=64, variant=variant))
    ref, _ = _oracle_grid(wl, delta)
    np.testing.assert_array_equal(g.astype(np.complex128), ref)
    # small-integer taps in {0, 1, 2}
    ints = rng.integers(0, 3, (1, 8, 8)).astype(np.float64)
    g = _custom_taps_run(R, wl, ints, R.tuning(cu, cv, vis_per_wg=64, variant=variant))
    ref, _ = _oracle_grid(wl, ints)
    assert np.abs(ref).max() < 2 ** 20
    np.testing.assert_array_equal(g.astype(np.complex128), ref)


@pytest.mark.parametrize("variant", [1, 2])
def test_integer_complex_taps_quad_pol_bit_exact(R, variant):
    _say(f"integer complex taps, quad pol, bit-exact, variant={variant}")
    rng = np.random.default_rng(7)
    wl = random_point_workload(2000, 4, 48, 56, 16, 4, seed=12, n_planes=3, weights=False,
                               kernel="wsep")
    wl.vis = (rng.integers(-2, 3, (wl.n_vis, 4)) + 1j * rng.integers(-2, 3, (wl.n_vis, 4))).astype(np.complex64)
    taps = (rng.integers(-1, 2, (3, 4, 16)) + 1j * rng.integers(-1, 2, (3, 4, 16)))
    taps_np = np.stack([taps.real, taps.imag], axis=-1)
    g = _custom_taps_run(R, wl, taps_np, R.tuning(4 if variant == 1 else 0, 2 if variant == 1 else 0,
                                                   vis_per_wg=128, variant=variant))
    ref, _ = _oracle_grid(wl, taps)
    np.testing.assert_array_equal(g.astype(np.complex128), ref)


@pytest.mark.parametrize("variant", [1, 2])
def test_accumulates_and_edge_cases(R, variant):
    _say(f"accumulate into existing grid; empty input; all dropped; variant={variant}")
    tune = R.tuning(variant=variant)
    wl = random_point_workload(500, 4, 40, 40, 8, 8, seed=2, n_planes=1, kernel="kb")
    dw = R.upload(wl, DEV)
    base = (torch.randn(4, 40, 40, dtype=torch.complex64, device=DEV))
    g0 = base.clone()
    R.grid(dw, grid_out=g0, tune=tune)
    ref, _ = _oracle_grid(wl, _oracle_taps(wl))
    got = g0.cpu().numpy().astype(np.complex128) - base.cpu().numpy()
    assert _rel_l2(got, ref) <= 1e-5
    # empty input leaves the grid untouched
    e = copy.copy(wl)
    e.uvw, e.vis = wl.uvw[:0], wl.vis[:0]
    de = R.upload(e, DEV)
    g1 = base.clone()
    R.grid(de, grid_out=g1, tune=tune)
    assert torch.equal(g1, base)
    # every visibility off the grid: dropped and counted, grid untouched
    off = copy.copy(wl)
    off.uvw = wl.uvw.copy()
    off.uvw[:, 0] += 1000.0
    do = R.upload(off, DEV)
    stats = torch.zeros(2, dtype=torch.int64, device=DEV)
    g2 = base.clone()
    R.grid(do, grid_out=g2, stats=stats, tune=tune)
    assert torch.equal(g2, base)
    assert stats.cpu().tolist() == [0, wl.n_vis]


# ------------------------------------------------------------------ full shape

@pytest.fixture(scope="module")
def full_S16():
    return full_shape_workload(16)


@pytest.mark.parametrize("S,variant", [(16, 2), (32, 2), (32, 1)])
def test_full_shape_sampled_rows(R, c_oracle, S, variant, full_S16):
    """The 64-antenna, 16-channel, 1024-dump, quad-pol 4096^2 workload at full
    size, in the default launch configuration, checked on sampled grid rows
    against the FP64 C oracle (which computes those rows from every visibility)."""
    wl = full_S16 if S == 16 else full_shape_workload(32)
    _say(f"full shape S={S} variant={variant}: N={wl.n_vis}")
    dw = R.upload(wl, DEV)
    stats = torch.zeros(2, dtype=torch.int64, device=DEV)
    g = R.grid(dw, stats=stats, tune=R.tuning(variant=variant))
    torch.cuda.synchronize()
    assert stats.cpu().tolist() == [wl.n_vis, 0]
    rows = [64, 1100, 2047, 2048, 2049, 2900, 3990]
    got = g[:, rows].cpu().numpy()
    del g, dw
    torch.cuda.empty_cache()
    ref, dropped = c_oracle.grid_separable(wl.vis, wl.uvw, None, _oracle_taps(wl), wl.inv_cell_u,
                                           wl.inv_cell_v, 8, wl.height, wl.width, wl.n_planes,
                                           wl.w_min, wl.inv_dw, rows=rows)
    assert dropped == 0
    err = _rel_l2(got, ref)
    _say(f"full shape S={S}: sampled-row rel L2 = {err:.3e}")
    assert err <= 1e-5


# ------------------------------------------------------------------ autotuning

def test_autotune_picks_fastest_valid_candidate(R, c_oracle):
    from paper_1605_07023_amd import autotune as A
    from paper_1605_07023_amd import binding as B
    _say("autotune sweep on a small workload")
    wl = full_shape_workload(16, n_baselines=16)
    dw = R.upload(wl, DEV)
    cands = [B.GrTuning(1, 1, 0, 0, 1024, 1), B.GrTuning(4, 2, 0, 0, 1024, 1),
             B.GrTuning(8, 8, 0, 0, 1024, 1),            # over the register budget at P = 4
             B.GrTuning(0, 0, 0, 0, 512, 2), B.GrTuning(0, 0, 0, 0, 4096, 2)]
    best, times = A.tune(dw, cands, reps=2)
    assert times[2] == float("inf")
    finite = [t for t in times if t != float("inf")]
    assert len(finite) == 4 and min(finite) == times[cands.index(best)]
    g = R.grid(dw, tune=best).cpu().numpy()
    ref, _ = c_oracle.grid_separable(wl.vis, wl.uvw, None, _oracle_taps(wl), wl.inv_cell_u,
                                     wl.inv_cell_v, 8, wl.height, wl.width, wl.n_planes, wl.w_min,
                                     wl.inv_dw)
    assert _rel_l2(g, ref) <= 1e-5


# ------------------------------------------------------------------ exact 2-D W kernel

@pytest.mark.parametrize("S,O,planes,fov", [(8, 2, 3, 0.5), (16, 4, 2, 0.9)])
def test_wkernel2d_table_fp64_matches_oracle(R, S, O, planes, fov):
    from paper_1605_07023_amd import binding as B
    _say(f"2-D W table S={S} O={O} planes={planes} fov={fov}")
    w0, dw = -float(S - 8) or -3.0, 2.0 * (float(S - 8) or 3.0) / max(planes - 1, 1)
    out = torch.empty((planes, O, O, S, S, 2), dtype=torch.float64, device=DEV)
    B.gr_make_wkernel2d_table(S, O, planes, w0, dw, fov, 8, 8.6, 0, B.GR_F64, out)
    got = out.cpu().numpy()
    got = got[..., 0] + 1j * got[..., 1]
    ref = G.wkernel_2d_table(S, O, w0 + dw * np.arange(planes), fov, 8, 8.6)
    assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()


@pytest.mark.parametrize("P,seg,S", [(4, 0, 16), (1, 37, 16), (4, 5, 16), (4, 0, 32), (1, 11, 40), (4, 0, 40)])
def test_grid_table2d(R, P, seg, S):
    """The 2-D table path over the 32-, 48- and 64-cell windows (S = 16, 32, 40)."""
    _say(f"grid with the 2-D table P={P} seg={seg} S={S}")
    wl = random_point_workload(2500, P, 96, 72, S, 4, seed=P + seg, n_planes=5, margin=5,
                               weights=True, kernel="w2d")
    dw = R.upload(wl, DEV)
    stats = torch.zeros(2, dtype=torch.int64, device=DEV)
    g = R.grid(dw, tune=R.tuning(vis_per_wg=seg), stats=stats).cpu().numpy()
    ref, dropped = G.grid_table2d(wl.vis, wl.uvw, wl.weights, _oracle_taps(wl), 1.0, 1.0, 4, 96, 72,
                                  5, wl.w_min, wl.inv_dw)
    assert _rel_l2(g, ref) <= 1e-5
    assert stats.cpu().tolist() == [wl.n_vis - dropped, dropped]
