"""gr_grid_records, the paper's kernel called directly (its waves take their
64-lane runs with a fixed stride over the launch; gr_grid's workspace path
takes them from a work counter), against the oracle.

Integer-valued visibilities and taps keep every partial sum an exact FP32
integer, so the grid must equal the FP64 oracle bit for bit, whatever the
order of the flushes.  Cases: coarsenings with the short side along u and
along v (the factored form forms the product along the shorter side first),
P = 4 and P = 1, the default and rectangular block orders, equal and ragged
chunks, and a stream of more than 2^26 visibilities (the launch is cut into
pieces of 2^26, the kernel's 32-bit offsets), checked on sampled rows against
the C oracle.
"""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import gridding as G  # noqa: E402
from synth import random_point_workload  # noqa: E402

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


def _int_upload(R, wl, rng):
    from paper_1605_07023_amd import binding as B
    S, O = wl.support, wl.oversample
    taps = rng.integers(-1, 2, (wl.n_planes, O, S)) + 1j * rng.integers(-1, 2, (wl.n_planes, O, S))
    wl.vis = (rng.integers(-2, 3, (wl.n_vis, wl.n_pol)) + 1j * rng.integers(-2, 3, (wl.n_vis, wl.n_pol))
              ).astype(np.complex64)
    t = torch.from_numpy(np.ascontiguousarray(np.stack([taps.real, taps.imag], -1), dtype=np.float32)).to(DEV)
    dw = R.upload(wl, DEV, taps=t)
    dw.kernel = B.make_kernel(t, S, O, wl.n_planes, taps_complex=True, w_min=wl.w_min, inv_dw=wl.inv_dw)
    return dw, taps


def _records_grid(R, dw, tune):
    from paper_1605_07023_amd import binding as B
    wl = dw.wl
    rec, wv = R.preprocess(dw)
    g = torch.zeros((wl.n_pol, wl.height, wl.width), dtype=torch.complex64, device=DEV)
    B.gr_grid_records(rec, wv, wl.n_vis, wl.n_pol, dw.kernel, g, wl.height, wl.width, tune)
    torch.cuda.synchronize()
    return g


@pytest.mark.parametrize("P", [4, 1])
@pytest.mark.parametrize("cu,cv,wg_u,wg_v,vpw", [(1, 8, 0, 0, 0), (8, 1, 0, 0, 0), (2, 4, 3, 5, 0),
                                                 (4, 2, 0, 0, 97), (1, 1, 16, 4, 1000), (2, 2, 0, 0, 64)])
def test_grid_records_integer_bit_exact(R, P, cu, cv, wg_u, wg_v, vpw):
    if cu * cv * P > 64:
        pytest.skip("register budget")
    _say(f"gr_grid_records integer: P={P} c={cu}x{cv} tile {wg_u}x{wg_v} chunk {vpw}")
    rng = np.random.default_rng(1000 + 7 * cu + cv + P + vpw)
    S = 16
    wl = random_point_workload(12000, P, 112, 136, S, 8, seed=int(rng.integers(1 << 30)), n_planes=8,
                               margin=3, weights=False, kernel="wsep")
    dw, taps = _int_upload(R, wl, rng)
    g = _records_grid(R, dw, R.tuning(cu, cv, wg_u, wg_v, vpw, variant=1))
    ref, dropped = G.grid_separable(wl.vis, wl.uvw, None, taps, wl.inv_cell_u, wl.inv_cell_v, 8, wl.height,
                                    wl.width, wl.n_planes, wl.w_min, wl.inv_dw)
    assert dropped > 0
    np.testing.assert_array_equal(g.cpu().numpy().astype(np.complex128), ref)


def test_grid_records_tracks_against_gr_grid(R):
    """On an Earth-rotation track set (nearby consecutive visibilities, so most
    64-lane runs lie in one chunk and take the scalar decode), the fixed-stride
    launch of gr_grid_records and the work-counter launch inside gr_grid agree
    within FP32 rounding, and both match the oracle."""
    from synth import full_shape_workload
    wl = full_shape_workload(16, n_baselines=24)
    _say(f"gr_grid_records vs gr_grid on tracks: N={wl.n_vis}")
    dw = R.upload(wl, DEV)
    tune = R.tuning(1, 4, variant=1)
    a = _records_grid(R, dw, tune).cpu().numpy()
    b = R.grid(dw, tune=tune).cpu().numpy()
    assert np.linalg.norm(a - b) / np.linalg.norm(b) <= 1e-6
    taps = G.wkernel_table(wl.support, wl.oversample, wl.plane_w_hat(), wl.support_aa, wl.beta)
    rows = [1900, 2048, 2100]
    from oracle import cgrid
    cgrid.build()
    ref, _ = cgrid.grid_separable(wl.vis, wl.uvw, None, taps, wl.inv_cell_u, wl.inv_cell_v, wl.oversample,
                                  wl.height, wl.width, wl.n_planes, wl.w_min, wl.inv_dw, rows=rows)
    got = a[:, rows].astype(np.complex128)
    assert np.abs(ref).max() > 0
    assert np.linalg.norm(got - ref) / np.linalg.norm(ref) <= 1e-5


def test_grid_records_more_than_2_26_visibilities(R, c_oracle):
    """67,113,864 + 4,000 single-polarisation visibilities on a 4096^2 grid (two
    launch pieces whose footprints overlap everywhere), integer values: sampled
    rows equal the C oracle bit for bit."""
    n = (1 << 26) + 4000
    rng = np.random.default_rng(2026)
    _say(f"gr_grid_records over 2^26: N={n}")
    wl = random_point_workload(n, 1, 4096, 4096, 8, 8, seed=26, n_planes=4, margin=0, weights=False,
                               kernel="wsep")
    dw, taps = _int_upload(R, wl, rng)
    g = _records_grid(R, dw, R.tuning(1, 8, vis_per_wg=1024, variant=1))
    rows = [5, 1234, 2048, 4090]
    got = g[:, rows].cpu().numpy().astype(np.complex128)
    del g, dw
    torch.cuda.empty_cache()
    ref, dropped = c_oracle.grid_separable(wl.vis, wl.uvw, None, taps, wl.inv_cell_u, wl.inv_cell_v, 8,
                                           wl.height, wl.width, wl.n_planes, wl.w_min, wl.inv_dw, rows=rows)
    assert dropped == 0
    assert np.abs(ref).max() > 0
    np.testing.assert_array_equal(got, ref)
