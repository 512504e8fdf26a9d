"""gr_grid_noalloc, the entry point for callers that cannot allocate device
memory: its grid equals gr_grid's on the same inputs, on two calls in a row
(the second smaller, on the static scratch the first one left behind), in the
default binned path and in the VALU path, and a call that needs more scratch
than the static array holds is refused before anything is enqueued.  Runs on
the GPU through the C ABI (ctypes)."""
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


def _noalloc(dw, tune=None, g=None):
    from paper_1605_07023_amd import binding as B
    wl = dw.wl
    if g is None:
        g = torch.zeros((wl.n_pol, wl.height, wl.width), dtype=torch.complex64, device=DEV)
    stats = torch.zeros(2, dtype=torch.int64, device=DEV)
    B.gr_grid_noalloc(dw.uvw, dw.vis, dw.vis_dtype, dw.vis_scale, dw.weights, wl.n_vis, wl.n_pol, dw.kernel,
                      wl.inv_cell_u, wl.inv_cell_v, g, wl.height, wl.width, tune, stats)
    return g, stats


def _with_workspace(R, dw, tune=None):
    stats = torch.zeros(2, dtype=torch.int64, device=DEV)
    g = R.grid(dw, tune=tune, stats=stats)
    return g, stats


def _rel_l2(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def _int_upload(R, wl, rng):
    from paper_1605_07023_amd import binding as B
    S, O = wl.support, wl.oversample
    taps = (rng.integers(-1, 2, (wl.n_planes, O, S)) + 1j * rng.integers(-1, 2, (wl.n_planes, O, S)))
    wl.vis = (rng.integers(-2, 3, (wl.n_vis, wl.n_pol)) + 1j * rng.integers(-2, 3, (wl.n_vis, wl.n_pol))
              ).astype(np.complex64)
    t = torch.from_numpy(np.ascontiguousarray(np.stack([taps.real, taps.imag], -1), dtype=np.float32)).to(DEV)
    dw = R.upload(wl, DEV, taps=t)
    dw.kernel = B.make_kernel(t, S, O, wl.n_planes, taps_complex=True, w_min=wl.w_min, inv_dw=wl.inv_dw)
    return dw, taps


def test_noalloc_equals_gr_grid_two_calls(R):
    """Full-shape geometry on the first 20 baselines (327,680 quad-pol
    visibilities, 4096^2, S = 32), then a smaller scattered set on 300 x 260
    cells (S = 16): each gr_grid_noalloc grid within 1e-5 of gr_grid's, with the
    same statistics; the second also against the FP64 oracle."""
    from paper_1605_07023_amd import binding as B
    cap = B.gr_grid_noalloc_scratch_bytes()
    big = full_shape_workload(32, n_baselines=20)
    small = random_point_workload(6000, 4, 300, 260, 16, 8, seed=77, n_planes=9, margin=3, weights=True,
                                  kernel="wsep")
    for wl in (big, small):
        _say(f"noalloc vs gr_grid: N={wl.n_vis} P={wl.n_pol} S={wl.support} grid {wl.height}x{wl.width}")
        dw = R.upload(wl, DEV)
        need = B.gr_grid_workspace_bytes(wl.n_vis, wl.n_pol, dw.kernel, wl.height, wl.width)
        assert 0 < need <= cap, (need, cap)
        g1, s1 = _noalloc(dw)
        g0, s0 = _with_workspace(R, dw)
        torch.cuda.synchronize()
        a, b = g1.cpu().numpy(), g0.cpu().numpy()
        assert s1.cpu().tolist() == s0.cpu().tolist()
        assert np.abs(b).max() > 0
        assert _rel_l2(a, b) <= 1e-5
        if wl is small:
            taps = G.wkernel_table(wl.support, wl.oversample, wl.plane_w_hat(), wl.support_aa, wl.beta)
            ref, dropped = G.grid_separable(wl.vis, wl.uvw, wl.weights, taps, wl.inv_cell_u, wl.inv_cell_v,
                                            wl.oversample, wl.height, wl.width, wl.n_planes, wl.w_min, wl.inv_dw)
            assert s1.cpu().tolist() == [wl.n_vis - dropped, dropped] and dropped > 0
            assert _rel_l2(a.astype(np.complex128), ref) <= 1e-5


@pytest.mark.parametrize("variant", [0, 1])
def test_noalloc_integer_bit_exact_two_calls(R, variant):
    """Integer-valued visibilities and taps: every partial sum is exact, so
    gr_grid_noalloc, gr_grid and the oracle agree bit for bit, for a larger
    then a smaller call (binned path, and the VALU path with variant 1)."""
    from paper_1605_07023_amd import binding as B
    rng = np.random.default_rng(910 + variant)
    tune = R.tuning(variant=1) if variant == 1 else None
    for n, side, S in [(40000, 400, 32), (3000, 96, 16)]:
        _say(f"noalloc integer: variant={variant} N={n} grid {side}^2 S={S}")
        wl = random_point_workload(n, 4, side, side, S, 8, seed=int(rng.integers(1 << 30)), n_planes=16,
                                   margin=2, weights=False, kernel="wsep")
        dw, taps = _int_upload(R, wl, rng)
        g1, s1 = _noalloc(dw, tune)
        g0, s0 = _with_workspace(R, dw, tune)
        torch.cuda.synchronize()
        ref, dropped = G.grid_separable(wl.vis, wl.uvw, None, taps, wl.inv_cell_u, wl.inv_cell_v, 8, side, side,
                                        16, wl.w_min, wl.inv_dw)
        assert s1.cpu().tolist() == s0.cpu().tolist() == [n - dropped, dropped]
        np.testing.assert_array_equal(g1.cpu().numpy(), g0.cpu().numpy())
        np.testing.assert_array_equal(g1.cpu().numpy().astype(np.complex128), ref)


def test_noalloc_refuses_more_than_its_scratch(R):
    """A call needing more scratch than the static array is refused with
    GR_ENOMEM, and nothing is enqueued (the grid stays zero)."""
    from paper_1605_07023_amd import binding as B
    wl = full_shape_workload(32, n_baselines=96)
    dw = R.upload(wl, DEV)
    need = B.gr_grid_workspace_bytes(wl.n_vis, wl.n_pol, dw.kernel, wl.height, wl.width)
    assert need > B.gr_grid_noalloc_scratch_bytes()
    g = torch.zeros((wl.n_pol, wl.height, wl.width), dtype=torch.complex64, device=DEV)
    with pytest.raises(B.GridderError) as e:
        _noalloc(dw, g=g)
    assert e.value.status == B.GR_ENOMEM and "scratch" in str(e.value)
    torch.cuda.synchronize()
    assert float(g.abs().max()) == 0.0
