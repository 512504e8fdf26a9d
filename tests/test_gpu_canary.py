"""Guard-band canaries: every gridder writes its grid through a pointer into the
middle of a larger buffer whose margins hold a sentinel, with footprints packed
against all four grid edges (some off the grid and dropped).  After the call
the margins must be untouched (no write past either end of the grid) and the
grid must still match the oracle, so writes past a row end into the next
polarisation plane are caught as well."""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import gridding as G  # noqa: E402
from synth import aterm_taps, random_point_workload  # noqa: E402

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
PAD = 1 << 16                  # floats of margin on each side
SENTINEL = 12345.678


def _say(msg):
    print(msg, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def R():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1605_07023_amd import binding, runner
    binding.load_library()
    return runner


def _guarded_grid(P, H, W):
    buf = torch.full((2 * PAD + P * H * W * 2,), SENTINEL, dtype=torch.float32, device=DEV)
    buf[PAD:PAD + P * H * W * 2] = 0.0
    grid = buf[PAD:PAD + P * H * W * 2].view(torch.complex64).view(P, H, W)
    return buf, grid


def _margins_intact(buf):
    m = torch.cat([buf[:PAD], buf[-PAD:]])
    return bool(torch.all(m == SENTINEL))


def _edge_workload(P, S, kernel, seed, H=96, W=80, n=3000, n_planes=3):
    # points spread a few cells past every edge: footprints touch the borders, some fall off
    return random_point_workload(n, P, H, W, S, 8, seed=seed, n_planes=n_planes if kernel != "kb" else 1,
                                 margin=S // 2 + 3, weights=True, kernel=kernel)


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.mark.parametrize("P,S,variant", [(4, 16, 2), (4, 32, 2), (1, 56, 2), (4, 16, 1), (1, 8, 1)])
def test_separable_gridders_stay_inside(R, P, S, variant):
    _say(f"canaries: separable gridder variant {variant} P={P} S={S}")
    wl = _edge_workload(P, S, "wsep" if S > 8 else "kb", seed=S + P + variant)
    dw = R.upload(wl, DEV)
    buf, grid = _guarded_grid(P, wl.height, wl.width)
    R.grid(dw, grid_out=grid, tune=R.tuning(variant=variant))
    torch.cuda.synchronize()
    assert _margins_intact(buf)
    taps = G.kb_table(S, 8, wl.beta) if wl.kernel == "kb" else \
        G.wkernel_table(S, 8, wl.plane_w_hat(), wl.support_aa, wl.beta)
    ref, dropped = G.grid_separable(wl.vis, wl.uvw, wl.weights, taps, wl.inv_cell_u, wl.inv_cell_v, 8,
                                    wl.height, wl.width, wl.n_planes, wl.w_min, wl.inv_dw)
    assert dropped > 0
    assert _rel(grid.cpu().numpy(), ref) <= 1e-5


@pytest.mark.parametrize("P,S", [(4, 16), (1, 40)])
def test_table2d_gridder_stays_inside(R, P, S):
    _say(f"canaries: 2-D table gridder P={P} S={S}")
    wl = random_point_workload(2500, P, 96, 80, S, 4, seed=S + P, n_planes=3, margin=S // 2 + 3, weights=True,
                               kernel="w2d")
    dw = R.upload(wl, DEV)
    buf, grid = _guarded_grid(P, wl.height, wl.width)
    R.grid(dw, grid_out=grid)
    torch.cuda.synchronize()
    assert _margins_intact(buf)
    t = G.wkernel_2d_table(S, 4, wl.plane_w_hat(), wl.fov, wl.support_aa, wl.beta)
    ref, dropped = G.grid_table2d(wl.vis, wl.uvw, wl.weights, t, wl.inv_cell_u, wl.inv_cell_v, 4, wl.height,
                                  wl.width, 3, wl.w_min, wl.inv_dw)
    assert dropped > 0
    assert _rel(grid.cpu().numpy(), ref) <= 1e-5


def test_aterm_gridder_stays_inside(R):
    from paper_1605_07023_amd import binding as B
    _say("canaries: A-term gridder P=4 S=16")
    P, S, n_ids = 4, 16, 3
    wl = _edge_workload(P, S, "wsep", seed=5)
    ids = np.random.default_rng(5).integers(0, n_ids, wl.n_vis).astype(np.int32)
    taps = aterm_taps(2, n_ids, wl.n_planes, 8, P, S)
    t_dev = torch.from_numpy(np.ascontiguousarray(taps).view(np.float32)).to(DEV)
    dw = R.upload(wl, DEV, taps=t_dev)
    dw.kernel = B.make_kernel(t_dev, S, 8, wl.n_planes, taps_complex=True, w_min=wl.w_min, inv_dw=wl.inv_dw,
                              kind=B.GR_TABLE2D)
    buf, grid = _guarded_grid(P, wl.height, wl.width)
    R.grid_aterm(dw, torch.from_numpy(ids).to(DEV), n_ids, grid_out=grid)
    torch.cuda.synchronize()
    assert _margins_intact(buf)
    ref, dropped = G.grid_aterm(wl.vis, wl.uvw, wl.weights, ids, taps.astype(np.complex128), wl.inv_cell_u,
                                wl.inv_cell_v, 8, wl.height, wl.width, wl.n_planes, wl.w_min, wl.inv_dw)
    assert dropped > 0
    assert _rel(grid.cpu().numpy(), ref) <= 1e-5


def test_batch_gridders_stay_inside(R):
    """A batch of three items with guarded grids, one above 2^19 visibilities (its own wave-form launch)."""
    _say("canaries: batch of 3 items")
    wls = [_edge_workload(4, 16, "wsep", seed=11), _edge_workload(1, 32, "wsep", seed=12),
           _edge_workload(4, 8, "kb", seed=13, n=600000)]
    dws = [R.upload(wl, DEV) for wl in wls]
    guarded = [_guarded_grid(wl.n_pol, wl.height, wl.width) for wl in wls]
    R.grid_batch(dws, grids=[g for _, g in guarded])
    torch.cuda.synchronize()
    for (buf, g), wl in zip(guarded, wls):
        assert _margins_intact(buf), wl.name
        taps = G.kb_table(wl.support, 8, wl.beta) if wl.kernel == "kb" else \
            G.wkernel_table(wl.support, 8, wl.plane_w_hat(), wl.support_aa, wl.beta)
        ref, _ = G.grid_separable(wl.vis, wl.uvw, wl.weights, taps, wl.inv_cell_u, wl.inv_cell_v, 8,
                                  wl.height, wl.width, wl.n_planes, wl.w_min, wl.inv_dw)
        assert _rel(g.cpu().numpy(), ref) <= 1e-5, wl.name
