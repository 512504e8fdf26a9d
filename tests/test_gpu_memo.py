"""The library's tuning memo on the GPU: gr_autotune stores its winner, calls
without a tuning read it (gr_grid, gr_grid_workspace_bytes, gr_grid_records,
and gr_grid_binned for the row groups per wave), and the results stay equal to
the oracle's whatever the memo holds."""
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


def _workload(P=4, S=16):
    return random_point_workload(5000, P, 144, 160, S, 8, seed=77 + S, n_planes=6, margin=3, weights=True,
                                 kernel="wsep")


def _ref(wl):
    taps = G.wkernel_table(wl.support, wl.oversample, wl.plane_w_hat(), wl.support_aa, wl.beta)
    return G.grid_separable(wl.vis, wl.uvw, wl.weights, taps, wl.inv_cell_u, wl.inv_cell_v, wl.oversample,
                            wl.height, wl.width, wl.n_planes, wl.w_min, wl.inv_dw)[0]


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def test_autotune_winner_goes_to_the_memo(R):
    """gr_autotune over one VALU and two MFMA candidates: slot 0 holds the
    fastest with its variant made explicit, slot 1 the VALU candidate; a grid
    with no tuning then equals the oracle."""
    from paper_1605_07023_amd import autotune as A, binding as B
    B.gr_tuning_memo_clear()
    wl = _workload()
    dw = R.upload(wl, DEV)
    cands = [B.GrTuning(2, 4, 0, 0, 0, 1), B.GrTuning(0, 0, 0, 4, 512, 2), B.GrTuning(0, 0, 0, 8, 1024, 2)]
    best, times = A.tune(dw, cands, reps=2)
    assert all(np.isfinite(times))
    s0 = B.gr_tuning_memo_get(wl.n_pol, dw.kernel, wl.height, wl.width, 0)
    s1 = B.gr_tuning_memo_get(wl.n_pol, dw.kernel, wl.height, wl.width, 1)
    assert (s0.cu, s0.cv, s0.wg_v, s0.vis_per_wg) == (best.cu, best.cv, best.wg_v, best.vis_per_wg)
    assert s0.variant == (1 if best.variant == 1 else 2)
    assert (s1.cu, s1.cv, s1.variant) == (2, 4, 1)
    _say(f"memo slot 0 after autotune: variant {s0.variant} cu {s0.cu} cv {s0.cv} rg {s0.wg_v} seg {s0.vis_per_wg}")
    g = R.grid(dw).cpu().numpy()
    assert _rel(g, _ref(wl)) <= 1e-5
    B.gr_tuning_memo_clear()


def test_null_tuning_follows_the_memo(R):
    """A VALU-kernel entry in slot 0: gr_grid_workspace_bytes with no tuning gives
    that variant's size, and gr_grid with no tuning and exactly that workspace
    runs it (the binned path would need more) and matches the oracle."""
    from paper_1605_07023_amd import binding as B
    B.gr_tuning_memo_clear()
    wl = _workload()
    dw = R.upload(wl, DEV)
    binned = B.gr_grid_workspace_bytes(wl.n_vis, wl.n_pol, dw.kernel, wl.height, wl.width)
    t1 = B.GrTuning(1, 8, 0, 0, 0, 1)
    valu = B.gr_grid_workspace_bytes(wl.n_vis, wl.n_pol, dw.kernel, wl.height, wl.width, t1)
    assert valu < binned
    B.gr_tuning_memo_put(wl.n_pol, dw.kernel, wl.height, wl.width, 0, t1)
    assert B.gr_grid_workspace_bytes(wl.n_vis, wl.n_pol, dw.kernel, wl.height, wl.width) == valu
    ws = torch.empty(valu, dtype=torch.uint8, device=DEV)
    g = R.grid(dw, workspace=ws).cpu().numpy()
    assert _rel(g, _ref(wl)) <= 1e-5
    B.gr_tuning_memo_clear()


def test_grid_binned_reads_row_groups_from_the_memo(R):
    """gr_grid_binned takes the wave form's row groups per wave from the memo's
    variant-2 entry: a supported count grids as the oracle does, and a count
    with no gridder for the window is refused (so the entry is indeed read)."""
    from paper_1605_07023_amd import binding as B
    B.gr_tuning_memo_clear()
    wl = _workload(S=32)
    dw = R.upload(wl, DEV)
    rec, wv = R.preprocess(dw)
    seg = 1024
    nb = B.gr_bin_bytes(wl.n_vis, wl.n_pol, wl.support, wl.height, wl.width, seg)
    bins = torch.empty(nb, dtype=torch.uint8, device=DEV)
    B.gr_bin(rec, wv, wl.n_vis, wl.n_pol, wl.support, wl.height, wl.width, seg, bins, nb)
    ref = _ref(wl)
    for rg in (2, 4, 6):
        B.gr_tuning_memo_put(wl.n_pol, dw.kernel, wl.height, wl.width, 0, B.GrTuning(0, 0, 0, rg, seg, 2))
        g = torch.zeros((wl.n_pol, wl.height, wl.width), dtype=torch.complex64, device=DEV)
        B.gr_grid_binned(bins, wl.n_vis, wl.n_pol, dw.kernel, seg, g, wl.height, wl.width)
        torch.cuda.synchronize()
        assert _rel(g.cpu().numpy(), ref) <= 1e-5, rg
    B.gr_tuning_memo_put(wl.n_pol, dw.kernel, wl.height, wl.width, 0, B.GrTuning(0, 0, 0, 5, seg, 2))
    g = torch.zeros((wl.n_pol, wl.height, wl.width), dtype=torch.complex64, device=DEV)
    with pytest.raises(B.GridderError) as e:
        B.gr_grid_binned(bins, wl.n_vis, wl.n_pol, dw.kernel, seg, g, wl.height, wl.width)
    assert e.value.status == B.GR_EUNSUPPORTED and "row groups" in str(e.value)
    B.gr_tuning_memo_clear()
