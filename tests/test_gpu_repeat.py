"""Repeat runs: the gridders add their windows with FP32 atomics, so two runs on
the same input may differ only by the order of those additions (within 1e-6
relative L2); degridding and compression use no atomics on their outputs and
must repeat bit for bit."""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from synth import compression_workload, full_shape_workload  # noqa: E402

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


@pytest.mark.parametrize("S", [16, 32])
def test_gridding_repeats_within_reassociation(R, S):
    _say(f"repeat gridding S={S}")
    wl = full_shape_workload(S, n_baselines=64)
    dw = R.upload(wl, DEV)
    a = R.grid(dw).cpu().numpy().astype(np.complex128)
    b = R.grid(dw).cpu().numpy().astype(np.complex128)
    d = float(np.linalg.norm(a - b) / np.linalg.norm(a))
    _say(f"  rel L2 between runs {d:.2e}")
    assert d <= 1e-6


def test_degridding_repeats_bit_for_bit(R):
    from paper_1605_07023_amd import binding as B
    _say("repeat degridding S=32")
    wl = full_shape_workload(32, n_baselines=64)
    dw = R.upload(wl, DEV)
    g = torch.randn((wl.n_pol, wl.height, wl.width), dtype=torch.complex64, device=DEV,
                    generator=torch.Generator(device=DEV).manual_seed(3))
    need = B.gr_degrid_workspace_bytes(wl.n_vis, wl.n_pol, 32, wl.height, wl.width, 0)
    ws = torch.empty(need, dtype=torch.uint8, device=DEV)
    outs = []
    for _ in range(2):
        out = torch.empty((wl.n_vis, wl.n_pol), dtype=torch.complex64, device=DEV)
        B.gr_degrid(dw.uvw, wl.n_vis, wl.n_pol, dw.kernel, wl.inv_cell_u, wl.inv_cell_v, g, wl.height, wl.width,
                    out, 0, ws, need)
        outs.append(out)
    torch.cuda.synchronize()
    assert torch.equal(outs[0].view(torch.float32), outs[1].view(torch.float32))


def test_compression_repeats_bit_for_bit(R):
    from paper_1605_07023_amd import binding as B
    _say("repeat compression")
    wl = compression_workload(n_baselines=200, n_pol=4, grid=1024, support=16, n_planes=8)
    dw = R.upload(wl, DEV)
    rec, wv = R.preprocess(dw)
    n = wl.n_vis
    nw = B.gr_compress_workspace_bytes(n)
    ws = torch.empty(nw, dtype=torch.uint8, device=DEV)
    res = []
    for _ in range(2):
        orec, owv = torch.empty_like(rec), torch.empty_like(wv)
        cnt = torch.zeros(1, dtype=torch.int64, device=DEV)
        B.gr_compress(rec, wv, n, 4, orec, owv, cnt, ws, nw)
        res.append((orec, owv, cnt))
    torch.cuda.synchronize()
    assert torch.equal(res[0][2], res[1][2])
    assert torch.equal(res[0][0], res[1][0])             # the padding records too (all invalid)
    m = int(res[0][2].item())                            # the summed values of the m runs; slots after them
    assert torch.equal(res[0][1][:m].view(torch.float32), res[1][1][:m].view(torch.float32))   # are unspecified
