"""Reduced precision: FP16 / BF16 taps and scaled-FP16 visibilities, FP32
accumulation, against the FP64 oracle.

Two errors are reported per case:
  * accuracy: against the oracle with exact FP64 taps and the original
    complex64 visibilities (the bound is 1e-3 relative L2 for FP16 taps);
  * parity: against the oracle fed the same rounded taps (FP64 -> FP32 ->
    FP16/BF16, the GPU generator's conversion) and the dequantised
    visibilities, which isolates the FP32 accumulation (bound 1e-5).
"""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import gridding as G  # noqa: E402
from synth import (dequantize_vis_f16, full_shape_workload, quantize_vis_f16,  # noqa: E402
                   random_point_workload, tiny_kb_workload)

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
ACCURACY_BOUND = {"f16": 1e-3, "bf16": 5e-3}


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
    return float(np.linalg.norm(got - ref) / np.linalg.norm(ref))


def _taps64(wl):
    if wl.kernel == "kb":
        return G.kb_table(wl.support, wl.oversample, wl.beta)
    return G.wkernel_table(wl.support, wl.oversample, wl.plane_w_hat(), wl.support_aa, wl.beta)


def _round_like_gpu(taps64, kind):
    """FP64 -> FP32 -> FP16 / BF16 -> FP64 (oracle side, with torch CPU casts)."""
    t = torch.from_numpy(np.ascontiguousarray(taps64.real if not np.iscomplexobj(taps64) else
                                              np.stack([taps64.real, taps64.imag], -1)))
    t = t.to(torch.float32).to(torch.float16 if kind == "f16" else torch.bfloat16).to(torch.float64)
    t = t.numpy()
    return t if not np.iscomplexobj(taps64) else t[..., 0] + 1j * t[..., 1]


def _oracle(wl, taps, vis, rows=None, c_oracle=None):
    if rows is None:
        g, _ = G.grid_separable(vis, wl.uvw, wl.weights, taps, wl.inv_cell_u, wl.inv_cell_v,
                                wl.oversample, wl.height, wl.width, wl.n_planes, wl.w_min, wl.inv_dw)
        return g
    g, _ = c_oracle.grid_separable(vis, wl.uvw, wl.weights, taps, wl.inv_cell_u, wl.inv_cell_v,
                                   wl.oversample, wl.height, wl.width, wl.n_planes, wl.w_min,
                                   wl.inv_dw, rows=rows)
    return g


def _run(R, wl, kind, vis16, variant):
    from paper_1605_07023_amd import binding as B
    dt = B.GR_F16 if kind == "f16" else B.GR_BF16
    enc = quantize_vis_f16(wl.vis) if vis16 else None
    dw = R.upload(wl, DEV, tap_dtype=dt, vis_f16=enc)
    g = R.grid(dw, tune=R.tuning(variant=variant))
    torch.cuda.synchronize()
    return g, enc


@pytest.mark.parametrize("kind", ["f16", "bf16"])
@pytest.mark.parametrize("vis16", [False, True])
@pytest.mark.parametrize("variant", [1, 2])
def test_points_reduced_precision(R, kind, vis16, variant):
    wl = random_point_workload(3000, 4, 96, 80, 16, 8, seed=4, n_planes=7, margin=3,
                               weights=False, kernel="wsep")
    _say(f"reduced precision points: taps {kind}, fp16 vis {vis16}, variant {variant}")
    g, enc = _run(R, wl, kind, vis16, variant)
    got = g.cpu().numpy().astype(np.complex128)
    t64 = _taps64(wl)
    acc = _rel_l2(got, _oracle(wl, t64, wl.vis))
    vis_used = dequantize_vis_f16(*enc) if vis16 else wl.vis
    par = _rel_l2(got, _oracle(wl, _round_like_gpu(t64, kind), vis_used))
    _say(f"    accuracy {acc:.3e}  parity {par:.3e}")
    assert par <= 1e-5
    assert acc <= ACCURACY_BOUND[kind]


@pytest.mark.parametrize("kind", ["f16", "bf16"])
def test_tiny_config_reduced_precision(R, kind):
    wl = tiny_kb_workload()
    _say(f"reduced precision tiny KB config: taps {kind}, fp16 vis")
    g, enc = _run(R, wl, kind, True, 2)
    got = g.cpu().numpy().astype(np.complex128)
    t64 = _taps64(wl)
    acc = _rel_l2(got, _oracle(wl, t64, wl.vis))
    par = _rel_l2(got, _oracle(wl, _round_like_gpu(t64, kind), dequantize_vis_f16(*enc)))
    _say(f"    accuracy {acc:.3e}  parity {par:.3e}")
    assert par <= 1e-5 and acc <= ACCURACY_BOUND[kind]


@pytest.mark.parametrize("S", [16, 32])
@pytest.mark.parametrize("kind", ["f16", "bf16"])
def test_full_shape_reduced_precision(R, c_oracle, S, kind):
    """The full 33M-visibility quad-pol 4096^2 workload with FP16/BF16 taps and
    scaled-FP16 visibilities, default launch; accuracy on sampled rows."""
    wl = full_shape_workload(S)
    _say(f"full shape reduced precision S={S} taps {kind}")
    g, enc = _run(R, wl, kind, True, 0)
    rows = [300, 1500, 2047, 2600, 3800]
    got = g[:, rows].cpu().numpy().astype(np.complex128)
    del g
    torch.cuda.empty_cache()
    t64 = _taps64(wl)
    acc = _rel_l2(got, _oracle(wl, t64, wl.vis, rows, c_oracle))
    _say(f"    S={S} {kind}: sampled-row accuracy {acc:.3e}")
    assert acc <= ACCURACY_BOUND[kind]
