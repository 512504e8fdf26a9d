"""Reduced precision: FP16 / BF16 taps and scaled-FP16 visibilities, FP32
accumulation, against the FP64 oracle.

Two errors are reported per case:
  * accuracy: against the oracle with exact FP64 taps and the original
    complex64 visibilities, bound 1e-3 relative L2 for both tap types.  FP16
    taps meet it.  BF16 taps (8-bit significand, unit roundoff 2^-9) do not:
    the product of two rounded separable taps carries a relative error of
    about 1.6e-3 per tap, and the grids measure 1.6e-3 (KB, tiny config) to
    2.9e-3 (W kernels).  Those cases are strict expected failures that raise
    AccuracyAboveBound, so a parity failure still fails the test and a BF16
    result that met the bound would be reported;
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
ACCURACY_BOUND = 1e-3


class AccuracyAboveBound(Exception):
    """Relative L2 against the exact-tap oracle above ACCURACY_BOUND."""


def _check_accuracy(acc):
    if acc > ACCURACY_BOUND:
        raise AccuracyAboveBound(f"relative L2 {acc:.3e} > {ACCURACY_BOUND:.0e}")


def _bf16(measured):
    return pytest.param("bf16", marks=pytest.mark.xfail(
        strict=True, raises=AccuracyAboveBound,
        reason=f"BF16 taps measure {measured} relative L2, above the 1e-3 bound"))


KINDS_POINTS = ["f16", _bf16("2.46e-3 to 2.47e-3")]
KINDS_TINY = ["f16", _bf16("1.65e-3")]
KINDS_FULL = ["f16", _bf16("2.84e-3 to 2.85e-3")]


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


@pytest.mark.parametrize("kind", KINDS_POINTS)
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
    _check_accuracy(acc)


@pytest.mark.parametrize("kind", KINDS_TINY)
def test_tiny_config_reduced_precision(R, kind):
    wl = tiny_kb_workload()
    _say(f"reduced precision tiny KB config: taps {kind}, fp16 vis")
    g, enc = _run(R, wl, kind, True, 2)
    got = g.cpu().numpy().astype(np.complex128)
    t64 = _taps64(wl)
    acc = _rel_l2(got, _oracle(wl, t64, wl.vis))
    par = _rel_l2(got, _oracle(wl, _round_like_gpu(t64, kind), dequantize_vis_f16(*enc)))
    _say(f"    accuracy {acc:.3e}  parity {par:.3e}")
    assert par <= 1e-5
    _check_accuracy(acc)


@pytest.mark.parametrize("S", [16, 32])
@pytest.mark.parametrize("kind", KINDS_FULL)
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
    _check_accuracy(acc)
