"""GPU tests of gr_grid_batch (persistent batched launch) through the C ABI.

Bars: every instance of a batch within 1e-5 relative L2 of the FP64 oracle
(FP32 accumulation, as for gr_grid); integer-valued inputs bit-exact (the
work queue neither loses nor repeats a segment); graph replays identical to
the eager result.
"""
import copy
import sys
import time

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import gridding as G  # noqa: E402
from synth import batch_workload, random_point_workload  # noqa: E402

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


def _rel(got, ref):
    return float(np.linalg.norm(got - ref) / max(np.linalg.norm(ref), 1e-300))


def _taps(wl):
    if wl.kernel == "kb":
        return G.kb_table(wl.support, wl.oversample, wl.beta)
    return G.wkernel_table(wl.support, wl.oversample, wl.plane_w_hat(), wl.support_aa, wl.beta)


def _oracle(wl, taps=None):
    return G.grid_separable(wl.vis, wl.uvw, wl.weights, _taps(wl) if taps is None else taps,
                            wl.inv_cell_u, wl.inv_cell_v, wl.oversample, wl.height, wl.width,
                            wl.n_planes, wl.w_min, wl.inv_dw)


def _mixed():
    """Five instances: both polarisation counts, real and complex taps, three
    supports, one empty, ragged sizes, an explicit short segment length."""
    wls = [random_point_workload(1200, 4, 96, 80, 16, 8, seed=1, n_planes=4, margin=4, weights=True,
                                 kernel="wsep"),
           random_point_workload(700, 1, 64, 64, 8, 8, seed=2, margin=3),
           random_point_workload(0, 1, 72, 72, 16, 4, seed=3, n_planes=2, kernel="wsep"),
           random_point_workload(333, 4, 48, 48, 8, 4, seed=4, weights=True),
           random_point_workload(900, 1, 128, 128, 32, 8, seed=5, n_planes=3, margin=6, kernel="wsep")]
    segs = [0, 64, 0, 0, 37]
    return wls, segs


def test_batch_matches_oracle(R):
    _say("batch of 5 mixed instances vs the oracle")
    wls, segs = _mixed()
    dws = [R.upload(wl, DEV) for wl in wls]
    stats = [torch.zeros(2, dtype=torch.int64, device=DEV) for _ in wls]
    grids, _ = R.grid_batch(dws, seg_lens=segs, stats=stats)
    for wl, g, st in zip(wls, grids, stats):
        ref, dropped = _oracle(wl)
        got = g.cpu().numpy()
        if wl.n_vis:
            err = _rel(got, ref)
            _say(f"  {wl.name} P={wl.n_pol} S={wl.support}: rel L2 {err:.2e}, dropped {dropped}")
            assert err <= 1e-5
        else:
            assert not got.any()
        assert st.cpu().tolist() == [wl.n_vis - dropped, dropped]


def _integer_batch(rng):
    wls = []
    for i, (P, S, H, W, n, kern) in enumerate([(1, 8, 64, 64, 3000, "kb"), (4, 16, 48, 56, 1500, "wsep"),
                                               (4, 8, 40, 40, 800, "kb"), (1, 16, 80, 64, 2500, "wsep")]):
        wl = random_point_workload(n, P, H, W, S, 4, seed=20 + i, n_planes=3 if kern == "wsep" else 1,
                                   kernel=kern)
        wl.vis = (rng.integers(-2, 3, (n, P)) + 1j * rng.integers(-2, 3, (n, P))).astype(np.complex64)
        wls.append(wl)
    return wls


def _integer_taps(rng, wl):
    if wl.kernel == "kb":
        t = rng.integers(0, 3, (1, wl.oversample, wl.support)).astype(np.float64)
        return t, t
    t = rng.integers(-1, 2, (3, wl.oversample, wl.support)) + 1j * rng.integers(-1, 2, (3, wl.oversample, wl.support))
    return t, np.stack([t.real, t.imag], axis=-1)


def _upload_with(R, wl, taps_np):
    from paper_1605_07023_amd import binding as B
    taps = torch.from_numpy(np.ascontiguousarray(taps_np, dtype=np.float32)).to(DEV)
    dw = R.upload(wl, DEV, taps=taps)
    dw.kernel = B.make_kernel(taps, wl.support, wl.oversample, wl.n_planes, taps_complex=(taps_np.ndim == 4),
                              w_min=wl.w_min, inv_dw=wl.inv_dw)
    return dw


def test_batch_integer_inputs_bit_exact(R):
    _say("integer-valued batch bit-exact")
    rng = np.random.default_rng(3)
    wls = _integer_batch(rng)
    refs, dws = [], []
    for wl in wls:
        t_or, t_dev = _integer_taps(rng, wl)
        refs.append(_oracle(wl, t_or)[0])
        dws.append(_upload_with(R, wl, t_dev))
    grids, _ = R.grid_batch(dws, seg_lens=[50, 0, 17, 200])
    for g, ref in zip(grids, refs):
        np.testing.assert_array_equal(g.cpu().numpy().astype(np.complex128), ref)


def test_batch_graph_replays(R):
    """The whole batch sequence captured in one HIP graph: each replay (with
    eager work and synchronisation in between) equals the eager result."""
    _say("batch captured in a HIP graph, 3 replays")
    rng = np.random.default_rng(4)
    wls = _integer_batch(rng)
    dws = []
    for wl in wls:
        dws.append(_upload_with(R, wl, _integer_taps(rng, wl)[1]))
    grids, ws = R.grid_batch(dws, seg_lens=[64, 0, 0, 128])
    eager = [g.clone() for g in grids]
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        for g in grids:
            g.zero_()
        R.grid_batch(dws, grids=grids, seg_lens=[64, 0, 0, 128], workspace=ws)
    for rep in range(3):
        for g in grids:
            g.fill_(7.0)
        a = torch.randn(512, 512, device=DEV)
        (a @ a).sum().item()                               # unrelated eager work
        graph.replay()
        torch.cuda.synchronize()
        for g, e in zip(grids, eager):
            assert torch.equal(g, e), f"replay {rep}"


def test_batch_native_graph_replays(R):
    """gr_grid_batch_graph: the library captures the batch into one HIP graph;
    three launches (grids zeroed and unrelated eager work in between) each equal
    the eager result bit for bit."""
    _say("batch captured by the library, 3 graph launches")
    rng = np.random.default_rng(5)
    wls = _integer_batch(rng)
    dws = [_upload_with(R, wl, _integer_taps(rng, wl)[1]) for wl in wls]
    segs = [32, 0, 0, 100]
    eager, _ = R.grid_batch(dws, seg_lens=segs)
    eager = [g.clone() for g in eager]
    grids = [torch.zeros_like(g) for g in eager]
    bg = R.BatchGraph(dws, grids, seg_lens=segs)
    try:
        for rep in range(3):
            for g in grids:
                g.zero_()
            a = torch.randn(256, 256, device=DEV)
            (a @ a).sum().item()
            bg.launch()
            torch.cuda.synchronize()
            for g, e in zip(grids, eager):
                assert torch.equal(g, e), f"launch {rep}"
        # a launch without zeroing accumulates: twice the eager grid, exactly (integers)
        bg.launch()
        torch.cuda.synchronize()
        for g, e in zip(grids, eager):
            assert torch.equal(g, 2 * e)
    finally:
        bg.close()


def test_batch_full_shape_against_single_calls(R):
    """The 32-instance uneven batch (lognormal sizes 1e4..1e6, grids 1024..4096,
    S in {8, 16, 32}, P in {1, 4}): each instance against its own gr_grid call
    (within FP32 reassociation), the three smallest against the oracle."""
    wls = batch_workload(seed=0)
    _say(f"full batch: {len(wls)} instances, {sum(w.n_vis for w in wls)} visibilities")
    dws = [R.upload(wl, DEV) for wl in wls]
    grids, ws = R.grid_batch(dws)
    torch.cuda.synchronize()
    t0 = time.time()
    for g in grids:
        g.zero_()
    R.grid_batch(dws, grids=grids, workspace=ws)
    torch.cuda.synchronize()
    t_batch = time.time() - t0
    t0 = time.time()
    singles = []
    for dw in dws:
        singles.append(R.grid(dw))
    torch.cuda.synchronize()
    t_single = time.time() - t0
    bg = R.BatchGraph(dws, [torch.zeros_like(g) for g in grids])
    try:
        bg.launch()
        torch.cuda.synchronize()
        t0 = time.time()
        for _ in range(3):
            bg.launch()
        torch.cuda.synchronize()
        t_graph = (time.time() - t0) / 3
        for i, (gg, g) in enumerate(zip(bg.grids, grids)):                   # 4 launches accumulated
            r = float(torch.linalg.vector_norm(gg / 4 - g) / torch.linalg.vector_norm(g))
            assert r <= 1e-6, (i, r)
    finally:
        bg.close()
    _say(f"  batch {t_batch * 1e3:.2f} ms, one graph launch {t_graph * 1e3:.2f} ms, "
         f"one call per instance {t_single * 1e3:.2f} ms")
    worst = 0.0
    for wl, g, s in zip(wls, grids, singles):
        a, b = g.cpu().numpy().astype(np.complex128), s.cpu().numpy().astype(np.complex128)
        worst = max(worst, _rel(a, b))
        del a, b
    _say(f"  worst batch/single rel L2 {worst:.2e}")
    assert worst <= 1e-6
    for i in np.argsort([w.n_vis for w in wls])[:3]:
        ref, _ = _oracle(wls[i])
        err = _rel(grids[i].cpu().numpy(), ref)
        _say(f"  {wls[i].name} n={wls[i].n_vis} vs oracle {err:.2e}")
        assert err <= 1e-5


def test_batch_empty_and_all_dropped(R):
    from paper_1605_07023_amd import binding as B
    _say("empty batch, all-dropped instance")
    B.gr_grid_batch([], None, 0)
    wl = random_point_workload(300, 1, 40, 40, 8, 8, seed=9)
    off = copy.copy(wl)
    off.uvw = wl.uvw.copy()
    off.uvw[:, 0] += 1000.0
    dws = [R.upload(wl, DEV), R.upload(off, DEV)]
    stats = [torch.zeros(2, dtype=torch.int64, device=DEV) for _ in dws]
    grids, _ = R.grid_batch(dws, stats=stats)
    assert not grids[1].cpu().numpy().any()
    assert stats[1].cpu().tolist() == [0, 300]
    ref, _ = _oracle(wl)
    assert _rel(grids[0].cpu().numpy(), ref) <= 1e-5


def test_batch_with_autotuned_segment_lengths(R, tmp_path):
    """Per-instance segment lengths from the autotuner (one sweep per instance
    class, remembered in a memo), then one batched call."""
    from paper_1605_07023_amd import autotune
    _say("batch with autotuned segment lengths")
    wls, _ = _mixed()
    dws = [R.upload(wl, DEV) for wl in wls]
    memo = autotune.Memo(str(tmp_path / "memo.json"))
    segs = autotune.batch_seg_lens(dws, memo)
    assert len(segs) == len(wls) and all(s in autotune.SEG_LENS for s in segs)
    assert len(memo.data) == len({(w.n_pol, w.support, w.kernel, max(w.height, w.width)) for w in wls})
    again = autotune.batch_seg_lens(dws, memo)            # served from the memo
    assert again == segs
    grids, _ = R.grid_batch(dws, seg_lens=segs)
    for wl, g in zip(wls, grids):
        if wl.n_vis:
            assert _rel(g.cpu().numpy(), _oracle(wl)[0]) <= 1e-5
