#!/usr/bin/env python3
"""Benchmark: convolutional gridding throughput on one MI355X.

Workload: 64 antennas (2016 baselines) x 1024 dumps over 8 h x 16 channels
(33,030,144 visibilities, ordered baseline / time / channel), four
polarisations, 4096^2 complex64 grid per polarisation, separable complex W
kernels with 32 planes and oversampling 8, supports 16 and 32.

One step = the whole hot path over that batch for both supports: preprocess
(FP64 index conversion, weighting) and gridding, S = 16 then S = 32, each into
its own grid.  Inputs and kernel tables are resident in HBM before timing.

value = useful vis-tap updates per second over the step (a vis-tap update is
one polarisation of one visibility times one in-footprint tap: 8 flops with
complex taps; padding taps are not counted).

Prints one JSON line.  Progress goes to stderr.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import tempfile
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

FP32_VALU_PEAK = 157.3e12   # MI355X FP32 vector peak (packed), flop/s
FP32_VALU_NONPACKED = 78.6e12   # the same without packed FP32 (every HIP file here is built without it)
FP32_MFMA_PEAK = 157.3e12   # MI355X dense FP32 matrix peak, flop/s
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic.json")
KERNEL_SOURCES = {1: [os.path.join(ROOT, "paper_1605_07023_amd", "csrc", "grid_romein.hip")],
                  2: [os.path.join(ROOT, "paper_1605_07023_amd", "csrc", "grid_mfma.hip")]}


def log(msg: str) -> None:
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def source_hash(variant: int) -> str:
    """sha256[:16] over the kernel's source and the hipcc flags it is compiled with."""
    from paper_1605_07023_amd.build import HIPCC_FLAGS, SOURCE_FLAGS
    h = hashlib.sha256()
    for f in KERNEL_SOURCES[variant]:
        with open(f, "rb") as fh:
            h.update(fh.read())
        h.update(" ".join(HIPCC_FLAGS + SOURCE_FLAGS.get(os.path.basename(f), [])).encode())
    return h.hexdigest()[:16]


def cpu_baseline(wl_fn, support: int, budget_s: float, threads: int) -> dict:
    """The FP64 C oracle, as it stands, on a bounded sample of the workload:
    the first k baselines (all dumps and channels), k sized for ~budget_s."""
    import numpy as np
    from oracle import cgrid
    from oracle import gridding as G
    cgrid.build()
    cgrid.set_threads(threads)
    per_bl = 1024 * 16

    def run(k):
        wl = wl_fn(support, n_baselines=k)
        taps = G.wkernel_table(support, 8, wl.plane_w_hat(), wl.support_aa, wl.beta)
        t0 = time.perf_counter()
        _, dropped = cgrid.grid_separable(wl.vis, wl.uvw, None, taps, wl.inv_cell_u, wl.inv_cell_v,
                                          8, wl.height, wl.width, wl.n_planes, wl.w_min, wl.inv_dw)
        dt = time.perf_counter() - t0
        return (wl.n_vis - dropped) * wl.n_pol * support * support, dt

    upd, dt = run(32)
    k = int(max(32, min(2016, 32 * budget_s / max(dt, 1e-3))))
    log(f"cpu baseline: calibration 32 baselines {dt:.2f}s -> sample {k} baselines")
    upd, dt = run(k)
    single_per_bl = dt * threads / k                   # seconds per baseline on one thread, roughly
    # the same oracle on one thread, over a sample of about 3 s
    k1 = int(max(1, min(32, 3.0 / max(single_per_bl, 1e-3))))
    cgrid.set_threads(1)
    upd1, dt1 = run(k1)
    cgrid.set_threads(threads)
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            model = next((ln.split(":", 1)[1].strip() for ln in f if ln.startswith("model name")), model)
    except OSError:
        pass
    return {"value": upd / dt, "unit": "updates/s", "cores": threads, "kind": "oracle",
            "sample": f"first {k} of 2016 baselines x 1024 dumps x 16 channels "
                      f"({k * per_bl} vis, S={support}, quad pol, 4096^2), C FP64 oracle, {dt:.1f} s",
            "single_thread": {"value": upd1 / dt1, "unit": "updates/s",
                              "sample": f"first {k1} baselines ({k1 * per_bl} vis, S={support}), {dt1:.1f} s"},
            "host": {"cpu_model": model, "logical_cpus": os.cpu_count()}}


def learned_leg(dev, uvw, vis, wl_plain, rec, wvis, bins, bins_bytes, seg_len, stream, steps: int,
                reps: int) -> dict:
    """The learned tap network against the exact 2-D W-kernel table it is trained
    on, on the full-shape visibilities (support 32, 64 planes, oversampling 8:
    a 33.5 MB table).  Training, the tap fit on the table and both gridding
    paths are measured on the device; errors against the exact continuous
    kernel are measured by the gain test, which needs the FP64 reference."""
    import dataclasses
    import torch
    from paper_1605_07023_amd import binding as B
    from paper_1605_07023_amd import tapnet as T
    from synth import learned_kernel_workload
    wl = learned_kernel_workload()
    if wl.n_vis != wl_plain.n_vis or not (wl.uvw[:1000] == wl_plain.uvw[:1000]).all():
        raise RuntimeError("learned-kernel workload does not share the plain workload's visibilities")
    S, O, planes = wl.support, wl.oversample, wl.n_planes
    N, P = wl.n_vis, wl.n_pol
    wh = wl.plane_w_hat()
    w_rng = 2 * float(abs(wh).max())
    table = torch.empty((planes, O, O, S, S, 2), dtype=torch.float32, device=dev)
    B.gr_make_wkernel2d_table(S, O, planes, float(wh[0]), float(wh[1] - wh[0]), wl.fov, wl.support_aa,
                              wl.beta, 0, B.GR_F32, table, stream)
    scale = float(torch.view_as_complex(table).abs().max().item())
    x, t = T.dataset_from_table(table, S, O, wh, w_rng, scale, stream)
    net = T.TapNet(dev, seed=0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    tlog = net.train(x, t, steps, batch=16384, lr=2e-3, lr_final=2e-5, log_every=max(steps // 4, 1))
    torch.cuda.synchronize()
    train_s = time.perf_counter() - t0
    net.set_header(0.0, 0.0, scale)
    y = torch.view_as_complex(net.eval(x).contiguous())
    tv = torch.view_as_complex(table.view(-1, 2))
    fit = float(torch.linalg.norm(y - tv) / torch.linalg.norm(tv))
    del x, t, y
    n_fine, o_fine = 16384, 128
    wmf, invf = T.fine_planes(wl.w_min, wl.inv_dw, planes, n_fine)
    off, stp = T.header_for_planes(wmf, invf, wl.w_hat_scale, w_rng)
    net.set_header(off, stp, scale)
    k_tab = B.make_kernel(table, S, O, planes, True, B.GR_F32, wl.w_min, wl.inv_dw, kind=B.GR_TABLE2D)
    k_mlp = net.kernel(S, o_fine, n_fine, wmf, invf)
    out = {}
    grids = {}
    stats = torch.zeros(2, dtype=torch.int64, device=dev)
    for name, k in (("table", k_tab), ("network", k_mlp)):
        g = torch.zeros((P, wl.height, wl.width), dtype=torch.complex64, device=dev)
        times = []
        for r in range(reps + 1):
            g.zero_()
            stats.zero_()
            B.gr_preprocess(uvw, vis, B.GR_F32, None, None, N, P, k, wl.inv_cell_u, wl.inv_cell_v,
                            wl.height, wl.width, rec, wvis, stats, stream)
            B.gr_bin(rec, wvis, N, P, S, wl.height, wl.width, seg_len, bins, bins_bytes, stream)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            B.gr_grid_binned(bins, N, P, k, seg_len, g, wl.height, wl.width, stream)
            e1.record(stream)
            torch.cuda.synchronize()
            if r > 0:
                times.append(e0.elapsed_time(e1) * 1e-3)
        n_valid = int(stats[0].item())
        sec = sum(times) / len(times)
        out[f"{name}_path_grid_kernel_ms"] = sec * 1e3
        out[f"{name}_path_updates_per_s"] = n_valid * P * S * S / sec
        grids[name] = g
        log(f"learned-kernel leg: {name} path {sec * 1e3:.1f} ms")
    # the smallest nearest-entry table whose tap error matches the network's: at continuous w and
    # offsets the network (12,000 steps) measures 7.8e-3 against the exact kernel, the 64 x O 8
    # table 3.0e-2 and a 256-plane, O = 32 table 7.2e-3 (tests/test_gpu_mlp.py); that table is
    # 2.1 GB, generated on the device and gridded by the same 2-D table gridder
    mp, mo = 256, 32
    t_gen0 = time.perf_counter()
    big = torch.empty((mp, mo, mo, S, S, 2), dtype=torch.float32, device=dev)
    B.gr_make_wkernel2d_table(S, mo, mp, float(wh[0]), float(wh[-1] - wh[0]) / (mp - 1), wl.fov, wl.support_aa,
                              wl.beta, 0, B.GR_F32, big, stream)
    torch.cuda.synchronize()
    gen_s = time.perf_counter() - t_gen0
    k_big = B.make_kernel(big, S, mo, mp, True, B.GR_F32, wl.w_min, wl.inv_dw * (mp - 1) / (planes - 1),
                          kind=B.GR_TABLE2D)
    g = torch.zeros((P, wl.height, wl.width), dtype=torch.complex64, device=dev)
    stats.zero_()
    B.gr_preprocess(uvw, vis, B.GR_F32, None, None, N, P, k_big, wl.inv_cell_u, wl.inv_cell_v,
                    wl.height, wl.width, rec, wvis, stats, stream)
    B.gr_bin(rec, wvis, N, P, S, wl.height, wl.width, seg_len, bins, bins_bytes, stream)
    t_big = _timed(stream, lambda: B.gr_grid_binned(bins, N, P, k_big, seg_len, g, wl.height, wl.width, stream),
                   reps) * 1e-3
    n_valid = int(stats[0].item())
    out.update({"matched_table_planes": mp, "matched_table_oversample": mo,
                "matched_table_bytes": big.numel() * 4, "matched_table_generation_s": gen_s,
                "matched_table_grid_kernel_ms": t_big * 1e3,
                "matched_table_updates_per_s": n_valid * P * S * S / t_big})
    log(f"learned-kernel leg: matched-error table ({mp} planes x O {mo}, {big.numel() * 4 / 1e9:.2f} GB) "
        f"{t_big * 1e3:.1f} ms")
    del big, g
    diff = float(torch.linalg.norm(grids["network"] - grids["table"]) / torch.linalg.norm(grids["table"]))
    out.update({
        "workload": "the plain full-shape visibilities with the exact 2-D W kernel, S=32, fov 0.5 "
                    "direction cosines, w_hat in [-24, 24]: table of 64 planes x 8 x 8 phases (reference) vs "
                    f"network evaluated at {n_fine} planes x {o_fine} x {o_fine} phases",
        "table_bytes": table.numel() * 4, "network_bytes": net.blob.numel() * 4,
        "train_steps": steps, "train_batch": 16384, "train_s": train_s,
        "train_loss": [round(v, 8) for v in tlog.losses],
        "tap_rel_l2_on_table": fit,
        "network_vs_table_grid_rel_l2": diff,
        "error_vs_exact_kernel": "tests/test_gpu_mlp.py::test_learned_kernel_gain (FP64 continuous-kernel grid)",
    })
    del grids, table
    return out


def compression_leg(dev, stream, reps: int) -> dict:
    """Compression (adjacent visibilities on the same oversampled cell and w plane
    summed, as the paper's preprocess does) on the stand-in for the paper's data
    set: 2016 baselines x 3600 dumps of 2 s, one channel, quad pol, 2048^2 grid,
    S=16 W kernel, 32 planes.  Times gr_compress and the binned gridding (gr_bin +
    gr_grid_binned) of the stream before and after compression; the paper quotes
    its rates on compressed visibilities."""
    import torch
    from paper_1605_07023_amd import binding as B, runner
    from synth import compression_workload
    wl = compression_workload()
    N, P, S = wl.n_vis, wl.n_pol, wl.support
    dw = runner.upload(wl, dev)
    rec = torch.empty((N, 2), dtype=torch.int32, device=dev)
    wv = torch.empty((N, P), dtype=torch.complex64, device=dev)
    B.gr_preprocess(dw.uvw, dw.vis, B.GR_F32, None, None, N, P, dw.kernel, wl.inv_cell_u, wl.inv_cell_v,
                    wl.height, wl.width, rec, wv, None, stream)
    crec, cwv = torch.empty_like(rec), torch.empty_like(wv)
    cnt = torch.zeros(1, dtype=torch.int64, device=dev)
    nw = B.gr_compress_workspace_bytes(N)
    cws = torch.empty(nw, dtype=torch.uint8, device=dev)
    nb = B.gr_bin_bytes(N, P, S, wl.height, wl.width, 0)
    bins = torch.empty(nb, dtype=torch.uint8, device=dev)
    g = torch.zeros((P, wl.height, wl.width), dtype=torch.complex64, device=dev)

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        ms = []
        for _ in range(reps):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(stream)
            fn()
            b.record(stream)
            torch.cuda.synchronize()
            ms.append(a.elapsed_time(b))
        return sorted(ms)[len(ms) // 2]

    t_comp = timed(lambda: B.gr_compress(rec, wv, N, P, crec, cwv, cnt, cws, nw, stream))
    m = int(cnt.item())

    def grid_of(r, v):
        B.gr_bin(r, v, N, P, S, wl.height, wl.width, 0, bins, nb, stream)
        B.gr_grid_binned(bins, N, P, dw.kernel, 0, g, wl.height, wl.width, stream)

    t_full = timed(lambda: grid_of(rec, wv))
    t_comp_grid = timed(lambda: grid_of(crec, cwv))
    log(f"compression leg: {N} -> {m} visibilities, bin+grid {t_full:.2f} -> {t_comp_grid:.2f} ms")
    del bins, g, rec, wv, crec, cwv
    return {"workload": "2016 baselines x 3600 dumps of 2 s over 2 h, 1 channel at 1.4 GHz, quad pol, 2048^2, "
                        "separable W kernel S=16, 32 planes, oversampling 8 (stand-in for the paper's data set)",
            "n_vis": N, "n_compressed": m, "ratio": N / m, "compress_ms": t_comp,
            "bin_grid_ms_uncompressed": t_full, "bin_grid_ms_compressed": t_comp_grid,
            "updates_per_s_uncompressed": N * P * S * S / (t_full * 1e-3),
            "compressed_updates_per_s": m * P * S * S / (t_comp_grid * 1e-3),
            "input_updates_per_s_via_compression": N * P * S * S / (t_comp_grid * 1e-3)}


def wstack_leg(dev, stream, reps: int) -> dict:
    """W-stacking (Section 5: the stream split by w into 7 slices, each gridded as
    its own problem with a GCF for the w offset from the slice's centre) on the
    2 h, 2 s-dump tracks: gr_wslice_partition of the whole stream, then the 7
    slices gridded by one gr_grid_batch (persistent work list over every slice)
    and, as the paper launches them, by one gr_grid per slice; S=16 and S=32,
    32 residual planes per slice, 2048^2 grids.  HIP events on the stream, median
    of ``reps`` after one untimed call."""
    import torch
    from paper_1605_07023_amd import binding as B, runner
    from synth import wstack_workload

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        ms = []
        for _ in range(reps):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(stream)
            fn()
            b.record(stream)
            torch.cuda.synchronize()
            ms.append(a.elapsed_time(b))
        return sorted(ms)[len(ms) // 2]

    out = {"workload": "2016 baselines x 3600 dumps of 2 s over 2 h, 1 channel at 1.4 GHz, quad pol, "
                       "7 equal w slices over [-max|w|, max|w|], 2048^2 grid per slice, separable W kernel "
                       "of 32 planes over the slice width, oversampling 8", "per_support": {}}
    for S in (16, 32):
        wl = wstack_workload(n_pol=4, grid=2048, support=S)
        m = wl.meta
        N, P, n_sl = wl.n_vis, wl.n_pol, m["n_slices"]
        dw = runner.upload(wl, dev)
        uvw_p, vis_p = torch.empty_like(dw.uvw), torch.empty_like(dw.vis)
        offs = torch.empty(n_sl + 1, dtype=torch.int64, device=dev)
        nw = B.gr_wslice_partition_workspace_bytes(N, n_sl)
        pws = torch.empty(nw, dtype=torch.uint8, device=dev)

        def part():
            B.gr_wslice_partition(dw.uvw, dw.vis, None, N, P, m["w_first"], m["inv_width"], n_sl, uvw_p, vis_p,
                                  None, offs, pws, nw, stream)

        t_part = timed(part)
        off = offs.cpu().numpy()
        sizes = [int(off[s + 1] - off[s]) for s in range(n_sl)]
        grids = torch.zeros((n_sl, P, wl.height, wl.width), dtype=torch.complex64, device=dev)
        kernels = [B.gr_wslice_kernel(dw.kernel, m["w_first"], m["inv_width"], s) for s in range(n_sl)]
        items = [B.make_batch_item(uvw_p[int(off[s]):], vis_p[int(off[s]):], B.GR_F32, P, None, None, sizes[s],
                                   kernels[s], wl.inv_cell_u, wl.inv_cell_v, grids[s], wl.height, wl.width)
                 for s in range(n_sl)]
        need = B.gr_grid_batch_workspace_bytes(items)
        bws = torch.empty(need, dtype=torch.uint8, device=dev)
        t_batch = timed(lambda: B.gr_grid_batch(items, bws, need, stream))
        ws_need = max(B.gr_grid_workspace_bytes(sizes[s], P, kernels[s], wl.height, wl.width, None)
                      for s in range(n_sl))
        gws = torch.empty(ws_need, dtype=torch.uint8, device=dev)

        def per_slice():
            for s in range(n_sl):
                if sizes[s]:
                    a = int(off[s])
                    B.gr_grid(uvw_p[a:], vis_p[a:], B.GR_F32, None, None, sizes[s], P, kernels[s], wl.inv_cell_u,
                              wl.inv_cell_v, grids[s], wl.height, wl.width, None, gws, ws_need, None, stream)

        t_per = timed(per_slice)
        kept = int(off[n_sl])
        upd = kept * P * S * S
        log(f"w-stacking leg S={S}: partition {t_part:.3f} ms, batch {t_batch:.2f} ms, per slice {t_per:.2f} ms")
        out["per_support"][str(S)] = {
            "n_vis": N, "slice_sizes": sizes, "partition_ms": t_part,
            "partition_GB_per_s": 2 * N * (24 + 8 * P) / (t_part * 1e-3) / 1e9,
            "batch_ms": t_batch, "per_slice_ms": t_per,
            "batch_updates_per_s": upd / (t_batch * 1e-3), "per_slice_updates_per_s": upd / (t_per * 1e-3)}
        del grids, bws, gws, uvw_p, vis_p, dw
        torch.cuda.empty_cache()
    return out


def aterm_leg(dev, stream, reps: int) -> dict:
    """Gridding with non-separable GCFs that change per visibility and per
    polarisation (Section 6, A-projection) on the full-shape tracks: 16 GCF ids
    (8 time intervals x 2 channel groups), 4 w planes, oversampling 8, one
    synthetic complex GCF per (id, plane, phase, polarisation), quad pol,
    4096^2, S=16 and S=32.  Times whole gr_grid_aterm calls (fused preprocess
    and binning, the register-window gridder); HIP events on the stream, median
    of ``reps`` after one untimed call."""
    import numpy as np
    import torch
    from paper_1605_07023_amd import binding as B, runner
    from synth import aterm_taps, aterm_workload
    out = {"workload": "full-shape tracks (33,030,144 vis, quad pol, 4096^2), 16 GCF ids (8 time intervals x "
                       "2 channel groups), 4 w planes, oversampling 8, synthetic complex GCFs per polarisation, "
                       "FP32 taps (67 MB table at S=16, 268 MB at S=32)", "per_support": {}}
    for S in (16, 32):
        wl = aterm_workload(S)
        n_ids = wl.meta["n_ids"]
        taps = aterm_taps(0, n_ids, wl.n_planes, wl.oversample, wl.n_pol, S)
        t_dev = torch.from_numpy(np.ascontiguousarray(taps).view(np.float32)).to(dev)
        del taps
        dw = runner.upload(wl, dev, taps=t_dev)
        dw.kernel = B.make_kernel(t_dev, S, wl.oversample, wl.n_planes, taps_complex=True, w_min=wl.w_min,
                                  inv_dw=wl.inv_dw, kind=B.GR_TABLE2D)
        ids = torch.from_numpy(wl.meta["kernel_id"]).to(dev)
        g = torch.zeros((wl.n_pol, wl.height, wl.width), dtype=torch.complex64, device=dev)
        need = B.gr_grid_aterm_workspace_bytes(wl.n_vis, wl.n_pol, S, wl.height, wl.width)
        ws = torch.empty(need, dtype=torch.uint8, device=dev)
        st = torch.zeros(2, dtype=torch.int64, device=dev)

        def call():
            B.gr_grid_aterm(dw.uvw, dw.vis, B.GR_F32, None, None, ids, n_ids, wl.n_vis, wl.n_pol, dw.kernel,
                            wl.inv_cell_u, wl.inv_cell_v, g, wl.height, wl.width, ws, need, st, stream)

        call()
        torch.cuda.synchronize()
        kept = int(st[0].item())
        ms = []
        for _ in range(reps):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(stream)
            call()
            b.record(stream)
            torch.cuda.synchronize()
            ms.append(a.elapsed_time(b))
        t = sorted(ms)[len(ms) // 2]
        upd = kept * wl.n_pol * S * S
        # the same table stored as FP16 (half the tap bytes, FP32 arithmetic)
        t16_dev = t_dev.to(torch.float16)
        k16 = B.make_kernel(t16_dev, S, wl.oversample, wl.n_planes, taps_complex=True, tap_dtype=B.GR_F16,
                            w_min=wl.w_min, inv_dw=wl.inv_dw, kind=B.GR_TABLE2D)
        ms16 = []
        for _ in range(reps + 1):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(stream)
            B.gr_grid_aterm(dw.uvw, dw.vis, B.GR_F32, None, None, ids, n_ids, wl.n_vis, wl.n_pol, k16,
                            wl.inv_cell_u, wl.inv_cell_v, g, wl.height, wl.width, ws, need, st, stream)
            b.record(stream)
            torch.cuda.synchronize()
            ms16.append(a.elapsed_time(b))
        t16 = sorted(ms16[1:])[len(ms16[1:]) // 2]
        log(f"A-term leg S={S}: {t:.2f} ms per call, {upd / (t * 1e-3):.3e} updates/s; FP16 taps {t16:.2f} ms")
        out["per_support"][str(S)] = {"n_vis": wl.n_vis, "kept": kept, "call_ms": t,
                                      "updates_per_s": upd / (t * 1e-3), "tap_GB_per_s": upd * 8 / (t * 1e-3) / 1e9,
                                      "f16_taps_call_ms": t16, "f16_taps_updates_per_s": upd / (t16 * 1e-3)}
        del g, ws, dw, t_dev, t16_dev, ids
        torch.cuda.empty_cache()
    return out


def _timed(stream, fn, reps: int) -> float:
    """Median of ``reps`` HIP-event timings (ms) on ``stream`` after one untimed call."""
    import torch
    fn()
    torch.cuda.synchronize()
    ms = []
    for _ in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        fn()
        b.record(stream)
        torch.cuda.synchronize()
        ms.append(a.elapsed_time(b))
    return sorted(ms)[len(ms) // 2]


def precision_leg(dev, uvw, wls, kern32, grids_f32, n_done, stream, reps: int) -> dict:
    """Reduced precision on the full shape: taps stored FP16 or BF16, visibilities
    as FP16 pairs with one FP32 scale per 256 visibilities, FP32 accumulation.
    Per support and tap type: the fused preprocess-and-bin and the gridder timed
    apart (HIP events), and the relative L2 distance of the grid from the FP32
    path's grid of the timed steps (which is within ~1e-7 of the FP64 oracle; the
    error against the oracle itself is measured by tests/test_gpu_precision.py)."""
    import torch
    from paper_1605_07023_amd import binding as B, runner
    from synth import quantize_vis_f16
    wl0 = wls[min(wls)]
    N, P = wl0.n_vis, wl0.n_pol
    halves, scales = quantize_vis_f16(wl0.vis)
    vis16 = torch.from_numpy(halves).to(dev)
    sc = torch.from_numpy(scales).to(dev)
    del halves, scales
    out = {"workload": "the full-shape visibilities (33,030,144, quad pol, 4096^2) with taps stored FP16 or BF16 "
                       "and visibilities as FP16 pairs with one FP32 scale per 256; FP32 arithmetic",
           "per_support": {}}
    for S, wl in sorted(wls.items()):
        ref = grids_f32[S] / float(n_done)
        res = {}
        for name, dt in (("f16", B.GR_F16), ("bf16", B.GR_BF16)):
            taps = runner.make_taps(wl, dev, dt, stream)
            k = B.make_kernel(taps, S, wl.oversample, wl.n_planes, taps_complex=True, tap_dtype=dt,
                              w_min=wl.w_min, inv_dw=wl.inv_dw)
            nb = B.gr_preprocess_bin_bytes(N, P, S, wl.height, wl.width, 0)
            bins = torch.empty(nb, dtype=torch.uint8, device=dev)
            g = torch.zeros((P, wl.height, wl.width), dtype=torch.complex64, device=dev)

            def pre():
                B.gr_preprocess_bin(uvw, vis16, B.GR_F16, sc, None, N, P, k, wl.inv_cell_u, wl.inv_cell_v,
                                    wl.height, wl.width, 0, bins, nb, None, stream)

            def grd():
                B.gr_grid_binned(bins, N, P, k, 0, g, wl.height, wl.width, stream)

            t_pre = _timed(stream, pre, reps)
            t_grid = _timed(stream, grd, reps)
            g.zero_()
            grd()
            torch.cuda.synchronize()
            err = float(torch.linalg.norm(g - ref) / torch.linalg.norm(ref))
            upd = N * P * S * S
            res[name] = {"preprocess_bin_ms": t_pre, "grid_kernel_ms": t_grid,
                         "grid_kernel_updates_per_s": upd / (t_grid * 1e-3),
                         "grid_kernel_pct_fp32_matrix_peak": 100.0 * 8 * upd / (t_grid * 1e-3) / FP32_MFMA_PEAK,
                         "rel_l2_vs_f32_path": err}
            log(f"precision leg S={S} {name}: preprocess+bin {t_pre:.2f} ms, grid {t_grid:.2f} ms, "
                f"rel L2 vs FP32 path {err:.2e}")
            del bins, g, taps
        out["per_support"][str(S)] = res
        del ref
        torch.cuda.empty_cache()
    del vis16, sc
    return out


def batch_leg(dev, stream, reps: int) -> dict:
    """The uneven 32-instance batch (visibility counts lognormal over 1e4..1e6,
    grids 1024^2 / 2048^2 / 4096^2, supports 8 / 16 / 32, single and quad pol):
    segment lengths per instance class from the autotuner, then the whole batch
    as one launch of its captured HIP graph, as one gr_grid_batch call, and as one
    gr_grid call per instance (HIP events on the stream); per-instance rates from
    one gr_grid call each."""
    import torch
    from paper_1605_07023_amd import autotune, binding as B, runner
    from synth import batch_workload
    wls = batch_workload()
    dws = [runner.upload(wl, dev) for wl in wls]
    memo = autotune.Memo(os.path.join(tempfile.gettempdir(), "gridder_bench_batch_memo.json"))
    segs = autotune.batch_seg_lens(dws, memo)
    grids = [torch.zeros((wl.n_pol, wl.height, wl.width), dtype=torch.complex64, device=dev) for wl in wls]
    stats = [torch.zeros(2, dtype=torch.int64, device=dev) for _ in wls]
    bg = runner.BatchGraph(dws, grids, seg_lens=segs, stats=stats)
    t_graph = _timed(stream, lambda: bg.launch(stream), reps)
    for st in stats:
        st.zero_()
    bg.launch(stream)
    torch.cuda.synchronize()
    kept = [int(st[0].item()) for st in stats]
    items = runner.batch_items(dws, grids, segs)
    need = B.gr_grid_batch_workspace_bytes(items)
    ws = torch.empty(max(need, 1), dtype=torch.uint8, device=dev)
    t_eager = _timed(stream, lambda: B.gr_grid_batch(items, ws, need, stream), reps)
    per = []
    wss = None
    for dw, g, sl in zip(dws, grids, segs):
        wl = dw.wl
        tn = runner.tuning(vis_per_wg=sl)
        nw = B.gr_grid_workspace_bytes(wl.n_vis, wl.n_pol, dw.kernel, wl.height, wl.width, tn)
        if wss is None or wss.numel() < nw:
            wss = torch.empty(max(nw, 1), dtype=torch.uint8, device=dev)
        per.append(_timed(stream, lambda dw=dw, g=g, tn=tn: runner.grid(dw, g, tn, wss, stream=stream), reps))
    upd_i = [k * wl.n_pol * wl.support ** 2 for k, wl in zip(kept, wls)]
    total = sum(upd_i)
    bg.close()
    log(f"batch leg: graph {t_graph:.2f} ms, one call {t_eager:.2f} ms, per-instance calls {sum(per):.2f} ms")
    out = {"workload": "32 instances, N lognormal over 1e4..1e6 (clipped), grids 1024^2/2048^2/4096^2, S in "
                       "{8, 16, 32}, P in {1, 4}, single-channel 64-antenna tracks each",
           "n_instances": len(wls), "n_vis_total": int(sum(wl.n_vis for wl in wls)), "updates": total,
           "graph_launch_ms": t_graph, "batch_call_ms": t_eager, "per_instance_calls_ms": sum(per),
           "graph_updates_per_s": total / (t_graph * 1e-3),
           "per_instance_mean_updates_per_s_in_graph": total / (t_graph * 1e-3) / len(wls),
           "instances": [{"n_vis": wl.n_vis, "P": wl.n_pol, "S": wl.support, "side": wl.width, "seg_len": sl,
                          "call_ms": t, "updates_per_s": u / (t * 1e-3)}
                         for wl, sl, t, u in zip(wls, segs, per, upd_i)]}
    del dws, grids, ws, wss
    torch.cuda.empty_cache()
    return out


_FIXED_ROMEIN = None   # --romein-tuning: one VALU-kernel configuration instead of a sweep


def _romein_tuning(dw, n_baselines: int = 2016, reps: int = 2, quick: bool = False):
    """Coarsening, block order and chunk length of the VALU kernel from the
    autotuner, timed on the first ``n_baselines`` baselines' worth of the
    workload (2016 baselines in all: the whole set by default, since the
    kernel's parallelism is chunks x residues and a subset shortens every
    chunk); ``quick``: row-by-row block order and equal chunks only."""
    import copy
    from paper_1605_07023_amd import autotune, runner
    if _FIXED_ROMEIN is not None:
        return _FIXED_ROMEIN, {}
    wl = dw.wl
    n = min(wl.n_vis, n_baselines * max(1, wl.n_vis // 2016))
    if n < wl.n_vis:
        small = copy.copy(wl)
        small.uvw, small.vis = wl.uvw[:n], wl.vis[:n]
        sdw = runner.upload(small, dw.uvw.device, taps=dw.taps)
        sdw.kernel = dw.kernel
    else:
        sdw = dw
    cands = autotune.candidates(wl.n_pol, wl.support, variants=(1,),
                                **(dict(tiles=("flat",), vis_per_wg=(0,)) if quick else
                                   dict(tiles=("flat",), vis_per_wg=(0, 512, 1024, 2048))))
    best, times = autotune.tune(sdw, cands, reps=reps)
    return best, {autotune.describe(c): round(t, 4) for c, t in zip(cands, times)}


def order_leg(dev, stream, reps: int, supports=(16, 32)) -> dict:
    """The full-shape visibilities in two orders: baseline, time, channel (the
    timed step's order) and baseline, channel, time (consecutive visibilities
    are consecutive dumps of one channel).  Per support: the whole binned MFMA
    path (gr_grid) and the paper's VALU kernel (gr_grid with variant 1, its
    coarsening autotuned on the order's own first baselines), HIP events."""
    import torch
    from paper_1605_07023_amd import binding as B, runner
    from synth import full_shape_workload
    out = {"workload": "full shape (33,030,144 quad-pol vis, 4096^2, separable W kernels, 32 planes) in "
                       "(baseline, time, channel) and (baseline, channel, time) order", "per_order": {}}
    for order in ("btc", "bct"):
        res = {}
        for S in supports:
            wl = full_shape_workload(S, order=order)
            dw = runner.upload(wl, dev)
            g = torch.zeros((wl.n_pol, wl.height, wl.width), dtype=torch.complex64, device=dev)
            upd = wl.n_vis * wl.n_pol * S * S
            t2 = runner.tuning(variant=2)
            nw = B.gr_grid_workspace_bytes(wl.n_vis, wl.n_pol, dw.kernel, wl.height, wl.width, t2)
            ws = torch.empty(nw, dtype=torch.uint8, device=dev)
            t_mfma = _timed(stream, lambda: runner.grid(dw, g, t2, ws, stream=stream), reps)
            del ws
            best, sweep = _romein_tuning(dw, n_baselines=64, quick=True)
            nw1 = B.gr_grid_workspace_bytes(wl.n_vis, wl.n_pol, dw.kernel, wl.height, wl.width, best)
            ws1 = torch.empty(nw1, dtype=torch.uint8, device=dev)
            t_val = _timed(stream, lambda: runner.grid(dw, g, best, ws1, stream=stream), 1 if order == "btc" else reps)
            log(f"order leg {order} S={S}: MFMA path {t_mfma:.2f} ms, VALU kernel {t_val:.1f} ms "
                f"(cu {best.cu} cv {best.cv} wg {best.wg_u}x{best.wg_v} vis/item {best.vis_per_wg})")
            res[str(S)] = {"mfma_path_ms": t_mfma, "mfma_path_updates_per_s": upd / (t_mfma * 1e-3),
                           "valu_kernel_call_ms": t_val, "valu_kernel_updates_per_s": upd / (t_val * 1e-3),
                           "valu_pct_nonpacked_fp32": 100.0 * 8 * upd / (t_val * 1e-3) / FP32_VALU_NONPACKED,
                           "valu_tuning": [best.cu, best.cv, best.wg_u, best.wg_v, best.vis_per_wg]}
            del ws1, g, dw
            torch.cuda.empty_cache()
        out["per_order"][order] = res
    return out



def romein_tracks_leg(dev, stream, reps: int, supports=(16, 32)) -> dict:
    """The paper's own method (variant 1: Romein work distribution with thread
    coarsening on the vector units, FP32 atomic flushes) beside the MFMA path on
    the paper-like single-channel tracks (2016 baselines x 3600 dumps of 2 s,
    quad pol, 2048^2, separable W kernel, 32 planes), where consecutive
    visibilities of a baseline stay on nearby cells; whole gr_grid calls, HIP
    events on the stream, median of ``reps`` after one untimed call."""
    import torch
    from paper_1605_07023_amd import binding as B, runner
    from synth import compression_workload
    out = {"workload": "2016 baselines x 3600 dumps of 2 s over 2 h, 1 channel at 1.4 GHz, quad pol, 2048^2, "
                       "separable W kernel, 32 planes, oversampling 8 (uncompressed)", "per_support": {}}
    for S in supports:
        wl = compression_workload(support=S)
        dw = runner.upload(wl, dev)
        g = torch.zeros((wl.n_pol, wl.height, wl.width), dtype=torch.complex64, device=dev)
        res = {}
        best, sweep = _romein_tuning(dw)
        res["romein_tuning"] = {"cu": best.cu, "cv": best.cv, "wg_u": best.wg_u, "wg_v": best.wg_v,
                                "vis_per_item": best.vis_per_wg, "sweep_ms": sweep}
        for name, variant in (("romein_valu", 1), ("mfma", 2)):
            tune = best if variant == 1 else runner.tuning(variant=variant)
            need = B.gr_grid_workspace_bytes(wl.n_vis, wl.n_pol, dw.kernel, wl.height, wl.width, tune)
            ws = torch.empty(need, dtype=torch.uint8, device=dev)
            runner.grid(dw, g, tune, ws, stream=stream)
            torch.cuda.synchronize()
            ms = []
            for _ in range(reps):
                a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                a.record(stream)
                runner.grid(dw, g, tune, ws, stream=stream)
                b.record(stream)
                torch.cuda.synchronize()
                ms.append(a.elapsed_time(b))
            t = sorted(ms)[len(ms) // 2]
            res[name] = {"call_ms": t, "updates_per_s": wl.n_vis * wl.n_pol * S * S / (t * 1e-3)}
            del ws
        res["romein_pct_fp32_valu_nonpacked"] = 100.0 * 8 * res["romein_valu"]["updates_per_s"] / FP32_VALU_NONPACKED
        res["romein_pct_fp32_peak"] = 100.0 * 8 * res["romein_valu"]["updates_per_s"] / FP32_VALU_PEAK
        log(f"paper's method on 2 s-dump tracks S={S}: {res['romein_valu']['call_ms']:.2f} ms "
            f"(MFMA path {res['mfma']['call_ms']:.2f} ms)")
        out["per_support"][str(S)] = res
        del g, dw
        torch.cuda.empty_cache()
    return out


def degrid_leg(dev, uvw, wl, kern, grid, stream, reps: int) -> dict:
    """gr_degrid (the adjoint operation, predicting every visibility from the grid)
    on the full-shape S=32 visibilities and the grid the timed steps produced:
    whole calls (binning, per-segment ordering, MFMA degridder), HIP events on the
    stream, after one untimed call."""
    import torch
    from paper_1605_07023_amd import binding as B
    N, P, S = wl.n_vis, wl.n_pol, wl.support
    need = B.gr_degrid_workspace_bytes(N, P, S, wl.height, wl.width, 0)
    ws = torch.empty(need, dtype=torch.uint8, device=dev)
    out = torch.empty((N, P), dtype=torch.complex64, device=dev)
    st = torch.zeros(2, dtype=torch.int64, device=dev)

    def call():
        B.gr_degrid(uvw, N, P, kern, wl.inv_cell_u, wl.inv_cell_v, grid, wl.height, wl.width, out, 0, ws, need,
                    st, stream)

    call()
    torch.cuda.synchronize()
    ms = []
    for _ in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        call()
        b.record(stream)
        torch.cuda.synchronize()
        ms.append(a.elapsed_time(b))
    kept = int(st.cpu()[0]) // (reps + 1)
    med = sorted(ms)[len(ms) // 2]
    upd = kept * P * S * S
    log(f"degridding leg: {med:.2f} ms per call")
    del ws, out
    return {"workload": "the full-shape S=32 visibilities predicted from the S=32 grid of the timed steps",
            "ms_per_call": med, "updates_per_call": upd, "updates_per_s": upd / (med * 1e-3),
            "pct_fp32_matrix_peak": 100.0 * 8 * upd / (med * 1e-3) / FP32_MFMA_PEAK,
            "call": "gr_degrid: binning, per-segment Z ordering, MFMA degridder (16x16x4 FP32)"}


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--supports", default="16,32")
    ap.add_argument("--cu", type=int, default=0)
    ap.add_argument("--cv", type=int, default=0)
    ap.add_argument("--variant", type=int, default=2, help="1: VALU work-item kernel, 2: MFMA")
    ap.add_argument("--seg-len", type=int, default=0)
    ap.add_argument("--row-groups", type=int, default=0,
                    help="MFMA gridder: row groups per wave (with --seg-len or --no-autotune; 0: default)")
    ap.add_argument("--cpu-budget", type=float, default=20.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--precision", choices=["f32", "f16", "bf16"], default="f32",
                    help="storage of taps and visibilities (f16/bf16: taps in that type, "
                         "visibilities as float16 pairs with one float32 scale per 256)")
    ap.add_argument("--no-autotune", action="store_true",
                    help="skip the segment-length sweep on a small subset (library default instead)")
    ap.add_argument("--no-learned", action="store_true",
                    help="skip the learned-kernel leg (network vs 2-D table, after the timed region)")
    ap.add_argument("--learned-steps", type=int, default=12000)
    ap.add_argument("--no-compression", action="store_true",
                    help="skip the compression leg (2 s-dump tracks, after the timed region)")
    ap.add_argument("--no-wstack", action="store_true",
                    help="skip the w-stacking leg (7 w slices of the 2 s-dump tracks, after the timed region)")
    ap.add_argument("--no-aterm", action="store_true",
                    help="skip the A-term leg (per-visibility non-separable GCFs, after the timed region)")
    ap.add_argument("--no-romein-tracks", action="store_true",
                    help="skip the leg timing the paper's VALU method on the single-channel tracks")
    ap.add_argument("--no-degrid", action="store_true",
                    help="skip the degridding leg (gr_degrid of the S=32 grid, after the timed region)")
    ap.add_argument("--no-precision", action="store_true",
                    help="skip the reduced-precision leg (FP16/BF16 taps, scaled FP16 visibilities)")
    ap.add_argument("--no-batch", action="store_true",
                    help="skip the batch leg (32 uneven instances, one graph launch)")
    ap.add_argument("--no-order", action="store_true",
                    help="skip the order leg ((baseline, channel, time) against (baseline, time, channel))")
    ap.add_argument("--only", default="",
                    help="run only these legs (comma list of compression, wstack, aterm, batch, order, "
                         "romein_tracks), without the timed step, and print their JSON (for profiling)")
    ap.add_argument("--romein-tuning", default="",
                    help="cu,cv,wg_u,wg_v,vis_per_wg of the VALU kernel in the romein_tracks and order legs "
                         "(given: no sweep; for profiling one configuration)")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="run one device-to-device copy of this size before timing "
                         "(reference dispatch for HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print(json.dumps({"error": "this benchmark runs on exactly one GPU and has no multi-GPU mode",
                          "n_gpus": args.gpus}), flush=True)
        return 2

    import numpy as np
    import torch

    from paper_1605_07023_amd import binding as B
    from paper_1605_07023_amd import runner
    from synth import full_shape_workload

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    global _FIXED_ROMEIN
    if args.romein_tuning:
        f = [int(x) for x in args.romein_tuning.split(",")]
        _FIXED_ROMEIN = B.GrTuning(*(f + [0] * (5 - len(f)))[:5], 1)
    if args.only:
        supports = tuple(int(x) for x in args.supports.split(","))
        legs = {"compression": lambda st: compression_leg(dev, st, reps=5),
                "wstack": lambda st: wstack_leg(dev, st, reps=5),
                "aterm": lambda st: aterm_leg(dev, st, reps=3),
                "batch": lambda st: batch_leg(dev, st, reps=5),
                "order": lambda st: order_leg(dev, st, reps=3, supports=supports),
                "romein_tracks": lambda st: romein_tracks_leg(dev, st, reps=3, supports=supports)}
        names = [n for n in args.only.split(",") if n]
        unknown = [n for n in names if n not in legs]
        if unknown:
            print(json.dumps({"error": f"unknown legs {unknown}", "legs": sorted(legs)}), flush=True)
            return 2
        stream = torch.cuda.current_stream(dev)
        out = {"only": names}
        for n in names:
            log(f"leg {n}")
            out[n] = legs[n](stream)
        print(json.dumps(out), flush=True)
        return 0
    supports = [int(s) for s in args.supports.split(",")]
    log("generating inputs")
    wls = {S: full_shape_workload(S) for S in supports}
    wl0 = wls[supports[0]]
    N, P = wl0.n_vis, wl0.n_pol
    log(f"uploading N={N} P={P}")
    uvw = torch.from_numpy(np.ascontiguousarray(wl0.uvw)).to(dev)
    tap_dt = {"f32": B.GR_F32, "f16": B.GR_F16, "bf16": B.GR_BF16}[args.precision]
    vis_scale = None
    vis_dt = B.GR_F32
    if args.precision == "f32":
        vis = torch.from_numpy(np.ascontiguousarray(wl0.vis)).to(dev)
    else:
        from synth import quantize_vis_f16
        halves, scales = quantize_vis_f16(wl0.vis)
        vis = torch.from_numpy(halves).to(dev)
        vis_scale = torch.from_numpy(scales).to(dev)
        vis_dt = B.GR_F16
    taps, kern, grids, table_ms = {}, {}, {}, {}
    for S, wl in wls.items():
        runner.make_taps(wl, dev, tap_dt)                 # untimed first call (kernel load)
        t_a, t_b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        t_a.record()
        taps[S] = runner.make_taps(wl, dev, tap_dt)
        t_b.record()
        torch.cuda.synchronize()
        table_ms[S] = t_a.elapsed_time(t_b)
        kern[S] = B.make_kernel(taps[S], S, wl.oversample, wl.n_planes, taps_complex=True,
                                tap_dtype=tap_dt, w_min=wl.w_min, inv_dw=wl.inv_dw)
        grids[S] = torch.zeros((P, wl.height, wl.width), dtype=torch.complex64, device=dev)
    variant = args.variant if args.variant in (1, 2) else 2
    tune = runner.tuning(args.cu, args.cv, vis_per_wg=args.seg_len, variant=variant)
    seg_len = {S: args.seg_len for S in supports}
    tuned = {}
    if variant == 2 and not args.no_autotune and args.seg_len <= 0:
        # Section 4: time the candidate decompositions, then run with the winner.  The
        # sweep runs on the workload itself: on a 128-baseline subset the segments are
        # shorter, and the row-group count it picked at S = 32 ran 6 % slower at full size
        from paper_1605_07023_amd import autotune
        for S in supports:
            sdw = runner.DeviceWorkload(wls[S], uvw, vis, None, taps[S], kern[S], tap_dt, vis_dt, vis_scale)
            cands = autotune.candidates(P, S, variants=(2,))
            # gr_autotune keeps the winner in the library's memo, where gr_grid_binned
            # finds its row groups per wave for this problem class
            best, times = autotune.tune(sdw, cands, reps=3)
            seg_len[S] = best.vis_per_wg
            tuned[str(S)] = {"seg_len": best.vis_per_wg, "row_groups": best.wg_v,
                             "sweep_ms": {f"{c.vis_per_wg}/rg{c.wg_v}": round(t, 4) for c, t in zip(cands, times)}}
            log(f"autotune S={S}: seg_len {best.vis_per_wg}, row groups per wave {best.wg_v}")
            del sdw
        torch.cuda.synchronize()
    elif variant == 2 and args.row_groups > 0:
        for S in supports:     # a fixed configuration: into the memo that gr_grid_binned reads
            B.gr_tuning_memo_put(P, kern[S], wls[S].height, wls[S].width, 0,
                                 runner.tuning(0, 0, 0, args.row_groups, seg_len[S], 2))
            tuned[str(S)] = {"seg_len": seg_len[S], "row_groups": args.row_groups, "sweep_ms": {}}
    rec = torch.empty((N, 2), dtype=torch.int32, device=dev)
    wvis = torch.empty((N, P), dtype=torch.complex64, device=dev)
    stats = torch.zeros(2, dtype=torch.int64, device=dev)
    bins_bytes = max(B.gr_preprocess_bin_bytes(N, P, S, wls[S].height, wls[S].width, seg_len[S]) for S in supports)
    bins = torch.empty(bins_bytes, dtype=torch.uint8, device=dev) if variant == 2 else None
    stream = torch.cuda.current_stream(dev)
    ev = {S: [] for S in supports}

    def step(record: bool):
        for S in supports:
            wl = wls[S]
            if record:
                ep = torch.cuda.Event(enable_timing=True)
                ep.record(stream)
            if variant == 2:
                # preprocess and bin fused: records and tile counts from uvw, then the
                # weighted visibilities straight to their binned positions
                B.gr_preprocess_bin(uvw, vis, vis_dt, vis_scale, None, N, P, kern[S], wl.inv_cell_u,
                                    wl.inv_cell_v, wl.height, wl.width, seg_len[S], bins, bins_bytes, stats,
                                    stream)
            else:
                B.gr_preprocess(uvw, vis, vis_dt, vis_scale, None, N, P, kern[S], wl.inv_cell_u,
                                wl.inv_cell_v, wl.height, wl.width, rec, wvis, stats, stream)
            if record:
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record(stream)
            if variant == 2:
                B.gr_grid_binned(bins, N, P, kern[S], seg_len[S], grids[S], wl.height, wl.width, stream)
            else:
                B.gr_grid_records(rec, wvis, N, P, kern[S], grids[S], wl.height, wl.width, tune, stream)
            if record:
                e1.record(stream)
                ev[S].append((ep, e0, e1))

    if args.calib_copy_mib > 0:
        n = args.calib_copy_mib << 18                     # float32 elements
        src = torch.ones(n, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"calibration copy of {args.calib_copy_mib} MiB done")
        del src, dst
    log(f"warmup {args.warmup} steps")
    for _ in range(args.warmup):
        step(False)
    torch.cuda.synchronize()
    stats.zero_()
    torch.cuda.synchronize()
    log(f"timing {args.steps} steps")
    t0 = time.perf_counter()
    for i in range(args.steps):
        step(True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    gridded, dropped = [int(x) for x in stats.cpu().tolist()]
    n_valid = gridded // (args.steps * len(supports))
    log(f"timed region {t1 - t0:.3f}s, gridded per pass {n_valid}, dropped {dropped}")

    per_support = {}
    total_updates = 0
    for S in supports:
        upd = n_valid * P * S * S
        total_updates += upd
        kms = [a.elapsed_time(b) for _, a, b in ev[S]]
        pms = [p.elapsed_time(a) for p, a, _ in ev[S]]
        avg = sum(kms) / len(kms) * 1e-3
        per_support[str(S)] = {"updates_per_step": upd, "grid_kernel_ms": avg * 1e3,
                               "preprocess_bin_ms": sum(pms) / len(pms),
                               "table_generation_ms": table_ms[S],
                               "grid_kernel_updates_per_s": upd / avg,
                               "grid_kernel_pct_fp32_matrix_peak": 100.0 * 8 * upd / avg / FP32_MFMA_PEAK}
    ms_per_step = (t1 - t0) / args.steps * 1e3
    value = total_updates * args.steps / (t1 - t0)

    dom = str(max(supports))
    d = per_support[dom]
    achieved = 8.0 * d["updates_per_step"] / (d["grid_kernel_ms"] * 1e-3)
    traffic = None
    if os.path.exists(TRAFFIC_FILE):
        try:
            tr = json.load(open(TRAFFIC_FILE))
            if tr.get("source_hash") == source_hash(variant) and tr.get("support") == int(dom):
                traffic = tr.get("bytes_per_launch")
        except (ValueError, OSError):
            traffic = None
    if variant == 2:
        roofline = {"bound": "mfma", "achieved": achieved / 1e12, "peak": FP32_MFMA_PEAK / 1e12,
                    "unit": "TFLOP/s", "frac": achieved / FP32_MFMA_PEAK, "traffic": traffic,
                    "kernel": f"grid_mfma_waves<4, complex, {48 if int(dom) <= 32 else 64}> (S={dom}), "
                              "FP32 MFMA 16x16x4"}
    else:
        roofline = {"bound": "alu", "achieved": achieved / 1e12, "peak": FP32_VALU_PEAK / 1e12,
                    "unit": "TFLOP/s", "frac": achieved / FP32_VALU_PEAK, "traffic": traffic,
                    "kernel": f"romein_valu_kernel (S={dom})"}

    learned = None
    if not args.no_learned and variant == 2 and args.precision == "f32" and 32 in supports:
        log("learned-kernel leg")
        learned = learned_leg(dev, uvw, vis, wls[32], rec, wvis, bins, bins_bytes, seg_len[32], stream,
                              args.learned_steps, reps=2)

    degrid = None
    if not args.no_degrid and variant == 2 and args.precision == "f32" and 32 in supports:
        log("degridding leg")
        degrid = degrid_leg(dev, uvw, wls[32], kern[32], grids[32], stream, reps=5)

    compression = None
    if not args.no_compression and variant == 2 and args.precision == "f32":
        log("compression leg")
        compression = compression_leg(dev, stream, reps=5)

    wstack = None
    if not args.no_wstack and variant == 2 and args.precision == "f32":
        log("w-stacking leg")
        wstack = wstack_leg(dev, stream, reps=5)

    aterm = None
    if not args.no_aterm and variant == 2 and args.precision == "f32":
        log("A-term leg")
        aterm = aterm_leg(dev, stream, reps=3)

    precision = None
    if not args.no_precision and variant == 2 and args.precision == "f32":
        log("reduced-precision leg")
        precision = precision_leg(dev, uvw, wls, kern.get(32), grids, args.warmup + args.steps, stream, reps=5)

    batch = None
    if not args.no_batch and variant == 2 and args.precision == "f32":
        log("batch leg")
        batch = batch_leg(dev, stream, reps=5)

    order = None
    if not args.no_order and variant == 2 and args.precision == "f32":
        log("order leg")
        order = order_leg(dev, stream, reps=3)

    romein_tracks = None
    if not args.no_romein_tracks and variant == 2 and args.precision == "f32":
        log("paper's method on the 2 s-dump tracks")
        romein_tracks = romein_tracks_leg(dev, stream, reps=3)

    cpu = None
    if not args.no_cpu_baseline:
        threads = min(16, os.cpu_count() or 1)
        log(f"cpu baseline on {threads} threads")
        cpu = cpu_baseline(full_shape_workload, int(dom), args.cpu_budget, threads)

    out = {
        "metric": "vis-tap updates/s", "value": value, "unit": "updates/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_per_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        # the arithmetic type: taps are widened to FP32 in LDS and every product and sum is FP32,
        # also when the taps and visibilities are stored in 16 bits (--precision f16 / bf16)
        "dtype": "f32",
        "storage": {"taps": args.precision,
                    "vis": "f32" if args.precision == "f32" else "f16 pairs, one f32 scale per 256"},
        "data": "synthetic",
        "config": {"workload": "earth-rotation uv tracks, 64 antennas (2016 baselines) x 1024 dumps "
                               "over 8 h x 16 channels, quad pol, 4096^2 grid, separable W kernels "
                               "S=16 and S=32, 32 planes, oversampling 8",
                   "n_vis": N, "n_pol": P, "grid": [wl0.height, wl0.width], "supports": supports,
                   "order": "baseline, time, channel"},
        # 157.3 TFLOP/s is both the dense FP32 matrix peak and the packed FP32 vector peak
        "pct_fp32_peak": 100.0 * 8 * value / FP32_MFMA_PEAK,
        "per_support": per_support,
        "tuning": tuned or None,
        "roofline": roofline,
        "learned_kernel": learned,
        "degrid": degrid,
        "compression": compression,
        "wstack": wstack,
        "aterm": aterm,
        "romein_tracks": romein_tracks,
        "precision": precision,
        "batch": batch,
        "order": order,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
