"""Autotuning driver and memo (Merry 2016, Section 4: the work decomposition --
coarsening factors and work-group shape -- is chosen by timing a synthetic
problem, per polarisation count, and the choice is kept for later runs).

The timing sweep runs in the library (gr_autotune), which also keeps the
winner in its in-process tuning memo: calls without a tuning then use it.
This module builds the candidate list, prepares the small data set on the
device, and keeps the memo across processes as JSON (Memo.save / Memo.install
move entries between the file and the library).  The file's key is
(device name, n_pol, support, tap kind, tap dtype, grid side class, variant
set).  A missing or unreadable file leaves the library defaults.
"""
from __future__ import annotations

import json
import os
import sys
from typing import Dict, Iterable, List, Optional, Tuple

import torch

from . import binding as B
from . import runner

DEFAULT_MEMO = os.environ.get(
    "GR_TUNE_MEMO", os.path.join(os.path.expanduser("~"), ".cache", "paper_1605_07023_amd", "tuning.json"))

SEG_LENS = (512, 1024, 2048, 4096, 8192, 16384)
COARSEN = (1, 2, 4, 8)


def _bin_blocks(support: int, c: int) -> int:
    """Blocks per bin along one axis for coarsening c: the smallest n with c n >= S + c - 1."""
    return (support + 2 * c - 2) // c


def _window(support: int) -> int:
    return 32 if support <= 16 else 48 if support <= 32 else 64


def row_group_options(n_pol: int, support: int) -> Tuple[int, ...]:
    """Row groups per wave the MFMA gridder's wave form is built for (per window)."""
    w = _window(support)
    if n_pol == 4:
        return {32: (2, 4, 8), 48: (2, 3, 4, 6), 64: (2, 4)}[w]
    return {32: (1, 2), 48: (1, 3), 64: (1, 2, 4)}[w]


def candidates(n_pol: int, support: int, variants: Iterable[int] = (1, 2),
               vis_per_wg: Iterable[int] = (0, 1024),
               tiles: Iterable[str] = ("flat", "rect"),
               seg_lens: Iterable[int] = SEG_LENS,
               row_groups: Optional[Iterable[int]] = None) -> List[B.GrTuning]:
    """Work decompositions to try.

    variant 1 (the VALU work-item kernel): coarsening cu x cv in {1, 2, 4, 8}^2
    (the paper's range) with cu * cv * n_pol <= 64 (register budget); for each,
    the order in which a chunk's work-items take the bin's blocks ("flat": row
    by row over the whole bin, "rect": tiles of up to 16 blocks along u and as
    many rows as make 64) and the visibilities per chunk (0: equal chunks, about
    four 64-lane runs per wave; 1024: the paper's chunk).  variant 2 (MFMA
    kernel): segment lengths x row groups per wave (the wave form's work-group
    shape; None: every option of the window)."""
    out = []
    if 1 in variants:
        for cu in COARSEN:
            for cv in COARSEN:
                if cu * cv * n_pol > 64:
                    continue
                nu, nv = _bin_blocks(support, cu), _bin_blocks(support, cv)
                shapes = []
                for t in tiles:
                    if t == "flat":
                        shapes.append((0, 0))
                    elif t == "rect":
                        wgu = min(nu, 16)
                        shapes.append((wgu, min(nv, max(1, 64 // wgu))))
                for wgu, wgv in shapes:
                    for vpw in vis_per_wg:
                        out.append(B.GrTuning(cu, cv, wgu, wgv, vpw, 1))
    if 2 in variants and support <= 56:
        rgs = tuple(row_groups) if row_groups is not None else row_group_options(n_pol, support)
        for sl in seg_lens:
            for rg in rgs:
                out.append(B.GrTuning(0, 0, 0, rg, sl, 2))
    return out


def describe(t: B.GrTuning) -> str:
    """Short text key of a tuning (for sweep reports)."""
    if t.variant == 1:
        tile = "flat" if t.wg_u == 0 else f"{t.wg_u}x{t.wg_v}"
        return f"valu c{t.cu}x{t.cv} tile {tile} vis {t.vis_per_wg or 'eq'}"
    return f"mfma seg {t.vis_per_wg or 'default'}" + (f" rg {t.wg_v}" if t.wg_v else "")


def memo_key(device_name: str, n_pol: int, support: int, kind: str, tap_dtype: int, side: int,
             variants: Iterable[int]) -> str:
    side_class = 1 << max(0, (int(side) - 1).bit_length())
    return f"{device_name}|P{n_pol}|S{support}|{kind}|t{tap_dtype}|g{side_class}|v{''.join(map(str, sorted(variants)))}"


def _c_class(n_pol: int, kernel: B.GrKernel, side: int, slot: int) -> list:
    """What the library's memo needs to rebuild an entry's key."""
    return [n_pol, kernel.kind, kernel.taps_complex, kernel.tap_dtype, kernel.support, int(side), slot]


class Memo:
    """JSON memo of chosen tunings; unreadable files are ignored (defaults apply)."""

    def __init__(self, path: str = DEFAULT_MEMO):
        self.path = path
        self.data: Dict[str, dict] = {}
        try:
            with open(path) as fh:
                raw = json.load(fh)
            if isinstance(raw, dict):
                self.data = {k: v for k, v in raw.items() if isinstance(v, dict) and "tuning" in v}
        except FileNotFoundError:
            pass
        except (OSError, ValueError) as e:
            print(f"[autotune] ignoring unreadable memo {path}: {e}", file=sys.stderr)

    def get(self, key: str) -> Optional[B.GrTuning]:
        e = self.data.get(key)
        if e is None:
            return None
        try:
            t = [int(x) for x in e["tuning"]]
            if len(t) != 6:
                return None
            return B.GrTuning(*t)
        except (TypeError, ValueError):
            return None

    def put(self, key: str, tuning: B.GrTuning, time_ms: float, c_class: Optional[list] = None) -> None:
        e = {"tuning": [tuning.cu, tuning.cv, tuning.wg_u, tuning.wg_v, tuning.vis_per_wg, tuning.variant],
             "time_ms": time_ms}
        if c_class is not None:
            e["c_class"] = list(c_class)
        self.data[key] = e

    def install(self, device_name: str) -> int:
        """Put this device's entries into the library's tuning memo (calls
        without a tuning then use them); returns how many were installed."""
        n = 0
        for key, e in self.data.items():
            cc = e.get("c_class")
            if not key.startswith(device_name + "|") or not isinstance(cc, list) or len(cc) != 7:
                continue
            t = self.get(key)
            if t is None:
                continue
            n_pol, kind, cplx, dtype, support, side, slot = (int(x) for x in cc)
            k = B.GrKernel(kind, dtype, cplx, support, 8, 1, 0.0, 1.0, None)
            try:
                B.gr_tuning_memo_put(n_pol, k, side, side, slot, t)
                n += 1
            except B.GridderError as err:
                print(f"[autotune] memo entry {key} not installed: {err}", file=sys.stderr)
        return n

    def save(self) -> None:
        d = os.path.dirname(self.path)
        if d:
            os.makedirs(d, exist_ok=True)
        tmp = self.path + ".tmp"
        with open(tmp, "w") as fh:
            json.dump(self.data, fh, indent=1, sort_keys=True)
        os.replace(tmp, self.path)


def tune(dw: runner.DeviceWorkload, cands: List[B.GrTuning], reps: int = 3,
         stream=None) -> Tuple[B.GrTuning, List[float]]:
    """Time every candidate on a device workload; returns (best, times in ms)."""
    wl = dw.wl
    dev = dw.uvw.device
    rec, wv = runner.preprocess(dw, stream=stream)
    grid = torch.zeros((wl.n_pol, wl.height, wl.width), dtype=torch.complex64, device=dev)
    seg = [c.vis_per_wg for c in cands if c.variant != 1] or [0]
    nb = max(B.gr_bin_bytes(wl.n_vis, wl.n_pol, wl.support, wl.height, wl.width, s) for s in seg) \
        if wl.support <= 56 else 0
    bins = torch.empty(max(nb, 1), dtype=torch.uint8, device=dev)
    best, times = B.gr_autotune(rec, wv, wl.n_vis, wl.n_pol, dw.kernel, grid, wl.height, wl.width,
                                bins, bins.numel(), cands, reps, stream)
    return cands[best], times


def tune_and_remember(dw: runner.DeviceWorkload, variants: Iterable[int] = (2,), reps: int = 3,
                      memo: Optional[Memo] = None, vis_per_wg: Iterable[int] = (0, 1024)) -> B.GrTuning:
    """Tune on the given (small) workload; the library keeps the winner for
    calls without a tuning, and the memo keeps it for later processes."""
    wl = dw.wl
    memo = memo if memo is not None else Memo()
    cands = candidates(wl.n_pol, wl.support, variants, vis_per_wg)
    best, times = tune(dw, cands, reps)
    name = torch.cuda.get_device_name(dw.uvw.device)
    side = max(wl.height, wl.width)
    key = memo_key(name, wl.n_pol, wl.support, wl.kernel, dw.tap_dtype, side, variants)
    side_class = 1 << max(0, (int(side) - 1).bit_length())
    slot = 1 if set(variants) == {1} else 0          # a VALU-only sweep feeds gr_grid_records
    memo.put(key, best, min(times), _c_class(wl.n_pol, dw.kernel, side_class, slot))
    return best


def tuning_for(device_name: str, n_pol: int, support: int, kind: str, tap_dtype: int, side: int,
               variants: Iterable[int] = (2,), memo: Optional[Memo] = None) -> Optional[B.GrTuning]:
    memo = memo if memo is not None else Memo()
    return memo.get(memo_key(device_name, n_pol, support, kind, tap_dtype, side, variants))


def batch_seg_lens(dws, memo: Optional[Memo] = None, max_vis: int = 131072, reps: int = 3) -> List[int]:
    """Segment length per instance of a batch (gr_grid_batch items).  Instances
    that share (n_pol, support, tap kind, tap dtype, grid side class) share one
    tuning, swept on the first max_vis visibilities of the largest of them and
    kept in the memo."""
    import copy
    memo = memo if memo is not None else Memo()
    out, chosen = [], {}
    name = torch.cuda.get_device_name(dws[0].uvw.device) if dws else ""
    groups: Dict[str, list] = {}
    for i, dw in enumerate(dws):
        wl = dw.wl
        key = memo_key(name, wl.n_pol, wl.support, wl.kernel, dw.tap_dtype, max(wl.height, wl.width), (2,))
        groups.setdefault(key, []).append(i)
    for key, members in groups.items():
        hit = memo.get(key)
        if hit is None:
            big = max(members, key=lambda j: dws[j].wl.n_vis)
            dw = dws[big]
            if dw.wl.n_vis > max_vis:
                wl = copy.copy(dw.wl)
                wl.uvw, wl.vis = dw.wl.uvw[:max_vis], dw.wl.vis[:max_vis]
                wl.weights = None if dw.wl.weights is None else dw.wl.weights[:max_vis]
                dw = runner.upload(wl, dw.uvw.device, tap_dtype=dw.tap_dtype, taps=dw.taps)
                dw.kernel = dws[big].kernel
            best, times = tune(dw, candidates(dw.wl.n_pol, dw.wl.support, (2,)), reps)
            memo.put(key, best, min(times))
            hit = best
        chosen[key] = hit.vis_per_wg
    for i, dw in enumerate(dws):
        wl = dw.wl
        out.append(chosen[memo_key(name, wl.n_pol, wl.support, wl.kernel, dw.tap_dtype,
                                   max(wl.height, wl.width), (2,))])
    return out


def main(argv=None) -> int:
    """Tune the full-shape geometry (first baselines only) for S = 16 and 32 and
    the tiny Kaiser-Bessel configuration; write the memo."""
    import argparse
    from synth import full_shape_workload, tiny_kb_workload
    ap = argparse.ArgumentParser()
    ap.add_argument("--baselines", type=int, default=128)
    ap.add_argument("--variants", default="1,2")
    ap.add_argument("--memo", default=DEFAULT_MEMO)
    args = ap.parse_args(argv)
    variants = tuple(int(v) for v in args.variants.split(","))
    memo = Memo(args.memo)
    dev = torch.device("cuda:0")
    for wl in [full_shape_workload(16, n_baselines=args.baselines),
               full_shape_workload(32, n_baselines=args.baselines), tiny_kb_workload()]:
        dw = runner.upload(wl, dev)
        best = tune_and_remember(dw, variants, memo=memo)
        print(f"{wl.name}: best {best.cu}x{best.cv} wg {best.wg_u}x{best.wg_v} "
              f"vis/wg {best.vis_per_wg} variant {best.variant}", flush=True)
    memo.save()
    return 0


if __name__ == "__main__":
    sys.exit(main())
