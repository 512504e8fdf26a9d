"""Device-side driver for a synthetic workload: upload inputs, build the kernel
table on the GPU (FP64 generation, cast to the tap dtype), and call the C ABI.

Used by the tests, the smoke check and the benchmark.  All arithmetic happens
in libgridder.so; this module only allocates torch tensors and passes pointers.
"""
from __future__ import annotations

import dataclasses
from typing import Optional

import numpy as np
import torch

from . import binding as B

_TAP_TORCH = {B.GR_F32: torch.float32, B.GR_F16: torch.float16, B.GR_BF16: torch.bfloat16,
              B.GR_F64: torch.float64}


def make_taps(wl, device, tap_dtype: int = B.GR_F32, stream=None) -> torch.Tensor:
    """Kernel table for a workload, generated on the device (gr_make_*_table)."""
    S, O = wl.support, wl.oversample
    dt = _TAP_TORCH[tap_dtype]
    if wl.kernel == "kb":
        out = torch.empty((1, O, S), dtype=dt, device=device)
        B.gr_make_kb_table(wl.beta, S, O, tap_dtype, out, stream)
    elif wl.kernel == "wsep":
        out = torch.empty((wl.n_planes, O, S, 2), dtype=dt, device=device)
        whs = wl.plane_w_hat()
        step = (whs[1] - whs[0]) if wl.n_planes > 1 else 0.0
        B.gr_make_wkernel_table(S, O, wl.n_planes, float(whs[0]), float(step), wl.support_aa,
                                wl.beta, 0, tap_dtype, out, stream)
    elif wl.kernel == "w2d":
        out = torch.empty((wl.n_planes, O, O, S, S, 2), dtype=dt, device=device)
        whs = wl.plane_w_hat()
        step = (whs[1] - whs[0]) if wl.n_planes > 1 else 0.0
        B.gr_make_wkernel2d_table(S, O, wl.n_planes, float(whs[0]), float(step), wl.fov,
                                  wl.support_aa, wl.beta, 0, tap_dtype, out, stream)
    else:
        raise ValueError(f"unknown kernel kind {wl.kernel}")
    return out


@dataclasses.dataclass
class DeviceWorkload:
    wl: object
    uvw: torch.Tensor
    vis: torch.Tensor
    weights: Optional[torch.Tensor]
    taps: torch.Tensor
    kernel: B.GrKernel
    tap_dtype: int
    vis_dtype: int = B.GR_F32
    vis_scale: Optional[torch.Tensor] = None

    @property
    def n_vis(self):
        return self.wl.n_vis

    @property
    def n_pol(self):
        return self.wl.n_pol


def upload(wl, device="cuda:0", tap_dtype: int = B.GR_F32, taps: Optional[torch.Tensor] = None,
           stream=None, vis_f16=None) -> DeviceWorkload:
    """vis_f16: optional (halves [N][P][2] float16, scales [ceil(N/256)] float32) encoding of the
    visibilities to pass instead of complex64."""
    uvw = torch.from_numpy(np.ascontiguousarray(wl.uvw)).to(device)
    scale = None
    if vis_f16 is None:
        vis = torch.from_numpy(np.ascontiguousarray(wl.vis)).to(device)
    else:
        vis = torch.from_numpy(np.ascontiguousarray(vis_f16[0])).to(device)
        scale = torch.from_numpy(np.ascontiguousarray(vis_f16[1], dtype=np.float32)).to(device)
    w = None if wl.weights is None else torch.from_numpy(np.ascontiguousarray(wl.weights)).to(device)
    if taps is None:
        taps = make_taps(wl, device, tap_dtype, stream)
    k = B.make_kernel(taps, wl.support, wl.oversample, wl.n_planes,
                      taps_complex=(wl.kernel != "kb"), tap_dtype=tap_dtype,
                      w_min=wl.w_min, inv_dw=wl.inv_dw,
                      kind=B.GR_TABLE2D if wl.kernel == "w2d" else B.GR_SEPARABLE)
    return DeviceWorkload(wl, uvw, vis, w, taps, k, tap_dtype,
                          B.GR_F32 if vis_f16 is None else B.GR_F16, scale)


def tuning(cu=0, cv=0, wg_u=0, wg_v=0, vis_per_wg=0, variant=0) -> B.GrTuning:
    return B.GrTuning(cu, cv, wg_u, wg_v, vis_per_wg, variant)


def grid(dw: DeviceWorkload, grid_out: Optional[torch.Tensor] = None,
         tune: Optional[B.GrTuning] = None, workspace: Optional[torch.Tensor] = None,
         stats: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
    """Run the whole path (preprocess + grid) into grid_out (zeros if None)."""
    wl = dw.wl
    dev = dw.uvw.device
    if grid_out is None:
        grid_out = torch.zeros((wl.n_pol, wl.height, wl.width), dtype=torch.complex64, device=dev)
    need = B.gr_grid_workspace_bytes(wl.n_vis, wl.n_pol, dw.kernel, wl.height, wl.width, tune)
    if workspace is None or workspace.numel() < need:
        workspace = torch.empty(max(need, 1), dtype=torch.uint8, device=dev)
    B.gr_grid(dw.uvw, dw.vis, dw.vis_dtype, dw.vis_scale, dw.weights, wl.n_vis, wl.n_pol, dw.kernel,
              wl.inv_cell_u, wl.inv_cell_v, grid_out, wl.height, wl.width, tune, workspace,
              workspace.numel(), stats, stream)
    return grid_out


def preprocess(dw: DeviceWorkload, stats: Optional[torch.Tensor] = None, stream=None):
    """gr_preprocess into fresh buffers: returns (records uint32 [N, 2], wvis complex64 [N, P])."""
    wl = dw.wl
    dev = dw.uvw.device
    rec = torch.empty((max(wl.n_vis, 1), 2), dtype=torch.int32, device=dev)
    wv = torch.empty((max(wl.n_vis, 1), wl.n_pol), dtype=torch.complex64, device=dev)
    B.gr_preprocess(dw.uvw, dw.vis, dw.vis_dtype, dw.vis_scale, dw.weights, wl.n_vis, wl.n_pol, dw.kernel,
                    wl.inv_cell_u, wl.inv_cell_v, wl.height, wl.width, rec, wv, stats, stream)
    return rec, wv


def decode_records(rec: np.ndarray) -> dict:
    """Unpack records (layout documented in include/gridder.h) for tests."""
    a = rec.view(np.uint32).reshape(-1, 2)
    x, y = a[:, 0].astype(np.int64), a[:, 1].astype(np.int64)
    return dict(x0=x & 0xFFFF, y0=x >> 16, sx=y & 0xFF, sy=(y >> 8) & 0xFF,
                plane=(y >> 16) & 0x7FFF, valid=(y >> 31) & 1)


def batch_items(dws, grids, seg_lens=None, stats=None):
    """gr_batch_item list for device workloads and their output grids."""
    items = []
    for i, (dw, g) in enumerate(zip(dws, grids)):
        wl = dw.wl
        items.append(B.make_batch_item(dw.uvw, dw.vis, dw.vis_dtype, wl.n_pol, dw.vis_scale, dw.weights,
                                       wl.n_vis, dw.kernel, wl.inv_cell_u, wl.inv_cell_v, g, wl.height,
                                       wl.width, seg_lens[i] if seg_lens else 0,
                                       None if stats is None else stats[i]))
    return items


def grid_batch(dws, grids=None, seg_lens=None, stats=None, workspace=None, stream=None):
    """Grid every device workload of a batch with one gr_grid_batch call; returns
    (grids, workspace)."""
    if grids is None:
        grids = [torch.zeros((dw.wl.n_pol, dw.wl.height, dw.wl.width), dtype=torch.complex64,
                             device=dw.uvw.device) for dw in dws]
    items = batch_items(dws, grids, seg_lens, stats)
    need = B.gr_grid_batch_workspace_bytes(items)
    if workspace is None or workspace.numel() < need:
        dev = dws[0].uvw.device if dws else "cuda"
        workspace = torch.empty(max(need, 1), dtype=torch.uint8, device=dev)
    B.gr_grid_batch(items, workspace, workspace.numel(), stream)
    return grids, workspace


class BatchGraph:
    """A batch captured by the library into one HIP graph (gr_grid_batch_graph);
    keeps the device workloads, grids and workspace alive."""

    def __init__(self, dws, grids, seg_lens=None, stats=None):
        self.dws, self.grids, self.stats = dws, grids, stats
        self.items = batch_items(dws, grids, seg_lens, stats)
        need = B.gr_grid_batch_workspace_bytes(self.items)
        dev = dws[0].uvw.device
        self.workspace = torch.empty(max(need, 1), dtype=torch.uint8, device=dev)
        self.handle = B.gr_grid_batch_graph(self.items, self.workspace, self.workspace.numel())

    def launch(self, stream=None):
        B.gr_graph_launch(self.handle, stream)

    def close(self):
        if self.handle:
            B.gr_graph_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def wslice_partition(dw: DeviceWorkload, w_first: float, inv_width: float, n_slices: int,
                     workspace: Optional[torch.Tensor] = None, stream=None):
    """gr_wslice_partition of a device workload into fresh buffers: returns
    (uvw, vis, weights or None, slice_offsets device int64 [n_slices + 1])."""
    if dw.vis_dtype != B.GR_F32:
        raise ValueError("gr_wslice_partition takes complex64 visibilities")
    wl = dw.wl
    dev = dw.uvw.device
    uvw_p = torch.empty_like(dw.uvw)
    vis_p = torch.empty_like(dw.vis)
    w_p = None if dw.weights is None else torch.empty_like(dw.weights)
    offs = torch.empty(n_slices + 1, dtype=torch.int64, device=dev)
    need = B.gr_wslice_partition_workspace_bytes(wl.n_vis, n_slices)
    if workspace is None or workspace.numel() < need:
        workspace = torch.empty(max(need, 1), dtype=torch.uint8, device=dev)
    B.gr_wslice_partition(dw.uvw, dw.vis, dw.weights, wl.n_vis, wl.n_pol, w_first, inv_width, n_slices,
                          uvw_p, vis_p, w_p, offs, workspace, workspace.numel(), stream)
    return uvw_p, vis_p, w_p, offs


def grid_wstack(dw: DeviceWorkload, w_first: float, inv_width: float, n_slices: int,
                grids: Optional[torch.Tensor] = None, mode: str = "batch", stream=None):
    """W-stacking: partition by w slice (gr_wslice_partition), then grid each
    slice into its own grid with dw.kernel's table, whose w_min is taken as
    relative to the slice centre (gr_wslice_kernel).  mode "batch": one
    gr_grid_batch over the slices; "per_slice": one gr_grid per slice.  The
    slice offsets are copied to the host (one synchronisation) to form the
    calls.  Returns (grids complex64 [n_slices][P][H][W], host offsets)."""
    wl = dw.wl
    dev = dw.uvw.device
    if grids is None:
        grids = torch.zeros((n_slices, wl.n_pol, wl.height, wl.width), dtype=torch.complex64, device=dev)
    uvw_p, vis_p, w_p, offs = wslice_partition(dw, w_first, inv_width, n_slices, stream=stream)
    off = offs.cpu().numpy()
    k = dw.kernel
    if mode == "batch":
        items = []
        for s in range(n_slices):
            a, b = int(off[s]), int(off[s + 1])
            items.append(B.make_batch_item(uvw_p[a:], vis_p[a:], B.GR_F32, wl.n_pol, None,
                                           None if w_p is None else w_p[a:], b - a,
                                           B.gr_wslice_kernel(k, w_first, inv_width, s),
                                           wl.inv_cell_u, wl.inv_cell_v, grids[s], wl.height, wl.width))
        need = B.gr_grid_batch_workspace_bytes(items)
        ws = torch.empty(max(need, 1), dtype=torch.uint8, device=dev)
        B.gr_grid_batch(items, ws, ws.numel(), stream)
    elif mode == "per_slice":
        ws = None
        for s in range(n_slices):
            a, b = int(off[s]), int(off[s + 1])
            if b == a:
                continue
            ks = B.gr_wslice_kernel(k, w_first, inv_width, s)
            need = B.gr_grid_workspace_bytes(b - a, wl.n_pol, ks, wl.height, wl.width, None)
            if ws is None or ws.numel() < need:
                ws = torch.empty(max(need, 1), dtype=torch.uint8, device=dev)
            B.gr_grid(uvw_p[a:], vis_p[a:], B.GR_F32, None, None if w_p is None else w_p[a:], b - a, wl.n_pol,
                      ks, wl.inv_cell_u, wl.inv_cell_v, grids[s], wl.height, wl.width, None, ws, ws.numel(),
                      None, stream)
    else:
        raise ValueError(f"unknown mode {mode}")
    return grids, off


def grid_aterm(dw: DeviceWorkload, kernel_id: torch.Tensor, n_ids: int, grid_out: Optional[torch.Tensor] = None,
               workspace: Optional[torch.Tensor] = None, stats: Optional[torch.Tensor] = None, stream=None):
    """gr_grid_aterm of a device workload whose kernel is a GR_TABLE2D descriptor of the
    per-id, per-polarisation table; kernel_id: device int32 [N].  Returns the grid."""
    wl = dw.wl
    dev = dw.uvw.device
    if grid_out is None:
        grid_out = torch.zeros((wl.n_pol, wl.height, wl.width), dtype=torch.complex64, device=dev)
    need = B.gr_grid_aterm_workspace_bytes(wl.n_vis, wl.n_pol, wl.support, wl.height, wl.width)
    if workspace is None or workspace.numel() < need:
        workspace = torch.empty(max(need, 1), dtype=torch.uint8, device=dev)
    B.gr_grid_aterm(dw.uvw, dw.vis, dw.vis_dtype, dw.vis_scale, dw.weights, kernel_id, n_ids, wl.n_vis, wl.n_pol,
                    dw.kernel, wl.inv_cell_u, wl.inv_cell_v, grid_out, wl.height, wl.width, workspace,
                    workspace.numel(), stats, stream)
    return grid_out
