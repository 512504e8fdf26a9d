"""ctypes binding to libgridder.so: argument marshalling only.

Every function has the name and argument order of the C entry point in
include/gridder.h.  Device buffers are torch tensors (their data pointers are
passed through); ``stream=None`` means torch's current stream on the
tensor's device.  A non-OK status raises :class:`GridderError` carrying the
library's message.  Nothing here computes any part of gridding.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libgridder.so")
_lib = None

GR_OK, GR_EINVAL, GR_ENOMEM, GR_EDEVICE, GR_EUNSUPPORTED = 0, -1, -2, -3, -4
GR_F32, GR_F16, GR_BF16, GR_F64 = 0, 1, 2, 3
GR_SEPARABLE, GR_TABLE2D, GR_MLP = 0, 1, 2
_STATUS = {GR_EINVAL: "EINVAL", GR_ENOMEM: "ENOMEM", GR_EDEVICE: "EDEVICE", GR_EUNSUPPORTED: "EUNSUPPORTED"}


class GridderError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{_STATUS.get(status, status)}: {message}")
        self.status = status


class GrKernel(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("tap_dtype", ctypes.c_int32),
                ("taps_complex", ctypes.c_int32), ("support", ctypes.c_int32),
                ("oversample", ctypes.c_int32), ("n_planes", ctypes.c_int32),
                ("w_min", ctypes.c_double), ("inv_dw", ctypes.c_double),
                ("taps", ctypes.c_void_p)]


class GrBatchItem(ctypes.Structure):
    _fields_ = [("uvw", ctypes.c_void_p), ("vis", ctypes.c_void_p), ("vis_dtype", ctypes.c_int32),
                ("n_pol", ctypes.c_int32), ("vis_scale", ctypes.c_void_p), ("weights", ctypes.c_void_p),
                ("n_vis", ctypes.c_int64), ("kernel", GrKernel), ("inv_cell_u", ctypes.c_double),
                ("inv_cell_v", ctypes.c_double), ("grid", ctypes.c_void_p), ("height", ctypes.c_int32),
                ("width", ctypes.c_int32), ("seg_len", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("dev_stats", ctypes.c_void_p)]


class GrTuning(ctypes.Structure):
    _fields_ = [("cu", ctypes.c_int32), ("cv", ctypes.c_int32), ("wg_u", ctypes.c_int32),
                ("wg_v", ctypes.c_int32), ("vis_per_wg", ctypes.c_int32),
                ("variant", ctypes.c_int32)]


def library_path() -> str:
    return _LIB_PATH


def load_library():
    """Load libgridder.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        raise GridderError(GR_EDEVICE, f"{_LIB_PATH} is missing: run __graft_entry__.build() "
                                       "(there is no CPU fallback)")
    lib = ctypes.CDLL(_LIB_PATH)
    P, I32, I64, D, SZ = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_size_t
    KP, TP = ctypes.POINTER(GrKernel), ctypes.POINTER(GrTuning)
    sigs = {
        "gr_preprocess": [P, P, I32, P, P, I64, I32, KP, D, D, I32, I32, P, P, P, P],
        "gr_grid_records": [P, P, I64, I32, KP, P, I32, I32, TP, P],
        "gr_grid": [P, P, I32, P, P, I64, I32, KP, D, D, P, I32, I32, TP, P, SZ, P, P],
        "gr_make_kb_table": [D, I32, I32, I32, P, P],
        "gr_make_wkernel_table": [I32, I32, I32, D, D, I32, D, I32, I32, P, P],
        "gr_bin": [P, P, I64, I32, I32, I32, I32, I32, P, SZ, P],
        "gr_preprocess_bin": [P, P, I32, P, P, I64, I32, KP, D, D, I32, I32, I32, P, SZ, P, P],
        "gr_degrid": [P, I64, I32, KP, D, D, P, I32, I32, P, I32, P, SZ, P, P],
        "gr_compress": [P, P, I64, I32, P, P, P, P, SZ, P],
        "gr_wslice_partition": [P, P, P, I64, I32, D, D, I32, P, P, P, P, P, SZ, P],
        "gr_grid_aterm": [P, P, I32, P, P, P, I32, I64, I32, KP, D, D, P, I32, I32, P, SZ, P, P],
        "gr_grid_binned": [P, I64, I32, KP, I32, P, I32, I32, P],
        "gr_autotune": [P, P, I64, I32, KP, P, I32, I32, P, SZ, TP, I32, I32, P, P, P],
        "gr_make_wkernel2d_table": [I32, I32, I32, D, D, D, I32, D, I32, I32, P, P],
        "gr_mlp_eval": [P, P, I64, P, P],
        "gr_mlp_dataset": [P, I32, I32, I32, D, D, D, ctypes.c_float, P, P, P],
        "gr_mlp_grads": [P, P, P, P, I32, P, P, P],
        "gr_mlp_train_step": [P, P, P, P, P, P, P, I32, I32, ctypes.c_float, P, P],
    }
    for name, args in sigs.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = ctypes.c_int
    lib.gr_grid_workspace_bytes.argtypes = [I64, I32, KP, I32, I32, TP]
    lib.gr_grid_workspace_bytes.restype = SZ
    lib.gr_bin_bytes.argtypes = [I64, I32, I32, I32, I32, I32]
    lib.gr_bin_bytes.restype = SZ
    lib.gr_preprocess_bin_bytes.argtypes = [I64, I32, I32, I32, I32, I32]
    lib.gr_preprocess_bin_bytes.restype = SZ
    lib.gr_degrid_workspace_bytes.argtypes = [I64, I32, I32, I32, I32, I32]
    lib.gr_degrid_workspace_bytes.restype = SZ
    lib.gr_compress_workspace_bytes.argtypes = [I64]
    lib.gr_compress_workspace_bytes.restype = SZ
    lib.gr_wslice_partition_workspace_bytes.argtypes = [I64, I32]
    lib.gr_wslice_partition_workspace_bytes.restype = SZ
    lib.gr_grid_aterm_workspace_bytes.argtypes = [I64, I32, I32, I32, I32]
    lib.gr_grid_aterm_workspace_bytes.restype = SZ
    lib.gr_last_error.argtypes = []
    lib.gr_last_error.restype = ctypes.c_char_p
    lib.gr_grid_batch.argtypes = [ctypes.POINTER(GrBatchItem), I32, P, SZ, P]
    lib.gr_grid_batch.restype = ctypes.c_int
    lib.gr_grid_batch_workspace_bytes.argtypes = [ctypes.POINTER(GrBatchItem), I32]
    lib.gr_grid_batch_workspace_bytes.restype = SZ
    lib.gr_grid_batch_graph.argtypes = [ctypes.POINTER(GrBatchItem), I32, P, SZ, ctypes.POINTER(ctypes.c_void_p)]
    lib.gr_grid_batch_graph.restype = ctypes.c_int
    lib.gr_graph_launch.argtypes = [P, P]
    lib.gr_graph_launch.restype = ctypes.c_int
    lib.gr_graph_destroy.argtypes = [P]
    lib.gr_graph_destroy.restype = ctypes.c_int
    lib.gr_mlp_blob_floats.argtypes = []
    lib.gr_mlp_blob_floats.restype = I32
    lib.gr_version.argtypes = []
    lib.gr_version.restype = I32
    lib.gr_tuning_memo_put.argtypes = [I32, KP, I32, I32, I32, TP]
    lib.gr_tuning_memo_put.restype = ctypes.c_int
    lib.gr_tuning_memo_get.argtypes = [I32, KP, I32, I32, I32, TP]
    lib.gr_tuning_memo_get.restype = ctypes.c_int
    lib.gr_tuning_memo_clear.argtypes = []
    lib.gr_tuning_memo_clear.restype = None
    lib.gr_wslice_kernel.argtypes = [KP, D, D, I32, KP]
    lib.gr_wslice_kernel.restype = ctypes.c_int
    lib.gr_grid_noalloc.argtypes = [P, P, I32, P, P, I64, I32, KP, D, D, P, I32, I32, TP, P, P]
    lib.gr_grid_noalloc.restype = ctypes.c_int
    lib.gr_grid_noalloc_scratch_bytes.argtypes = []
    lib.gr_grid_noalloc_scratch_bytes.restype = SZ
    _lib = lib
    return lib


def _ptr(t) -> Optional[int]:
    if t is None:
        return None
    if isinstance(t, int):
        return t
    return t.data_ptr()


def _stream(stream, *tensors):
    if stream is not None:
        return stream if isinstance(stream, int) else stream.cuda_stream
    import torch
    dev = next((t.device for t in tensors if t is not None and hasattr(t, "device")), None)
    return torch.cuda.current_stream(dev).cuda_stream


def _check(st: int) -> None:
    if st != GR_OK:
        raise GridderError(st, load_library().gr_last_error().decode())


def gr_version() -> int:
    return int(load_library().gr_version())


def gr_last_error() -> str:
    return load_library().gr_last_error().decode()


def gr_tuning_memo_put(n_pol: int, kernel: GrKernel, height: int, width: int, slot: int,
                       tuning: GrTuning) -> None:
    _check(load_library().gr_tuning_memo_put(n_pol, ctypes.byref(kernel), height, width, slot,
                                             ctypes.byref(tuning)))


def gr_tuning_memo_get(n_pol: int, kernel: GrKernel, height: int, width: int, slot: int) -> Optional[GrTuning]:
    """The memo's entry, or None when there is none."""
    out = GrTuning()
    st = load_library().gr_tuning_memo_get(n_pol, ctypes.byref(kernel), height, width, slot, ctypes.byref(out))
    if st == GR_EINVAL and "no entry" in gr_last_error():
        return None
    _check(st)
    return out


def gr_tuning_memo_clear() -> None:
    load_library().gr_tuning_memo_clear()


def gr_wslice_kernel(table: GrKernel, w_first: float, inv_width: float, slice_index: int) -> GrKernel:
    out = GrKernel()
    _check(load_library().gr_wslice_kernel(ctypes.byref(table), w_first, inv_width, slice_index,
                                           ctypes.byref(out)))
    return out


def gr_grid_workspace_bytes(n_vis: int, n_pol: int, kernel: GrKernel, height: int, width: int,
                            tuning: Optional[GrTuning] = None) -> int:
    return int(load_library().gr_grid_workspace_bytes(
        n_vis, n_pol, ctypes.byref(kernel), height, width,
        ctypes.byref(tuning) if tuning is not None else None))


def gr_bin_bytes(n_vis: int, n_pol: int, support: int, height: int, width: int, seg_len: int = 0) -> int:
    return int(load_library().gr_bin_bytes(n_vis, n_pol, support, height, width, seg_len))


def gr_bin(records, wvis, n_vis, n_pol, support, height, width, seg_len, bins, bins_bytes, stream=None):
    _check(load_library().gr_bin(_ptr(records), _ptr(wvis), n_vis, n_pol, support, height, width,
                                 seg_len, _ptr(bins), bins_bytes, _stream(stream, bins)))


def gr_preprocess_bin_bytes(n_vis: int, n_pol: int, support: int, height: int, width: int,
                            seg_len: int = 0) -> int:
    return int(load_library().gr_preprocess_bin_bytes(n_vis, n_pol, support, height, width, seg_len))


def gr_preprocess_bin(uvw, vis, vis_dtype, vis_scale, weights, n_vis, n_pol, kernel: GrKernel, inv_cell_u,
                      inv_cell_v, height, width, seg_len, bins, bins_bytes, dev_stats, stream=None):
    _check(load_library().gr_preprocess_bin(_ptr(uvw), _ptr(vis), vis_dtype, _ptr(vis_scale), _ptr(weights),
                                            n_vis, n_pol, ctypes.byref(kernel), inv_cell_u, inv_cell_v, height,
                                            width, seg_len, _ptr(bins), bins_bytes, _ptr(dev_stats),
                                            _stream(stream, uvw, vis, bins)))


def gr_compress_workspace_bytes(n_vis: int) -> int:
    return int(load_library().gr_compress_workspace_bytes(n_vis))


def gr_compress(records, wvis, n_vis, n_pol, out_records, out_wvis, out_count, workspace, workspace_bytes,
                stream=None):
    _check(load_library().gr_compress(_ptr(records), _ptr(wvis), n_vis, n_pol, _ptr(out_records), _ptr(out_wvis),
                                      _ptr(out_count), _ptr(workspace), workspace_bytes,
                                      _stream(stream, records, out_records)))


def gr_wslice_partition_workspace_bytes(n_vis: int, n_slices: int) -> int:
    return int(load_library().gr_wslice_partition_workspace_bytes(n_vis, n_slices))


def gr_wslice_partition(uvw, vis, weights, n_vis, n_pol, w_first, inv_width, n_slices, uvw_out, vis_out,
                        weights_out, slice_offsets, workspace, workspace_bytes, stream=None):
    _check(load_library().gr_wslice_partition(_ptr(uvw), _ptr(vis), _ptr(weights), n_vis, n_pol, w_first,
                                              inv_width, n_slices, _ptr(uvw_out), _ptr(vis_out),
                                              _ptr(weights_out), _ptr(slice_offsets), _ptr(workspace),
                                              workspace_bytes, _stream(stream, uvw, slice_offsets)))


def gr_grid_aterm_workspace_bytes(n_vis: int, n_pol: int, support: int, height: int, width: int) -> int:
    return int(load_library().gr_grid_aterm_workspace_bytes(n_vis, n_pol, support, height, width))


def gr_grid_aterm(uvw, vis, vis_dtype, vis_scale, weights, kernel_id, n_ids, n_vis, n_pol, kernel: GrKernel,
                  inv_cell_u, inv_cell_v, grid, height, width, workspace, workspace_bytes, dev_stats=None,
                  stream=None):
    _check(load_library().gr_grid_aterm(_ptr(uvw), _ptr(vis), vis_dtype, _ptr(vis_scale), _ptr(weights),
                                        _ptr(kernel_id), n_ids, n_vis, n_pol, ctypes.byref(kernel), inv_cell_u,
                                        inv_cell_v, _ptr(grid), height, width, _ptr(workspace), workspace_bytes,
                                        _ptr(dev_stats), _stream(stream, grid, uvw)))


def gr_degrid_workspace_bytes(n_vis: int, n_pol: int, support: int, height: int, width: int,
                              seg_len: int = 0) -> int:
    return int(load_library().gr_degrid_workspace_bytes(n_vis, n_pol, support, height, width, seg_len))


def gr_degrid(uvw, n_vis, n_pol, kernel: GrKernel, inv_cell_u, inv_cell_v, grid, height, width, vis_out,
              seg_len, workspace, workspace_bytes, dev_stats=None, stream=None):
    _check(load_library().gr_degrid(_ptr(uvw), n_vis, n_pol, ctypes.byref(kernel), inv_cell_u, inv_cell_v,
                                    _ptr(grid), height, width, _ptr(vis_out), seg_len, _ptr(workspace),
                                    workspace_bytes, _ptr(dev_stats), _stream(stream, grid, vis_out)))


def gr_grid_binned(bins, n_vis, n_pol, kernel: GrKernel, seg_len, grid, height, width, stream=None):
    _check(load_library().gr_grid_binned(_ptr(bins), n_vis, n_pol, ctypes.byref(kernel), seg_len,
                                         _ptr(grid), height, width, _stream(stream, grid)))


def make_kernel(taps, support: int, oversample: int, n_planes: int = 1, taps_complex: bool = True,
                tap_dtype: int = GR_F32, w_min: float = 0.0, inv_dw: float = 0.0,
                kind: int = GR_SEPARABLE) -> GrKernel:
    """Fill a gr_kernel descriptor; ``taps`` is a device tensor (kept alive by the caller)."""
    return GrKernel(kind, tap_dtype, 1 if taps_complex else 0, support, oversample, n_planes,
                    w_min, inv_dw, _ptr(taps))


def gr_preprocess(uvw, vis, vis_dtype, vis_scale, weights, n_vis, n_pol, kernel: GrKernel,
                  inv_cell_u, inv_cell_v, height, width, records, wvis, dev_stats, stream=None):
    lib = load_library()
    _check(lib.gr_preprocess(_ptr(uvw), _ptr(vis), vis_dtype, _ptr(vis_scale), _ptr(weights),
                             n_vis, n_pol, ctypes.byref(kernel), inv_cell_u, inv_cell_v, height,
                             width, _ptr(records), _ptr(wvis), _ptr(dev_stats),
                             _stream(stream, uvw, vis, records)))


def gr_grid_records(records, wvis, n_vis, n_pol, kernel: GrKernel, grid, height, width,
                    tuning: Optional[GrTuning] = None, stream=None):
    lib = load_library()
    _check(lib.gr_grid_records(_ptr(records), _ptr(wvis), n_vis, n_pol, ctypes.byref(kernel),
                               _ptr(grid), height, width,
                               ctypes.byref(tuning) if tuning is not None else None,
                               _stream(stream, grid)))


def gr_grid(uvw, vis, vis_dtype, vis_scale, weights, n_vis, n_pol, kernel: GrKernel, inv_cell_u,
            inv_cell_v, grid, height, width, tuning: Optional[GrTuning], workspace,
            workspace_bytes, dev_stats, stream=None):
    lib = load_library()
    _check(lib.gr_grid(_ptr(uvw), _ptr(vis), vis_dtype, _ptr(vis_scale), _ptr(weights), n_vis,
                       n_pol, ctypes.byref(kernel), inv_cell_u, inv_cell_v, _ptr(grid), height,
                       width, ctypes.byref(tuning) if tuning is not None else None,
                       _ptr(workspace), workspace_bytes, _ptr(dev_stats),
                       _stream(stream, grid, uvw)))


def gr_grid_noalloc(uvw, vis, vis_dtype, vis_scale, weights, n_vis, n_pol, kernel: GrKernel, inv_cell_u,
                    inv_cell_v, grid, height, width, tuning: Optional[GrTuning], dev_stats, stream=None):
    lib = load_library()
    _check(lib.gr_grid_noalloc(_ptr(uvw), _ptr(vis), vis_dtype, _ptr(vis_scale), _ptr(weights), n_vis,
                               n_pol, ctypes.byref(kernel), inv_cell_u, inv_cell_v, _ptr(grid), height,
                               width, ctypes.byref(tuning) if tuning is not None else None,
                               _ptr(dev_stats), _stream(stream, grid, uvw)))


def gr_grid_noalloc_scratch_bytes() -> int:
    return int(load_library().gr_grid_noalloc_scratch_bytes())


def gr_make_kb_table(beta, support, oversample, out_dtype, out, stream=None):
    _check(load_library().gr_make_kb_table(beta, support, oversample, out_dtype, _ptr(out),
                                           _stream(stream, out)))


def gr_make_wkernel_table(support, oversample, n_planes, w_hat_first, w_hat_step, support_aa,
                          beta, n_samples, out_dtype, out, stream=None):
    _check(load_library().gr_make_wkernel_table(support, oversample, n_planes, w_hat_first,
                                                w_hat_step, support_aa, beta, n_samples,
                                                out_dtype, _ptr(out), _stream(stream, out)))


def gr_autotune(records, wvis, n_vis, n_pol, kernel: GrKernel, grid, height, width, bins,
                bins_bytes, candidates, reps: int = 3, stream=None):
    """Returns (best index, list of mean times in ms; inf for unsupported candidates)."""
    n = len(candidates)
    arr = (GrTuning * n)(*candidates)
    times = (ctypes.c_float * n)()
    best = ctypes.c_int32(-1)
    _check(load_library().gr_autotune(_ptr(records), _ptr(wvis), n_vis, n_pol, ctypes.byref(kernel),
                                      _ptr(grid), height, width, _ptr(bins), bins_bytes, arr, n, reps,
                                      ctypes.cast(times, ctypes.c_void_p),
                                      ctypes.cast(ctypes.pointer(best), ctypes.c_void_p),
                                      _stream(stream, grid)))
    return int(best.value), [float(t) for t in times]


def gr_make_wkernel2d_table(support, oversample, n_planes, w_hat_first, w_hat_step, fov, support_aa,
                            beta, n_samples, out_dtype, out, stream=None):
    _check(load_library().gr_make_wkernel2d_table(support, oversample, n_planes, w_hat_first,
                                                  w_hat_step, fov, support_aa, beta, n_samples,
                                                  out_dtype, _ptr(out), _stream(stream, out)))


def gr_mlp_blob_floats() -> int:
    return int(load_library().gr_mlp_blob_floats())


def gr_mlp_eval(weights, inputs, n, out, stream=None):
    _check(load_library().gr_mlp_eval(_ptr(weights), _ptr(inputs), n, _ptr(out), _stream(stream, out)))


def gr_mlp_dataset(table2d, support, oversample, n_planes, w_hat_first, w_hat_step, w_hat_max,
                   out_scale, inputs, targets, stream=None):
    _check(load_library().gr_mlp_dataset(_ptr(table2d), support, oversample, n_planes, w_hat_first,
                                         w_hat_step, w_hat_max, out_scale, _ptr(inputs),
                                         _ptr(targets), _stream(stream, inputs)))


def gr_mlp_grads(weights, inputs, targets, idx, batch, grads, loss_sum, stream=None):
    _check(load_library().gr_mlp_grads(_ptr(weights), _ptr(inputs), _ptr(targets), _ptr(idx), batch,
                                       _ptr(grads), _ptr(loss_sum), _stream(stream, grads)))


def gr_mlp_train_step(weights, adam_m, adam_v, grads, inputs, targets, idx, batch, step, lr,
                      loss_sum, stream=None):
    _check(load_library().gr_mlp_train_step(_ptr(weights), _ptr(adam_m), _ptr(adam_v), _ptr(grads),
                                            _ptr(inputs), _ptr(targets), _ptr(idx), batch, step, lr,
                                            _ptr(loss_sum), _stream(stream, weights)))


def make_batch_item(uvw, vis, vis_dtype, n_pol, vis_scale, weights, n_vis, kernel: GrKernel, inv_cell_u,
                    inv_cell_v, grid, height, width, seg_len=0, dev_stats=None) -> GrBatchItem:
    """Fill a gr_batch_item; the tensors are kept alive by the caller."""
    return GrBatchItem(_ptr(uvw), _ptr(vis), vis_dtype, n_pol, _ptr(vis_scale), _ptr(weights), n_vis,
                       kernel, inv_cell_u, inv_cell_v, _ptr(grid), height, width, seg_len, 0,
                       _ptr(dev_stats))


def gr_grid_batch_workspace_bytes(items) -> int:
    arr = (GrBatchItem * max(len(items), 1))(*items)
    return int(load_library().gr_grid_batch_workspace_bytes(arr, len(items)))


def gr_grid_batch(items, workspace, workspace_bytes, stream=None):
    arr = (GrBatchItem * max(len(items), 1))(*items)
    _check(load_library().gr_grid_batch(arr, len(items), _ptr(workspace), workspace_bytes,
                                        _stream(stream, workspace)))


def gr_grid_batch_graph(items, workspace, workspace_bytes) -> int:
    """Capture the batch into a HIP graph; returns the opaque handle (an int)."""
    arr = (GrBatchItem * max(len(items), 1))(*items)
    h = ctypes.c_void_p(None)
    _check(load_library().gr_grid_batch_graph(arr, len(items), _ptr(workspace), workspace_bytes,
                                              ctypes.byref(h)))
    return h.value


def gr_graph_launch(handle, stream=None):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream().cuda_stream
    if not isinstance(s, int):
        s = s.cuda_stream
    _check(load_library().gr_graph_launch(handle, s))


def gr_graph_destroy(handle):
    _check(load_library().gr_graph_destroy(handle))
