"""Host-side checks of the C ABI: the library loads, exports every declared
entry point, and rejects bad arguments on the host before anything is
enqueued (no device work happens in this file)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = set()
    for f in os.listdir(os.path.join(ROOT, "include")):
        if f.endswith(".h"):
            txt = open(os.path.join(ROOT, "include", f)).read()
            names |= set(re.findall(r"^\s*(?:gr_status|size_t|int32_t|void|const char\*)\s+(gr_\w+)\(", txt, re.M))
    return sorted(names)


@pytest.fixture(scope="module")
def lib():
    from paper_1605_07023_amd import binding
    path = binding.library_path()
    if not os.path.exists(path):
        import __graft_entry__
        __graft_entry__.build()
    return binding.load_library()


def test_every_declared_symbol_is_exported(lib):
    names = _declared()
    assert len(names) >= 8
    for n in names:
        assert hasattr(lib, n), n


def test_version_and_workspace(lib):
    from paper_1605_07023_amd import binding as B
    assert B.gr_version() >= 1
    k = _kernel()
    n1 = B.gr_grid_workspace_bytes(1000, 4, k, 64, 64, B.GrTuning(0, 0, 0, 0, 0, 1))
    assert n1 >= 1000 * 8 + 1000 * 4 * 8
    # the binned path preprocesses and bins in one fused pass: the bins plus the unbinned records
    n2 = B.gr_grid_workspace_bytes(1000, 4, k, 64, 64)
    assert n2 == B.gr_preprocess_bin_bytes(1000, 4, 16, 64, 64)
    assert n2 >= B.gr_bin_bytes(1000, 4, 16, 64, 64) + 1000 * 8
    assert B.gr_grid_workspace_bytes(-1, 4, k, 64, 64) == 0
    assert B.gr_bin_bytes(10, 4, 58, 64, 64) == 0
    assert B.gr_preprocess_bin_bytes(10, 4, 58, 64, 64) == 0
    assert B.gr_preprocess_bin_bytes(-1, 4, 16, 64, 64) == 0


def _kernel(**kw):
    from paper_1605_07023_amd import binding as B
    base = dict(kind=B.GR_SEPARABLE, tap_dtype=B.GR_F32, taps_complex=1, support=16, oversample=8,
                n_planes=4, w_min=-1.0, inv_dw=1.5, taps=1 << 20)
    base.update(kw)
    return B.GrKernel(**base)


@pytest.mark.parametrize("bad,msg", [
    (dict(support=7), "support"), (dict(support=0), "support"), (dict(support=66), "support"),
    (dict(oversample=6), "oversample"), (dict(oversample=256), "oversample"),
    (dict(n_planes=0), "n_planes"), (dict(tap_dtype=9), "tap_dtype"),
    (dict(taps=None), "taps"), (dict(kind=1), "separable"), (dict(kind=5), "kernel.kind"),
    (dict(w_min=float("nan")), "w_min"),
])
def test_grid_records_rejects_bad_kernel(lib, bad, msg):
    from paper_1605_07023_amd import binding as B
    k = _kernel(**bad)
    st = lib.gr_grid_records(1 << 20, 1 << 20, 10, 4, ctypes.byref(k), 1 << 20, 64, 64, None, None)
    assert st in (B.GR_EINVAL, B.GR_EUNSUPPORTED)
    assert msg in lib.gr_last_error().decode()


@pytest.mark.parametrize("args,msg", [
    (dict(n_pol=3), "n_pol"), (dict(height=8), "height"), (dict(width=40000), "height"),
    (dict(n_vis=-1), "n_vis"), (dict(grid=None), "grid"), (dict(records=None), "records"),
])
def test_grid_records_rejects_bad_shapes(lib, args, msg):
    from paper_1605_07023_amd import binding as B
    a = dict(records=1 << 20, wvis=1 << 20, n_vis=10, n_pol=4, grid=1 << 20, height=64, width=64)
    a.update(args)
    k = _kernel()
    st = lib.gr_grid_records(a["records"], a["wvis"], a["n_vis"], a["n_pol"], ctypes.byref(k),
                             a["grid"], a["height"], a["width"], None, None)
    assert st == B.GR_EINVAL
    assert msg in lib.gr_last_error().decode()


def test_tuning_validation(lib):
    from paper_1605_07023_amd import binding as B
    k = _kernel()
    for t, code in [(B.GrTuning(3, 2, 0, 0, 0, 0), B.GR_EINVAL),
                    (B.GrTuning(8, 8, 0, 0, 0, 0), B.GR_EUNSUPPORTED),
                    (B.GrTuning(2, 2, 65, 1, 0, 0), B.GR_EINVAL),
                    (B.GrTuning(0, 0, 0, 0, 0, 7), B.GR_EUNSUPPORTED)]:
        st = lib.gr_grid_records(1 << 20, 1 << 20, 10, 4, ctypes.byref(k), 1 << 20, 64, 64,
                                 ctypes.byref(t), None)
        assert st == code, (t.cu, t.cv, t.wg_u, t.wg_v, t.variant, lib.gr_last_error())


def test_grid_rejects_small_workspace(lib):
    from paper_1605_07023_amd import binding as B
    k = _kernel()
    st = lib.gr_grid(1 << 20, 1 << 20, B.GR_F32, None, None, 100, 4, ctypes.byref(k), 1.0, 1.0,
                     1 << 20, 64, 64, None, 1 << 20, 10, None, None)
    assert st == B.GR_ENOMEM


@pytest.mark.parametrize("S", [58, 62, 64])
@pytest.mark.parametrize("kind,variant", [(1, 0), (2, 0), (0, 2)])
def test_binned_paths_reject_supports_past_56(lib, S, kind, variant):
    """Supports 58..64 pass the kernel descriptor's rule (2..64) but no binned
    gridder's window holds them: the workspace query answers 0 and every
    binned entry point refuses on the host (no division by a zero tile)."""
    from paper_1605_07023_amd import binding as B
    k = _kernel(kind=kind, support=S, tap_dtype=B.GR_F32, taps_complex=1)
    t = B.GrTuning(0, 0, 0, 0, 0, variant)
    assert B.gr_grid_workspace_bytes(1000, 1, k, 128, 128, t) == 0
    st = lib.gr_grid(1 << 20, 1 << 20, B.GR_F32, None, None, 1000, 1, ctypes.byref(k), 1.0, 1.0,
                     1 << 20, 128, 128, ctypes.byref(t), 1 << 20, 1 << 30, None, None)
    assert st == B.GR_EUNSUPPORTED and "56" in lib.gr_last_error().decode()
    st = lib.gr_grid_binned(1 << 20, 1000, 1, ctypes.byref(k), 0, 1 << 20, 128, 128, None)
    assert st == B.GR_EUNSUPPORTED and "56" in lib.gr_last_error().decode()


def test_preprocess_rejects(lib):
    from paper_1605_07023_amd import binding as B
    k = _kernel()
    st = lib.gr_preprocess(1 << 20, 1 << 20, B.GR_F16, None, None, 10, 4, ctypes.byref(k), 1.0, 1.0,
                           64, 64, 1 << 20, 1 << 20, None, None)
    assert st == B.GR_EINVAL and "vis_scale" in lib.gr_last_error().decode()
    st = lib.gr_preprocess(1 << 20, 1 << 20, B.GR_F32, None, None, 10, 4, ctypes.byref(k), 0.0, 1.0,
                           64, 64, 1 << 20, 1 << 20, None, None)
    assert st == B.GR_EINVAL and "inv_cell" in lib.gr_last_error().decode()


def test_preprocess_bin_rejects(lib):
    """Host-side validation of gr_preprocess_bin, before anything is enqueued."""
    from paper_1605_07023_amd import binding as B
    k = _kernel()
    need = B.gr_preprocess_bin_bytes(10, 4, 16, 64, 64, 0)
    call = lambda *a: lib.gr_preprocess_bin(*a)
    st = call(1 << 20, 1 << 20, B.GR_F32, None, None, 10, 4, ctypes.byref(k), 1.0, 1.0, 64, 64, 0,
              1 << 20, need - 1, None, None)
    assert st == B.GR_ENOMEM and "gr_preprocess_bin_bytes" in lib.gr_last_error().decode()
    st = call(1 << 20, 1 << 20, B.GR_F32, None, None, 10, 4, ctypes.byref(k), 1.0, 1.0, 64, 64, 0,
              None, need, None, None)
    assert st == B.GR_EINVAL and "bins" in lib.gr_last_error().decode()
    st = call(1 << 20, 1 << 20, B.GR_F16, None, None, 10, 4, ctypes.byref(k), 1.0, 1.0, 64, 64, 0,
              1 << 20, need, None, None)
    assert st == B.GR_EINVAL and "vis_scale" in lib.gr_last_error().decode()
    st = call(None, 1 << 20, B.GR_F32, None, None, 10, 4, ctypes.byref(k), 1.0, 1.0, 64, 64, 0,
              1 << 20, need, None, None)
    assert st == B.GR_EINVAL and "uvw" in lib.gr_last_error().decode()
    st = call(1 << 20, 1 << 20, B.GR_F32, None, None, 10, 3, ctypes.byref(k), 1.0, 1.0, 64, 64, 0,
              1 << 20, need, None, None)
    assert st == B.GR_EINVAL and "n_pol" in lib.gr_last_error().decode()


def test_degrid_rejects(lib):
    """Host-side validation of gr_degrid, before anything is enqueued."""
    from paper_1605_07023_amd import binding as B
    k = _kernel()
    need = B.gr_degrid_workspace_bytes(10, 4, 16, 64, 64, 0)
    assert need >= B.gr_bin_bytes(10, 4, 16, 64, 64) + 80
    st = lib.gr_degrid(1 << 20, 10, 4, ctypes.byref(k), 1.0, 1.0, 1 << 20, 64, 64, 1 << 20, 0, 1 << 20, need - 1,
                       None, None)
    assert st == B.GR_ENOMEM and "gr_degrid_workspace_bytes" in lib.gr_last_error().decode()
    st = lib.gr_degrid(1 << 20, 10, 3, ctypes.byref(k), 1.0, 1.0, 1 << 20, 64, 64, 1 << 20, 0, 1 << 20, need,
                       None, None)
    assert st == B.GR_EINVAL and "n_pol" in lib.gr_last_error().decode()
    st = lib.gr_degrid(1 << 20, 10, 4, ctypes.byref(k), 1.0, 1.0, None, 64, 64, 1 << 20, 0, 1 << 20, need,
                       None, None)
    assert st == B.GR_EINVAL and "grid" in lib.gr_last_error().decode()
    big = _kernel()
    big.n_planes = 400                 # (Re, Im) table of 400 x 8 x 18 entries: beyond LDS with the window
    st = lib.gr_degrid(1 << 20, 10, 4, ctypes.byref(big), 1.0, 1.0, 1 << 20, 64, 64, 1 << 20, 0, 1 << 20, need,
                       None, None)
    assert st == B.GR_EUNSUPPORTED and "LDS" in lib.gr_last_error().decode()
    t2 = _kernel()
    t2.kind = B.GR_TABLE2D
    st = lib.gr_degrid(1 << 20, 10, 4, ctypes.byref(t2), 1.0, 1.0, 1 << 20, 64, 64, 1 << 20, 0, 1 << 20, need,
                       None, None)
    assert st == B.GR_EUNSUPPORTED


def test_compress_rejects(lib):
    """Host-side validation of gr_compress, before anything is enqueued."""
    from paper_1605_07023_amd import binding as B
    nw = B.gr_compress_workspace_bytes(1000)
    assert nw >= 4 * 4 and B.gr_compress_workspace_bytes(-1) == 0
    a, b, c, d = 1 << 20, 1 << 24, 1 << 28, 1 << 32
    st = lib.gr_compress(a, b, 1000, 4, c, d, None, 1 << 36, nw - 1, None)
    assert st == B.GR_ENOMEM and "gr_compress_workspace_bytes" in lib.gr_last_error().decode()
    st = lib.gr_compress(a, b, 1000, 4, a + 800, d, None, 1 << 36, nw, None)    # out_records overlaps records
    assert st == B.GR_EINVAL and "overlap" in lib.gr_last_error().decode()
    st = lib.gr_compress(a, None, 1000, 4, c, d, None, 1 << 36, nw, None)
    assert st == B.GR_EINVAL and "non-NULL" in lib.gr_last_error().decode()
    st = lib.gr_compress(a, b, 1000, 2, c, d, None, 1 << 36, nw, None)
    assert st == B.GR_EINVAL and "n_pol" in lib.gr_last_error().decode()


def test_wslice_partition_rejects(lib):
    """Host-side validation of gr_wslice_partition, before anything is enqueued."""
    from paper_1605_07023_amd import binding as B
    nw = B.gr_wslice_partition_workspace_bytes(1000, 7)
    assert nw >= 4 * 8 * 4 and B.gr_wslice_partition_workspace_bytes(-1, 7) == 0
    assert B.gr_wslice_partition_workspace_bytes(10, 0) == 0 and B.gr_wslice_partition_workspace_bytes(10, 256) == 0
    u, v, w, uo, vo, wo, off, ws = (1 << k for k in (20, 24, 28, 32, 36, 40, 44, 46))

    def call(**kw):
        a = dict(uvw=u, vis=v, weights=w, n=1000, n_pol=4, w_first=-10.0, inv_width=0.1, n_slices=7,
                 uvw_out=uo, vis_out=vo, weights_out=wo, offsets=off, ws=ws, ws_bytes=nw)
        a.update(kw)
        st = lib.gr_wslice_partition(a["uvw"], a["vis"], a["weights"], a["n"], a["n_pol"], a["w_first"],
                                     a["inv_width"], a["n_slices"], a["uvw_out"], a["vis_out"],
                                     a["weights_out"], a["offsets"], a["ws"], a["ws_bytes"], None)
        return st, lib.gr_last_error().decode()

    st, msg = call(ws_bytes=nw - 1)
    assert st == B.GR_ENOMEM and "gr_wslice_partition_workspace_bytes" in msg
    st, msg = call(n_slices=0)
    assert st == B.GR_EINVAL and "n_slices" in msg
    st, msg = call(n_slices=256)
    assert st == B.GR_EINVAL and "n_slices" in msg
    st, msg = call(inv_width=0.0)
    assert st == B.GR_EINVAL and "inv_width" in msg
    st, msg = call(w_first=float("nan"))
    assert st == B.GR_EINVAL and "w_first" in msg
    st, msg = call(weights_out=None)
    assert st == B.GR_EINVAL and "weights_out" in msg
    st, msg = call(vis_out=u + 8)                                     # vis_out overlaps uvw
    assert st == B.GR_EINVAL and "overlap" in msg
    st, msg = call(offsets=v + 16)                                    # slice_offsets inside vis
    assert st == B.GR_EINVAL and "overlap" in msg
    st, msg = call(offsets=None)
    assert st == B.GR_EINVAL and "slice_offsets" in msg
    st, msg = call(n_pol=2)
    assert st == B.GR_EINVAL and "n_pol" in msg
    st, msg = call(n=-1)
    assert st == B.GR_EINVAL and "n_vis" in msg


def test_grid_aterm_rejects(lib):
    """Host-side validation of gr_grid_aterm, before anything is enqueued."""
    import ctypes
    from paper_1605_07023_amd import binding as B
    nw = B.gr_grid_aterm_workspace_bytes(1000, 4, 16, 512, 512)
    assert nw > 0 and B.gr_grid_aterm_workspace_bytes(-1, 4, 16, 512, 512) == 0
    assert B.gr_grid_aterm_workspace_bytes(10, 4, 64, 512, 512) == 0
    k = B.make_kernel(1 << 40, 16, 8, 4, taps_complex=True, w_min=-1.0, inv_dw=1.5, kind=B.GR_TABLE2D)

    def call(kern=k, ids=1 << 30, n_ids=16, n=1000, ws_bytes=nw, grid=1 << 34):
        st = lib.gr_grid_aterm(1 << 20, 1 << 24, B.GR_F32, None, None, ids, n_ids, n, 4, ctypes.byref(kern), 1.0,
                               1.0, grid, 512, 512, 1 << 36, ws_bytes, None, None)
        return st, lib.gr_last_error().decode()

    st, msg = call(ws_bytes=nw - 1)
    assert st == B.GR_ENOMEM and "gr_grid_aterm_workspace_bytes" in msg
    st, msg = call(ids=None)
    assert st == B.GR_EINVAL and "kernel_id" in msg
    st, msg = call(n_ids=0)
    assert st == B.GR_EINVAL and "n_ids" in msg
    st, msg = call(n_ids=8192)                                   # 8192 x 4 planes > 32767
    assert st == B.GR_EINVAL and "n_ids" in msg
    sep = B.make_kernel(1 << 40, 16, 8, 4, taps_complex=True, w_min=-1.0, inv_dw=1.5)
    st, msg = call(kern=sep)
    assert st == B.GR_EUNSUPPORTED and "GR_TABLE2D" in msg
    st, msg = call(grid=None)
    assert st == B.GR_EINVAL and "grid" in msg


def test_table_generators_reject(lib):
    from paper_1605_07023_amd import binding as B
    assert lib.gr_make_kb_table(8.6, 7, 8, B.GR_F32, 1 << 20, None) == B.GR_EINVAL
    assert lib.gr_make_kb_table(8.6, 8, 8, 7, 1 << 20, None) == B.GR_EINVAL
    assert lib.gr_make_wkernel_table(16, 8, 0, 0.0, 1.0, 8, 8.6, 0, B.GR_F32, 1 << 20, None) == B.GR_EINVAL
    assert lib.gr_make_wkernel_table(16, 8, 4, 0.0, 1.0, 20, 8.6, 0, B.GR_F32, 1 << 20, None) == B.GR_EINVAL
    assert lib.gr_make_wkernel_table(16, 8, 4, 0.0, 1.0, 8, 8.6, 0, B.GR_F32, None, None) == B.GR_EINVAL


def _item(B, **kw):
    k = _kernel()
    base = dict(uvw=1 << 20, vis=1 << 20, vis_dtype=B.GR_F32, n_pol=4, vis_scale=None, weights=None,
                n_vis=100, kernel=k, inv_cell_u=1.0, inv_cell_v=1.0, grid=1 << 20, height=64, width=64)
    base.update(kw)
    return B.make_batch_item(**base)


def test_batch_validation(lib):
    from paper_1605_07023_amd import binding as B
    good = _item(B)
    arr = (B.GrBatchItem * 3)(good, _item(B, n_pol=3), good)
    assert lib.gr_grid_batch(arr, 3, 1 << 20, 1 << 40, None) == B.GR_EINVAL
    assert "item 1" in lib.gr_last_error().decode()
    assert lib.gr_grid_batch_workspace_bytes(arr, 3) == 0
    assert lib.gr_grid_batch(arr, -1, 1 << 20, 1 << 40, None) == B.GR_EINVAL
    assert lib.gr_grid_batch(arr, 5000, 1 << 20, 1 << 40, None) == B.GR_EINVAL
    k2 = _kernel()
    k2.kind = B.GR_TABLE2D
    arr = (B.GrBatchItem * 2)(good, _item(B, kernel=k2))
    assert lib.gr_grid_batch(arr, 2, 1 << 20, 1 << 40, None) == B.GR_EUNSUPPORTED
    for bad in (dict(grid=None), dict(height=4), dict(inv_cell_u=float("nan")), dict(seg_len=-1),
                dict(vis_dtype=B.GR_F16), dict(n_vis=-1)):
        arr = (B.GrBatchItem * 1)(_item(B, **bad))
        assert lib.gr_grid_batch(arr, 1, 1 << 20, 1 << 40, None) == B.GR_EINVAL, bad
    arr = (B.GrBatchItem * 2)(good, _item(B, n_pol=1, n_vis=0))
    need = lib.gr_grid_batch_workspace_bytes(arr, 2)
    assert need > 0
    assert lib.gr_grid_batch(arr, 2, 1 << 20, need - 1, None) == B.GR_ENOMEM
    assert lib.gr_grid_batch(arr, 2, None, need, None) == B.GR_EINVAL
    assert lib.gr_grid_batch(arr, 0, None, 0, None) == B.GR_OK          # nothing to do


def test_mlp_entry_points_reject(lib):
    from paper_1605_07023_amd import binding as B
    P = 1 << 20
    assert lib.gr_mlp_blob_floats() == 12616
    assert lib.gr_mlp_eval(P, P, -1, P, None) == B.GR_EINVAL
    assert lib.gr_mlp_eval(None, P, 10, P, None) == B.GR_EINVAL
    assert lib.gr_mlp_grads(P, P, P, P, 0, P, None, None) == B.GR_EINVAL
    assert lib.gr_mlp_grads(P, P, None, P, 8, P, None, None) == B.GR_EINVAL
    assert lib.gr_mlp_train_step(P, P, P, P, P, P, P, 8, 0, 1e-3, None, None) == B.GR_EINVAL
    assert lib.gr_mlp_train_step(P, P, P, P, P, P, P, 8, 1, float("nan"), None, None) == B.GR_EINVAL
    assert lib.gr_mlp_train_step(P, None, P, P, P, P, P, 8, 1, 1e-3, None, None) == B.GR_EINVAL
    assert lib.gr_mlp_dataset(P, 16, 8, 0, 0.0, 1.0, 1.0, 1.0, P, P, None) == B.GR_EINVAL
    assert lib.gr_mlp_dataset(P, 16, 8, 4, 0.0, 1.0, 0.0, 1.0, P, P, None) == B.GR_EINVAL
    assert lib.gr_mlp_dataset(P, 16, 8, 4, 0.0, 1.0, 1.0, 1.0, None, P, None) == B.GR_EINVAL


def test_mlp_kernel_descriptor_rules(lib):
    from paper_1605_07023_amd import binding as B
    k = B.make_kernel(1 << 20, 16, 8, 4, True, B.GR_F16, 0.0, 1.0, kind=B.GR_MLP)
    st = lib.gr_preprocess(1 << 20, 1 << 20, B.GR_F32, None, None, 10, 4, ctypes.byref(k), 1.0, 1.0,
                           64, 64, 1 << 20, 1 << 20, None, None)
    assert st == B.GR_EUNSUPPORTED and "GR_MLP" in lib.gr_last_error().decode()


def test_batch_graph_validation(lib):
    """Invalid items or workspace are rejected on the host before any capture."""
    from paper_1605_07023_amd import binding as B
    out = ctypes.c_void_p(123)
    arr = (B.GrBatchItem * 1)(_item(B, n_pol=2))
    assert lib.gr_grid_batch_graph(arr, 1, 1 << 20, 1 << 40, ctypes.byref(out)) == B.GR_EINVAL
    assert out.value is None
    arr = (B.GrBatchItem * 1)(_item(B))
    need = lib.gr_grid_batch_workspace_bytes(arr, 1)
    assert lib.gr_grid_batch_graph(arr, 1, 1 << 20, need - 1, ctypes.byref(out)) == B.GR_ENOMEM
    assert lib.gr_grid_batch_graph(arr, 1, 1 << 20, need, None) == B.GR_EINVAL
    assert lib.gr_graph_launch(None, None) == B.GR_EINVAL
    assert lib.gr_graph_destroy(None) == B.GR_OK


def test_tuning_memo_round_trip(lib):
    """The library's tuning memo: an entry put for a problem class comes back
    from get, gr_grid_workspace_bytes with no tuning follows it (a VALU-kernel
    entry needs the preprocess buffers, the default binned path the bins), other
    classes (support, side class, n_pol, slot) are unaffected, and clear removes it."""
    from paper_1605_07023_amd import binding as B
    B.gr_tuning_memo_clear()
    k = _kernel()
    binned = B.gr_grid_workspace_bytes(1000, 4, k, 64, 64)
    valu = B.gr_grid_workspace_bytes(1000, 4, k, 64, 64, B.GrTuning(0, 0, 0, 0, 0, 1))
    assert binned != valu
    assert B.gr_tuning_memo_get(4, k, 64, 64, 0) is None
    t = B.GrTuning(4, 2, 3, 5, 512, 1)
    B.gr_tuning_memo_put(4, k, 64, 64, 0, t)
    got = B.gr_tuning_memo_get(4, k, 60, 50, 0)            # same side class (64)
    assert (got.cu, got.cv, got.wg_u, got.wg_v, got.vis_per_wg, got.variant) == (4, 2, 3, 5, 512, 1)
    assert B.gr_grid_workspace_bytes(1000, 4, k, 64, 64) == valu
    assert B.gr_tuning_memo_get(4, k, 128, 128, 0) is None  # other side class
    assert B.gr_tuning_memo_get(1, k, 64, 64, 0) is None    # other n_pol
    assert B.gr_tuning_memo_get(4, _kernel(support=8), 64, 64, 0) is None
    assert B.gr_tuning_memo_get(4, _kernel(tap_dtype=B.GR_F16), 64, 64, 0) is None
    assert B.gr_tuning_memo_get(4, k, 64, 64, 1) is None
    assert B.gr_grid_workspace_bytes(1000, 4, k, 128, 128) == B.gr_grid_workspace_bytes(
        1000, 4, k, 128, 128, B.GrTuning(0, 0, 0, 0, 0, 2))
    # slot 1 (gr_grid_records) takes VALU tunings only
    for bad in [B.GrTuning(0, 0, 0, 0, 0, 2), B.GrTuning(0, 0, 0, 0, 0, 3)]:
        assert lib.gr_tuning_memo_put(4, ctypes.byref(k), 64, 64, 1, ctypes.byref(bad)) == B.GR_EINVAL
    assert lib.gr_tuning_memo_put(4, ctypes.byref(k), 64, 64, 2, ctypes.byref(t)) == B.GR_EINVAL
    assert lib.gr_tuning_memo_put(4, ctypes.byref(k), 64, 64, 0, None) == B.GR_EINVAL
    assert lib.gr_tuning_memo_put(3, ctypes.byref(k), 64, 64, 0, ctypes.byref(t)) == B.GR_EINVAL
    B.gr_tuning_memo_put(4, k, 64, 64, 1, B.GrTuning(8, 1, 0, 0, 0, 1))
    assert B.gr_tuning_memo_get(4, k, 64, 64, 1).cu == 8
    B.gr_tuning_memo_clear()
    assert B.gr_tuning_memo_get(4, k, 64, 64, 0) is None
    assert B.gr_tuning_memo_get(4, k, 64, 64, 1) is None
    assert B.gr_grid_workspace_bytes(1000, 4, k, 64, 64) == binned


def test_per_source_flags_name_built_sources():
    """Every per-source hipcc addition names a source the library is built from,
    and every HIP translation unit is built with packed FP32 instructions off."""
    from paper_1605_07023_amd import build
    assert set(build.SOURCE_FLAGS) <= set(build.SOURCES)
    flags = " ".join(build.HIPCC_FLAGS)
    assert "-Xclang -target-feature -Xclang -packed-fp32-ops" in flags
    for src in build.SOURCES:
        assert os.path.exists(os.path.join(build.CSRC, src)), src


def test_traffic_record_hash_covers_the_compile_flags(monkeypatch):
    """The hash that ties the stored HBM byte counts to the gridder changes with
    the kernel's compile flags as well as with its source."""
    import sys
    sys.path.insert(0, ROOT)
    import bench
    from paper_1605_07023_amd import build
    h0 = bench.source_hash(2)
    monkeypatch.setitem(build.SOURCE_FLAGS, "grid_mfma.hip", ["-O2"])
    assert bench.source_hash(2) != h0
    monkeypatch.undo()
    assert bench.source_hash(2) == h0
