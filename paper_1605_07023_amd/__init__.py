"""MI355X (gfx950) convolutional gridding: Romein work distribution with thread
coarsening (Merry 2016, arXiv:1605.07023), hand-written HIP behind a C ABI.

The compute path is ``libgridder.so`` (built from ``csrc/`` by ``build.py``);
``binding`` marshals torch device tensors into its C entry points.  There is no
CPU fallback: if the library is missing, every call raises.
"""
from .binding import (  # noqa: F401
    GridderError, GrKernel, GrTuning, GR_F32, GR_F16, GR_BF16, GR_F64, GR_SEPARABLE,
    GR_TABLE2D, GR_MLP, library_path, load_library, gr_version, gr_last_error,
    gr_grid_workspace_bytes, gr_preprocess, gr_grid_records, gr_grid, gr_make_kb_table,
    gr_make_wkernel_table, make_kernel, gr_bin_bytes, gr_bin, gr_grid_binned, gr_autotune,
    gr_make_wkernel2d_table, gr_mlp_blob_floats, gr_mlp_eval, gr_mlp_dataset, gr_mlp_grads,
    gr_mlp_train_step, GrBatchItem, make_batch_item, gr_grid_batch, gr_grid_batch_workspace_bytes,
    gr_grid_batch_graph, gr_graph_launch, gr_graph_destroy,
)
