"""Seeded synthetic workloads shared by the FP64 oracle's tests and the GPU path.

This package generates inputs only (antenna layouts, Earth-rotation uvw tracks,
visibility values, weights).  It contains none of the gridding arithmetic: no
pixel conversion, no kernel tables, no accumulation.
"""
from .uvtracks import (  # noqa: F401
    C_LIGHT, antenna_enu, baseline_pairs, enu_baselines_to_uvw, Workload,
    tiny_kb_workload, full_shape_workload, batch_workload, random_point_workload,
    quantize_vis_f16, dequantize_vis_f16, learned_kernel_workload, compression_workload,
    wstack_workload, aterm_workload, aterm_taps,
)
