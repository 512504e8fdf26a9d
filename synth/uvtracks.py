"""Seeded synthetic interferometer workloads.

Everything here produces *inputs* to gridding: antenna positions, baseline
vectors, Earth-rotation (u, v, w) tracks in wavelengths, complex visibility
samples and weights.  The scale factors that make the tracks fit a grid
(cell size, w range) are chosen here too, because they are properties of the
synthetic observation, not of the gridding method.

The uvw transform is the textbook one (Thompson, Moran & Swenson,
"Interferometry and Synthesis in Radio Astronomy", ch. 4): a local
East-North-Up baseline is rotated into the equatorial (X, Y, Z) frame at the
site latitude, then projected onto (u, v, w) for hour angle H and declination
delta.

The paper's own data set (a simulated MeerKAT observation, Section 5) is not
available; these tracks stand in for it with the same structure: baselines of
an array observed over Earth rotation, visibilities ordered by baseline and
then time.
"""
from __future__ import annotations

import dataclasses
import functools
import math
from typing import Optional

import numpy as np

C_LIGHT = 299792458.0


def antenna_enu(rng: np.random.Generator, n_ant: int, radius_m: float) -> np.ndarray:
    """East/North positions uniform in a disk of ``radius_m``; Up = 0.  Shape [n_ant, 3]."""
    r = radius_m * np.sqrt(rng.random(n_ant))
    th = 2.0 * math.pi * rng.random(n_ant)
    enu = np.zeros((n_ant, 3), dtype=np.float64)
    enu[:, 0] = r * np.cos(th)
    enu[:, 1] = r * np.sin(th)
    return enu


def baseline_pairs(n_ant: int) -> np.ndarray:
    """All pairs p < q in p-major order, shape [n_bl, 2]."""
    p, q = np.triu_indices(n_ant, k=1)
    return np.stack([p, q], axis=1)


def enu_baselines_to_uvw(b_enu: np.ndarray, lat_rad: float, dec_rad: float,
                         hour_angles: np.ndarray, freqs_hz: np.ndarray) -> np.ndarray:
    """Baselines [n_bl, 3] (metres, ENU) -> uvw [n_bl, n_t, n_ch, 3] in wavelengths."""
    e, n, up = b_enu[:, 0], b_enu[:, 1], b_enu[:, 2]
    sl, cl = math.sin(lat_rad), math.cos(lat_rad)
    x = -sl * n + cl * up
    y = e
    z = cl * n + sl * up
    sd, cd = math.sin(dec_rad), math.cos(dec_rad)
    sh = np.sin(hour_angles)[None, :]
    ch = np.cos(hour_angles)[None, :]
    x, y, z = x[:, None], y[:, None], z[:, None]
    u = sh * x + ch * y
    v = -sd * ch * x + sd * sh * y + cd * z
    w = cd * ch * x - cd * sh * y + sd * z
    uvw_m = np.stack([u, v, w], axis=-1)                      # [n_bl, n_t, 3]
    inv_lambda = (freqs_hz / C_LIGHT)[None, None, :, None]     # [1, 1, n_ch, 1]
    return uvw_m[:, :, None, :] * inv_lambda                   # [n_bl, n_t, n_ch, 3]


def _hour_angles(span_h: float, n_t: int) -> np.ndarray:
    """Midpoints of ``n_t`` equal intervals over ``span_h`` hours, centred on transit."""
    step = span_h / n_t
    hours = (np.arange(n_t) + 0.5) * step - span_h / 2.0
    return hours * (2.0 * math.pi / 24.0)


@dataclasses.dataclass
class Workload:
    """One gridding problem: inputs plus the scale parameters of the observation."""
    name: str
    uvw: np.ndarray                 # float64 [N, 3], wavelengths
    vis: np.ndarray                 # complex64 [N, P]
    weights: Optional[np.ndarray]   # float32 [N, P] or None (all ones)
    height: int
    width: int
    support: int
    oversample: int
    inv_cell_u: float               # pixels per wavelength
    inv_cell_v: float
    n_planes: int = 1
    w_min: float = 0.0              # plane = rint((w - w_min) * inv_dw)
    inv_dw: float = 0.0
    w_hat_scale: float = 0.0        # w (wavelengths) -> w in pixel units for the W kernel
    beta: float = 8.6               # Kaiser-Bessel shape
    support_aa: int = 8             # anti-aliasing kernel width inside the W kernel
    kernel: str = "kb"              # "kb" (real separable), "wsep" (complex separable W),
                                    # "w2d" (exact 2-D W)
    fov: float = 0.0                # field of view (direction cosines) of the exact 2-D W kernel
    meta: dict = dataclasses.field(default_factory=dict)

    @property
    def n_vis(self) -> int:
        return int(self.uvw.shape[0])

    @property
    def n_pol(self) -> int:
        return int(self.vis.shape[1])

    def plane_w_hat(self) -> np.ndarray:
        """w (pixel units) at the centre of each plane."""
        if self.n_planes <= 1 or self.inv_dw == 0.0:
            return np.zeros(max(self.n_planes, 1))
        k = np.arange(self.n_planes, dtype=np.float64)
        return (self.w_min + k / self.inv_dw) * self.w_hat_scale


def _fit_scale(uvw: np.ndarray, height: int, width: int, support: int) -> float:
    """Pixels per wavelength so that max(|u|, |v|) lands S/2 + 2 pixels inside the edge."""
    umax = float(np.max(np.abs(uvw[:, 0])))
    vmax = float(np.max(np.abs(uvw[:, 1])))
    half = min(height, width) // 2 - support // 2 - 2
    return half / max(umax, vmax)


def _w_planes(uvw: np.ndarray, n_planes: int, w_hat_max: float):
    """Symmetric linear plane spacing over [-max|w|, +max|w|]."""
    wmax = float(np.max(np.abs(uvw[:, 2])))
    w_min = -wmax
    inv_dw = (n_planes - 1) / (2.0 * wmax)
    return w_min, inv_dw, w_hat_max / wmax


def _draw_vis(rng: np.random.Generator, n: int, n_pol: int) -> np.ndarray:
    """Real and imaginary parts i.i.d. N(0, 1), drawn interleaved (re, im) per value."""
    out = np.empty((n, n_pol), dtype=np.complex64)
    rng.standard_normal(out=out.view(np.float32), dtype=np.float32)
    return out


@functools.lru_cache(maxsize=2)
def _full_shape_arrays(seed: int, n_times: int, n_chan: int, n_pol: int, n_ant: int):
    """uvw [N, 3] (baseline, time, channel order), vis [N, P], and
    (max(|u|, |v|), max |w|) of the full array; shared by every support size."""
    rng = np.random.default_rng(seed)
    enu = antenna_enu(rng, n_ant, 1000.0)
    pairs = baseline_pairs(n_ant)
    b = enu[pairs[:, 1]] - enu[pairs[:, 0]]
    freqs = np.linspace(1.4e9 * 0.95, 1.4e9 * 1.05, n_chan)
    uvw = enu_baselines_to_uvw(b, math.radians(-30.7), math.radians(-30.0),
                               _hour_angles(8.0, n_times), freqs).reshape(-1, 3)
    uvw = np.ascontiguousarray(uvw)
    uv_max = float(max(np.max(np.abs(uvw[:, 0])), np.max(np.abs(uvw[:, 1]))))
    w_max = float(np.max(np.abs(uvw[:, 2])))
    vis = _draw_vis(rng, uvw.shape[0], n_pol)
    uvw.setflags(write=False)
    vis.setflags(write=False)
    return uvw, vis, (uv_max, w_max)


def quantize_vis_f16(vis: np.ndarray, block: int = 256):
    """Input encoding for reduced-precision runs: visibilities as (re, im)
    float16 pairs with one float32 scale per block of ``block`` consecutive
    visibilities (all polarisations).  The scale is the block's largest
    |component| / 2^14, so every scaled value is at most 2^14 in magnitude.
    Returns (halves [N][P][2] float16, scales [ceil(N / block)] float32)."""
    v = np.asarray(vis)
    n = v.shape[0]
    comp = v.view(np.float32).reshape(n, -1)
    nb = -(-n // block)
    pad = nb * block - n
    mag = np.abs(comp).max(axis=1)
    if pad:
        mag = np.concatenate([mag, np.zeros(pad, np.float32)])
    blk = mag.reshape(nb, block).max(axis=1).astype(np.float32)
    scale = np.where(blk > 0, blk / np.float32(2 ** 14), np.float32(1.0)).astype(np.float32)
    per_vis = np.repeat(scale, block)[:n]
    halves = (comp / per_vis[:, None]).astype(np.float16).reshape(n, v.shape[1], 2)
    return halves, scale


def dequantize_vis_f16(halves: np.ndarray, scale: np.ndarray, block: int = 256) -> np.ndarray:
    """complex128 values the scaled float16 encoding represents (exact in FP64)."""
    n = halves.shape[0]
    per_vis = np.repeat(scale.astype(np.float64), block)[:n]
    h = halves.astype(np.float64) * per_vis[:, None, None]
    return h[..., 0] + 1j * h[..., 1]


def tiny_kb_workload(seed: int = 0) -> Workload:
    """8 antennas (28 baselines), 1 channel at 1.4 GHz, 256 dumps over 1 h,
    512x512 grid, one polarisation, real Kaiser-Bessel kernel S=8, O=8."""
    rng = np.random.default_rng(seed)
    enu = antenna_enu(rng, 8, 1000.0)
    pairs = baseline_pairs(8)
    b = enu[pairs[:, 1]] - enu[pairs[:, 0]]
    uvw = enu_baselines_to_uvw(b, math.radians(-30.7), math.radians(-30.0),
                               _hour_angles(1.0, 256), np.array([1.4e9]))
    uvw = uvw.reshape(-1, 3)
    vis = _draw_vis(rng, uvw.shape[0], 1)
    s = _fit_scale(uvw, 512, 512, 8)
    return Workload("tiny-kb-512", uvw, vis, None, 512, 512, 8, 8, s, s,
                    kernel="kb", beta=8.6)


def full_shape_workload(support: int, seed: int = 0, n_baselines: Optional[int] = None,
                        n_times: int = 1024, n_chan: int = 16, grid: int = 4096,
                        n_planes: int = 32, n_pol: int = 4, n_ant: int = 64,
                        order: str = "btc") -> Workload:
    """64 antennas (2016 baselines) x 1024 dumps over 8 h x 16 channels across
    1.4 GHz +/- 5 %, four polarisations, 4096^2 grid, complex separable W
    kernel with ``support`` taps, 32 w-planes, oversampling 8.  Visibilities are
    ordered by baseline, then time, then channel (``order="btc"``), or by
    baseline, then channel, then time (``order="bct"``: the same visibilities,
    each with its own value, permuted so that consecutive ones are consecutive
    dumps of one channel).

    ``n_baselines`` keeps only the first baselines (same tracks, fewer rows) for
    tests that need the real geometry at a smaller size; the scale factors are
    always those of the full array so positions do not change.
    """
    uvw_full, vis_full, umax = _full_shape_arrays(seed, n_times, n_chan, n_pol, n_ant)
    half = grid // 2 - support // 2 - 2
    s = half / umax[0]
    wmax = umax[1]
    w_min, inv_dw, w_hat_scale = -wmax, (n_planes - 1) / (2.0 * wmax), float(support - 8) / wmax
    if n_baselines is not None:
        n_rows = n_baselines * n_times * n_chan
        flat, vis = uvw_full[:n_rows], vis_full[:n_rows]
    else:
        flat, vis = uvw_full, vis_full
    if order == "bct":
        n_bl = flat.shape[0] // (n_times * n_chan)
        flat = np.ascontiguousarray(flat.reshape(n_bl, n_times, n_chan, 3).transpose(0, 2, 1, 3).reshape(-1, 3))
        vis = np.ascontiguousarray(vis.reshape(n_bl, n_times, n_chan, n_pol).transpose(0, 2, 1, 3)
                                   .reshape(-1, n_pol))
    elif order != "btc":
        raise ValueError(f"unknown order {order}")
    return Workload(f"full-shape-S{support}-{order}", flat, vis, None, grid, grid, support, 8, s, s,
                    n_planes=n_planes, w_min=w_min, inv_dw=inv_dw, w_hat_scale=w_hat_scale,
                    kernel="wsep", beta=8.6, support_aa=8)


def batch_workload(seed: int = 0, n_instances: int = 32):
    """Uneven batch: per instance N ~ lognormal over 1e4..1e6 (clipped), grid side
    in {1024, 2048, 4096}, support in {8, 16, 32}, P in {1, 4}; each instance is
    a single-channel stream of a 64-antenna array (baselines then time)."""
    rng = np.random.default_rng(seed)
    enu = antenna_enu(rng, 64, 1000.0)
    pairs = baseline_pairs(64)
    b = enu[pairs[:, 1]] - enu[pairs[:, 0]]
    out = []
    for i in range(n_instances):
        n_i = int(np.clip(round(math.exp(rng.normal(math.log(1e5), 1.1513))), 1e4, 1e6))
        side = int(rng.choice([1024, 2048, 4096]))
        sup = int(rng.choice([8, 16, 32]))
        npol = int(rng.choice([1, 4]))
        freq = 1.4e9 * (0.95 + 0.1 * rng.random())
        n_t = -(-n_i // len(pairs))
        uvw = enu_baselines_to_uvw(b, math.radians(-30.7), math.radians(-30.0),
                                   _hour_angles(8.0, n_t), np.array([freq]))
        flat = np.ascontiguousarray(uvw.reshape(-1, 3)[:n_i])
        s = _fit_scale(flat, side, side, sup)
        n_planes = 32 if sup > 8 else 1
        if n_planes > 1:
            w_min, inv_dw, whs = _w_planes(flat, n_planes, float(sup - 8))
            kern = "wsep"
        else:
            w_min, inv_dw, whs = 0.0, 0.0, 0.0
            kern = "kb"
        vis = _draw_vis(rng, n_i, npol)
        out.append(Workload(f"batch{i}", flat, vis, None, side, side, sup, 8, s, s,
                            n_planes=n_planes, w_min=w_min, inv_dw=inv_dw, w_hat_scale=whs,
                            kernel=kern))
    return out


def random_point_workload(n_vis: int, n_pol: int, height: int, width: int, support: int,
                          oversample: int, seed: int, n_planes: int = 1,
                          margin: int = 0, weights: bool = False,
                          kernel: str = "kb") -> Workload:
    """Uniformly scattered (u, v, w) points: no track structure.  Used for small
    parity and edge-case tests.  ``margin`` pixels beyond the grid edge are
    allowed so that some footprints fall off the grid and get dropped."""
    rng = np.random.default_rng(seed)
    if kernel == "kb":
        n_planes = 1                    # the Kaiser-Bessel table has a single plane
    inv_cell = 1.0
    half_u = width / 2 - support / 2 - 1 + margin
    half_v = height / 2 - support / 2 - 1 + margin
    u = rng.uniform(-half_u, half_u, n_vis)
    v = rng.uniform(-half_v, half_v, n_vis)
    w = rng.uniform(-100.0, 100.0, n_vis)
    uvw = np.stack([u, v, w], axis=1)
    vis = _draw_vis(rng, n_vis, n_pol)
    wts = rng.uniform(0.5, 2.0, (n_vis, n_pol)).astype(np.float32) if weights else None
    if n_planes > 1:
        w_min, inv_dw, whs = -100.0, (n_planes - 1) / 200.0, float(max(support - 8, 0)) / 100.0
    else:
        w_min, inv_dw, whs = 0.0, 0.0, 0.0
    return Workload(f"points-{n_vis}", uvw, vis, wts, height, width, support, oversample,
                    inv_cell, inv_cell, n_planes=n_planes, w_min=w_min, inv_dw=inv_dw,
                    w_hat_scale=whs, kernel=kernel, fov=0.5 if kernel == "w2d" else 0.0)


def learned_kernel_workload(seed: int = 0, n_baselines: Optional[int] = None,
                            fov: float = 0.5) -> Workload:
    """The full-shape visibilities with the exact (non-separable) 2-D W kernel:
    support 32, 64 w-planes, oversampling 8 on both axes (a 33.5 MB complex64
    table), field of view ``fov`` direction cosines."""
    wl = full_shape_workload(32, seed=seed, n_baselines=n_baselines, n_planes=64)
    wl.name = "learned-w2d-S32"
    wl.kernel = "w2d"
    wl.fov = fov
    return wl


@functools.lru_cache(maxsize=2)
def _compression_extent(seed: int) -> np.ndarray:
    """Two rows of uvw spanning the whole 2 h array's extent: (max|u|, max|v|,
    max|w|) and its negation, enough for the scale and w-plane fits."""
    rng = np.random.default_rng(seed)
    enu = antenna_enu(rng, 64, 1000.0)
    pairs = baseline_pairs(64)
    b = enu[pairs[:, 1]] - enu[pairs[:, 0]]
    full = enu_baselines_to_uvw(b, math.radians(-30.7), math.radians(-30.0), _hour_angles(2.0, 3600),
                                np.array([1.4e9])).reshape(-1, 3)
    m = np.abs(full).max(axis=0)
    return np.stack([m, -m])


def compression_workload(seed: int = 0, n_baselines: Optional[int] = None, n_pol: int = 4,
                         grid: int = 2048, support: int = 16, n_planes: int = 32) -> Workload:
    """Stand-in for the paper's simulated MeerKAT set (Section 5: 2 h at 2 s
    dumps, one channel, 7,257,600 visibilities that compress about 3x): the
    64-antenna array, 2016 baselines x 3600 dumps of 2 s over 2 h, one channel at
    1.4 GHz, baselines then time, ``grid``^2 cells, separable W kernel
    (``support`` taps, ``n_planes`` planes, oversampling 8).  Consecutive dumps
    of short baselines fall on the same oversampled cell, which is what
    compression merges.  ``n_baselines`` keeps only the first baselines."""
    rng = np.random.default_rng(seed)
    enu = antenna_enu(rng, 64, 1000.0)
    pairs = baseline_pairs(64)
    if n_baselines is not None:
        pairs = pairs[:n_baselines]
    b = enu[pairs[:, 1]] - enu[pairs[:, 0]]
    uvw = enu_baselines_to_uvw(b, math.radians(-30.7), math.radians(-30.0), _hour_angles(2.0, 3600),
                               np.array([1.4e9]))
    flat = np.ascontiguousarray(uvw.reshape(-1, 3))
    full = _compression_extent(seed)         # scales of the whole array, whatever n_baselines
    s = _fit_scale(full, grid, grid, support)
    w_min, inv_dw, whs = _w_planes(full, n_planes, float(max(support - 8, 0)))
    vis = _draw_vis(rng, flat.shape[0], n_pol)
    return Workload(f"compress-E1-{grid}", flat, vis, None, grid, grid, support, 8, s, s,
                    n_planes=n_planes, w_min=w_min, inv_dw=inv_dw, w_hat_scale=whs, kernel="wsep",
                    beta=8.6, support_aa=8)


def wstack_workload(seed: int = 0, n_baselines: Optional[int] = None, n_pol: int = 4, grid: int = 2048,
                    support: int = 16, n_slices: int = 7, planes_per_slice: int = 32) -> Workload:
    """Stand-in for the paper's W-stacked runs (Section 5: the 2 h, 2 s-dump
    set split by w into 7 slices, each gridded on its own): the tracks and
    visibilities of :func:`compression_workload`.  ``meta`` holds the slicing:
    ``n_slices`` equal slices from ``w_first`` of width 1 / ``inv_width``
    spanning [-max|w|, +max|w|] of the whole array (padded by 2^-20 so that the
    extreme w falls inside).  ``n_planes`` / ``w_min`` / ``inv_dw`` describe
    one table for every slice, its planes spread over
    [-width/2, +width/2] about a slice's centre (``w_min`` relative to it)."""
    wl = compression_workload(seed, n_baselines, n_pol, grid, support, planes_per_slice)
    full = _compression_extent(seed)
    half = float(np.max(np.abs(full[:, 2]))) * (1.0 + 2.0 ** -20)
    width = 2.0 * half / n_slices
    return dataclasses.replace(
        wl, name=f"wstack{n_slices}-{grid}", n_planes=planes_per_slice, w_min=-0.5 * width,
        inv_dw=(planes_per_slice - 1) / width,
        meta=dict(n_slices=n_slices, w_first=-half, inv_width=n_slices / (2.0 * half)))


def aterm_workload(support: int, seed: int = 0, n_baselines: Optional[int] = None, n_times: int = 1024,
                   n_chan: int = 16, grid: int = 4096, n_planes: int = 4, n_pol: int = 4, time_slots: int = 8,
                   freq_groups: int = 2) -> Workload:
    """The tracks of :func:`full_shape_workload` (baseline, time, channel
    order) with a GCF id per visibility, as A-projection assigns GCFs by time
    and frequency (Section 6): ``time_slots`` equal intervals of the dumps
    times ``freq_groups`` equal groups of the channels.  ``meta`` holds
    ``kernel_id`` (int32 [N]) and ``n_ids``; the GCF values come from
    :func:`aterm_taps`."""
    wl = full_shape_workload(support, seed, n_baselines, n_times, n_chan, grid, n_planes, n_pol)
    n = np.arange(wl.n_vis, dtype=np.int64)
    t = (n // n_chan) % n_times
    c = n % n_chan
    ids = ((t * time_slots) // n_times) * freq_groups + (c * freq_groups) // n_chan
    return dataclasses.replace(wl, name=f"aterm-S{support}", kernel="aterm",
                               meta=dict(kernel_id=ids.astype(np.int32), n_ids=time_slots * freq_groups))


def aterm_taps(seed: int, n_ids: int, n_planes: int, oversample: int, n_pol: int, support: int) -> np.ndarray:
    """Synthetic GCF table complex64 [n_ids][planes][O][O][P][S][S] (there are
    no beam models here): real and imaginary parts i.i.d. N(0, 1/S^2)."""
    rng = np.random.default_rng(seed)
    shape = (n_ids, n_planes, oversample, oversample, n_pol, support, support)
    out = np.empty(shape, dtype=np.complex64)
    rng.standard_normal(out=out.view(np.float32), dtype=np.float32)
    out *= np.float32(1.0 / support)
    return out
