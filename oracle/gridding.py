"""FP64 NumPy oracle: the gridding definition, its index conversion and its tables.

Test infrastructure only (see the package docstring).  Each function cites the
passage of Merry (2016), "Faster GPU-based convolutional gridding via thread
coarsening", that it follows.  Where the paper is silent the reading used is
stated in the docstring.

Gridding, Section 2.2: each visibility is a Dirac delta convolved with the
gridding convolution function (GCF) and sampled on the regular grid; the GCF is
tabulated at ``oversample`` times the grid resolution.  Thread coarsening, bins,
tiles and compression (Sections 2.2-4) only reorder the additions, so the
oracle is the definition itself, summed in complex128.

Pins: tests/test_oracle_*.py check this module against closed forms, an
independent FFT evaluation of the kernel tables, brute-force evaluation of
the analytic kernel at every cell, delta tables, flux conservation, linearity,
permutation invariance and Hermitian symmetry.
"""
from __future__ import annotations

import math
from typing import Optional

import numpy as np


# ----------------------------------------------------------------------------
# Kernel functions and tables (Section 2.2: GCF tables are precomputed and
# oversampled; Section 4: a separable, polarisation-independent GCF)
# ----------------------------------------------------------------------------

def kaiser_bessel(delta, support: int, beta: float):
    """Kaiser-Bessel window of width ``support``:
    I0(beta * sqrt(1 - (2 delta / S)^2)) / I0(beta) for |delta| < S/2, else 0.

    Reading: the paper names an anti-aliasing GCF without fixing one; the
    Kaiser-Bessel window (peak 1, zero at and beyond half the support) is used.
    ``np.i0`` is the library Bessel function.
    """
    d = np.asarray(delta, dtype=np.float64)
    x = 2.0 * d / support
    inside = np.abs(d) < support / 2.0
    arg = np.sqrt(np.where(inside, 1.0 - x * x, 0.0))
    return np.where(inside, np.i0(beta * arg) / np.i0(beta), 0.0)


def tap_offsets(support: int, oversample: int) -> np.ndarray:
    """Kernel argument of tap k at oversampled phase s: delta[s, k] = k - S/2 + 1 - s/O.

    The footprint of a visibility at pixel position ix + s/O is cells
    ix - S/2 + 1 ... ix + S/2, and tap k multiplies cell ix - S/2 + 1 + k.
    Reading (paper silent): with the kernel zero for |delta| >= S/2, every
    placement mirrors exactly under u -> -u.
    """
    k = np.arange(support, dtype=np.float64)[None, :]
    s = np.arange(oversample, dtype=np.float64)[:, None]
    return k - support // 2 + 1 - s / oversample


def kb_table(support: int, oversample: int, beta: float) -> np.ndarray:
    """Real separable Kaiser-Bessel taps, float64 [1][O][S] (one plane)."""
    return kaiser_bessel(tap_offsets(support, oversample), support, beta)[None]


def kb_image_taper(nu, support_aa: int, beta: float):
    """Image-plane response of the Kaiser-Bessel window of width ``support_aa``
    at normalised image coordinate ``nu`` (field of view = [-1/2, 1/2]):
    sinh(sqrt(beta^2 - (pi S nu)^2)) / sqrt(...), continued as sin(sqrt(-r))/sqrt(-r)
    where the radicand r is negative.  (Standard Fourier pair of the window.)"""
    nu = np.asarray(nu, dtype=np.float64)
    r = beta * beta - (math.pi * support_aa * nu) ** 2
    out = np.empty_like(r)
    pos = r > 0
    neg = r < 0
    zero = ~(pos | neg)
    sp = np.sqrt(r[pos])
    out[pos] = np.sinh(sp) / sp
    sn = np.sqrt(-r[neg])
    out[neg] = np.sin(sn) / sn
    out[zero] = 1.0
    return out


def w_screen_samples(n_samples: int) -> np.ndarray:
    """Midpoint sample positions nu_j = (j + 1/2)/M - 1/2 across the field of view."""
    return (np.arange(n_samples, dtype=np.float64) + 0.5) / n_samples - 0.5


def wkernel_1d(w_hat: float, delta, support_aa: int, beta: float, n_samples: int):
    """Un-normalised separable W kernel at kernel argument(s) ``delta`` (pixels):

        g(delta) = sum_j t(nu_j) exp(-i pi w_hat nu_j^2) exp(-2 pi i delta nu_j)

    i.e. the discrete Fourier transform of the anti-aliasing taper times the
    paraxial w phase screen (Section 2.2 treats the w term of the measurement
    equation as a convolution, W-projection; Section 4 uses a separable
    approximation).  ``w_hat`` is w expressed in pixel units.
    Reading (paper silent): the paraxial n - 1 = -(l^2 + m^2)/2 makes the screen
    separable in u and v; the sign follows the exp(-2 pi i w (n - 1)) term of
    the measurement equation inverted for imaging.
    """
    nu = w_screen_samples(n_samples)
    screen = kb_image_taper(nu, support_aa, beta) * np.exp(-1j * math.pi * w_hat * nu * nu)
    d = np.asarray(delta, dtype=np.float64)
    phase = np.exp(-2j * math.pi * d[..., None] * nu)
    return phase @ screen


def wkernel_norm(support: int, support_aa: int, beta: float, n_samples: int) -> float:
    """Constant c making the w = 0, phase-0 taps sum to 1 (flux normalisation)."""
    d0 = tap_offsets(support, 1)[0]
    g = wkernel_1d(0.0, d0, support_aa, beta, n_samples)
    g = np.where(np.abs(d0) < support / 2.0, g, 0.0)
    return 1.0 / float(np.real(np.sum(g)))


def wkernel_table(support: int, oversample: int, w_hats, support_aa: int = 8,
                  beta: float = 8.6, n_samples: Optional[int] = None) -> np.ndarray:
    """Complex separable W-kernel taps, complex128 [planes][O][S].

    Tap (plane, s, k) = c * g_{w_hat[plane]}(delta[s, k]), zero where
    |delta| >= S/2 (truncation at the support).  The same 1-D table applies
    along u and along v (square cells).  Default M = 4 S screen samples.
    """
    m = 4 * support if n_samples is None else n_samples
    d = tap_offsets(support, oversample)
    c = wkernel_norm(support, support_aa, beta, m)
    w_hats = np.atleast_1d(np.asarray(w_hats, dtype=np.float64))
    out = np.empty((w_hats.size, oversample, support), dtype=np.complex128)
    inside = np.abs(d) < support / 2.0
    for p, wh in enumerate(w_hats):
        out[p] = np.where(inside, c * wkernel_1d(float(wh), d, support_aa, beta, m), 0.0)
    return out


def wkernel_2d_table(support: int, oversample: int, w_hats, fov: float,
                     support_aa: int = 8, beta: float = 8.6,
                     n_samples: Optional[int] = None) -> np.ndarray:
    """Exact (non-paraxial) 2-D W-kernel taps, complex128 [planes][O][O][S][S]
    indexed [plane][s_v][s_u][k_v][k_u]:

        C(du, dv) = c^2 sum_a sum_b t(nu_a) t(nu_b)
                    exp(2 pi i (w_hat / fov^2) (sqrt(1 - fov^2 (nu_a^2 + nu_b^2)) - 1))
                    exp(-2 pi i (du nu_a + dv nu_b))

    ``fov`` is the field of view in direction cosines (image coordinate
    l = fov * nu).  As fov -> 0 this tends to the outer product of two
    separable tables with the same w_hat.  Computed as a row-column DFT.
    """
    m = 4 * support if n_samples is None else n_samples
    nu = w_screen_samples(m)
    t = kb_image_taper(nu, support_aa, beta)
    c = wkernel_norm(support, support_aa, beta, m)
    d = tap_offsets(support, oversample)                       # [O][S]
    inside = np.abs(d) < support / 2.0
    ph = np.where(inside[..., None], np.exp(-2j * math.pi * d[..., None] * nu), 0.0)  # [O][S][M]
    rho2 = nu[:, None] ** 2 + nu[None, :] ** 2
    w_hats = np.atleast_1d(np.asarray(w_hats, dtype=np.float64))
    out = np.empty((w_hats.size, oversample, oversample, support, support), dtype=np.complex128)
    for p, wh in enumerate(w_hats):
        screen = (t[:, None] * t[None, :]) * np.exp(
            2j * math.pi * (wh / fov ** 2) * (np.sqrt(1.0 - fov * fov * rho2) - 1.0))
        # C[sv, su, kv, ku] = sum_a sum_b ph[sv,kv,b] ph[su,ku,a] screen[b, a]   (b: v axis, a: u axis)
        half = np.einsum("vkb,ba->vka", ph, screen)              # [O][S][M]
        out[p] = c * c * np.einsum("vka,uja->vukj", half, ph)
    return out


def wkernel_2d_at(w_hat: float, d_u, d_v, fov: float, support: int, support_aa: int = 8,
                  beta: float = 8.6, n_samples: Optional[int] = None) -> np.ndarray:
    """The exact 2-D W kernel of :func:`wkernel_2d_table` at arbitrary offsets:
    complex128 [len(d_v)][len(d_u)], C(d_u[j], d_v[i]), zero where |d_u| or
    |d_v| >= S/2, with the same normaliser c (a function of the support)."""
    m = 4 * support if n_samples is None else n_samples
    nu = w_screen_samples(m)
    t = kb_image_taper(nu, support_aa, beta)
    c = wkernel_norm(support, support_aa, beta, m)
    du = np.asarray(d_u, dtype=np.float64)
    dv = np.asarray(d_v, dtype=np.float64)
    rho2 = nu[:, None] ** 2 + nu[None, :] ** 2
    screen = (t[:, None] * t[None, :]) * np.exp(
        2j * math.pi * (w_hat / fov ** 2) * (np.sqrt(1.0 - fov * fov * rho2) - 1.0))   # [b (v), a (u)]
    pu = np.exp(-2j * math.pi * du[:, None] * nu[None, :])                             # [j, a]
    pv = np.exp(-2j * math.pi * dv[:, None] * nu[None, :])                             # [i, b]
    out = c * c * (pv @ screen @ pu.T)
    inside = (np.abs(dv)[:, None] < support / 2.0) & (np.abs(du)[None, :] < support / 2.0)
    return np.where(inside, out, 0.0)


def grid_w2d_continuous(vis: np.ndarray, uvw: np.ndarray, weights: Optional[np.ndarray],
                        inv_cell_u: float, inv_cell_v: float, oversample: int, support: int,
                        height: int, width: int, n_planes: int, w_min: float, inv_dw: float,
                        w_hat_scale: float, fov: float, support_aa: int = 8, beta: float = 8.6):
    """Reference grid with the exact 2-D W kernel at each visibility's own w_hat
    and exact pixel position (no w-plane or phase quantisation): visibility n
    adds C(w_n * w_hat_scale, x - p_u, y - p_v) V_n to cell (y, x) of the
    footprint that the quantised position selects (the same cells and the same
    kept visibilities as the table gridder), where p = u * inv_cell + W/2 is the
    exact pixel position.  One S x S kernel evaluation per visibility: meant for
    subsamples."""
    n_pol = vis.shape[1]
    pc = pixel_coords(uvw, inv_cell_u, inv_cell_v, oversample, support, height, width,
                      n_planes, w_min, inv_dw)
    valid = pc["valid"] & finite_values(vis, weights)
    wv = weighted_vis(vis, weights)
    out = np.zeros((n_pol, height, width), np.complex128)
    k = np.arange(support, dtype=np.float64)
    for n in np.nonzero(valid)[0]:
        pu = uvw[n, 0] * inv_cell_u + width / 2.0
        pv = uvw[n, 1] * inv_cell_v + height / 2.0
        x0, y0 = int(pc["x0"][n]), int(pc["y0"][n])
        kern = wkernel_2d_at(float(uvw[n, 2]) * w_hat_scale, x0 + k - pu, y0 + k - pv, fov, support,
                             support_aa, beta)
        for p in range(n_pol):
            out[p, y0:y0 + support, x0:x0 + support] += kern * wv[n, p]
    return out, int(np.count_nonzero(~valid))


# ----------------------------------------------------------------------------
# Index conversion and drop rule (Section 4: cell, oversampling phase and w
# plane of every visibility are worked out once, before gridding)
# ----------------------------------------------------------------------------

def pixel_coords(uvw: np.ndarray, inv_cell_u: float, inv_cell_v: float, oversample: int,
                 support: int, height: int, width: int, n_planes: int = 1,
                 w_min: float = 0.0, inv_dw: float = 0.0) -> dict:
    """Integer footprint origin, oversampled phase, w-plane and validity per visibility.

    Readings (paper silent):
      * uv = 0 sits at cell (H/2, W/2); u runs along columns x, v along rows y.
      * fx = rint(u * (inv_cell_u * O)) + (W/2) O with round-half-even, the
        centre added after rounding so u -> -u mirrors exactly;
        ix = fx >> log2(O), sx = fx & (O - 1); likewise v -> (fy, iy, sy).
      * footprint origin x0 = ix - S/2 + 1, y0 = iy - S/2 + 1.
      * plane = rint((w - w_min) * inv_dw); a single-plane kernel ignores w.
      * a visibility is dropped (and counted) if u, v or w is not finite, its
        plane is outside [0, n_planes), or its footprint leaves the grid.
    """
    uvw = np.asarray(uvw, dtype=np.float64)
    u, v, w = uvw[:, 0], uvw[:, 1], uvw[:, 2]
    lg = int(oversample).bit_length() - 1
    assert (1 << lg) == oversample
    finite = np.isfinite(u) & np.isfinite(v) & np.isfinite(w)
    xh = np.where(finite, u * (inv_cell_u * oversample), 0.0)
    yh = np.where(finite, v * (inv_cell_v * oversample), 0.0)
    # anything this large is off every supported grid; clamp before int conversion
    big = 2.0 ** 40
    ok = finite & (np.abs(xh) < big) & (np.abs(yh) < big)
    fx = np.rint(np.where(ok, xh, 0.0)).astype(np.int64) + (width // 2) * oversample
    fy = np.rint(np.where(ok, yh, 0.0)).astype(np.int64) + (height // 2) * oversample
    ix, sx = fx >> lg, fx & (oversample - 1)
    iy, sy = fy >> lg, fy & (oversample - 1)
    x0 = ix - support // 2 + 1
    y0 = iy - support // 2 + 1
    if n_planes > 1:
        ph = np.where(ok, (w - w_min) * inv_dw, 0.0)
        ok &= np.abs(ph) < big
        plane = np.rint(np.where(ok, ph, 0.0)).astype(np.int64)
    else:
        plane = np.zeros_like(x0)
    valid = ok & (plane >= 0) & (plane < n_planes) & (x0 >= 0) & (x0 + support <= width) \
        & (y0 >= 0) & (y0 + support <= height)
    return dict(x0=x0, y0=y0, sx=sx, sy=sy, plane=plane, valid=valid, fx=fx, fy=fy)


def finite_values(vis: np.ndarray, weights: Optional[np.ndarray]) -> np.ndarray:
    """True per visibility when all its visibility and weight values are finite.
    Reading (paper silent): such a visibility is dropped like one with bad uvw."""
    ok = np.all(np.isfinite(np.asarray(vis).view(np.float32 if np.asarray(vis).dtype == np.complex64
                                                  else np.float64)), axis=1)
    if weights is not None:
        ok &= np.all(np.isfinite(np.asarray(weights)), axis=1)
    return ok


def weighted_vis(vis: np.ndarray, weights: Optional[np.ndarray]) -> np.ndarray:
    """Pre-weighted visibilities (Section 4), complex128 [N][P]; weights default to 1."""
    v = np.asarray(vis).astype(np.complex128)
    if weights is not None:
        v = v * np.asarray(weights, dtype=np.float64)
    return v


# ----------------------------------------------------------------------------
# Gridding (Section 2.2 definition, summed in complex128)
# ----------------------------------------------------------------------------

def grid_separable(vis: np.ndarray, uvw: np.ndarray, weights: Optional[np.ndarray],
                   taps: np.ndarray, inv_cell_u: float, inv_cell_v: float, oversample: int,
                   height: int, width: int, n_planes: int = 1, w_min: float = 0.0,
                   inv_dw: float = 0.0, grid: Optional[np.ndarray] = None,
                   taps_v: Optional[np.ndarray] = None, chunk: int = 4096):
    """grid[p, y0+ky, x0+kx] += w[n,p] V[n,p] Tv[plane][sy][ky] Tu[plane][sx][kx]
    for every valid visibility n, polarisation p and tap pair (ky, kx).

    ``taps`` is [planes][O][S] (real or complex) and serves both axes unless
    ``taps_v`` is given.  Returns (grid complex128 [P][H][W], n_dropped).
    """
    taps = np.asarray(taps)
    tv_all = taps if taps_v is None else np.asarray(taps_v)
    support = taps.shape[-1]
    n_pol = vis.shape[1]
    pc = pixel_coords(uvw, inv_cell_u, inv_cell_v, oversample, support, height, width,
                      n_planes, w_min, inv_dw)
    pc["valid"] = pc["valid"] & finite_values(vis, weights)
    wv = weighted_vis(vis, weights)
    out = np.zeros((n_pol, height, width), np.complex128) if grid is None \
        else np.array(grid, dtype=np.complex128, copy=True)
    grid_coords(pc, wv, taps, out, taps_v=tv_all, chunk=chunk)
    return out, int(np.count_nonzero(~pc["valid"]))


def grid_coords(coords: dict, wv: np.ndarray, taps: np.ndarray, out: np.ndarray,
                taps_v: Optional[np.ndarray] = None, chunk: int = 4096) -> np.ndarray:
    """The definition of :func:`grid_separable` on precomputed coordinates:
    out[p, y0+ky, x0+kx] += wv[n,p] Tv[plane][sy][ky] Tu[plane][sx][kx] for every n
    with coords["valid"][n]; out is complex128 [P][H][W], updated in place."""
    taps = np.asarray(taps)
    tv_all = taps if taps_v is None else np.asarray(taps_v)
    support = taps.shape[-1]
    n_pol, height, width = out.shape
    idx = np.nonzero(coords["valid"])[0]
    k = np.arange(support)
    flat = out.reshape(n_pol, -1)
    for c0 in range(0, idx.size, chunk):
        sel = idx[c0:c0 + chunk]
        pl = coords["plane"][sel]
        tu = taps[pl, coords["sx"][sel]].astype(np.complex128)        # [n][S]
        tv = tv_all[pl, coords["sy"][sel]].astype(np.complex128)      # [n][S]
        kern = tv[:, :, None] * tu[:, None, :]                        # [n][S][S]
        rows = coords["y0"][sel][:, None] + k[None, :]
        cols = coords["x0"][sel][:, None] + k[None, :]
        cell = (rows[:, :, None] * width + cols[:, None, :]).ravel()
        for p in range(n_pol):
            contrib = (kern * wv[sel, p][:, None, None]).ravel()
            flat[p] += np.bincount(cell, weights=contrib.real, minlength=height * width) \
                + 1j * np.bincount(cell, weights=contrib.imag, minlength=height * width)
    return out


def compress(coords: dict, wv: np.ndarray):
    """Compression (Section 2.2, after Muscat; applied in the preprocess,
    Section 4): adjacent visibilities that sit at the same position of the
    oversampled grid and in the same w plane meet the same GCF samples, so they
    are added into one visibility.  Reading: "adjacent" means consecutive in
    the input stream, and a dropped visibility separates runs.

    coords: :func:`pixel_coords` output whose "valid" already includes the value
    rule; wv: weighted visibilities [N][P].  Returns (coords of the compressed
    stream, keyed like the input, all valid; summed visibilities complex128
    [M][P]; index of each run's first visibility in the input [M])."""
    valid = np.asarray(coords["valid"], bool)
    key = np.stack([np.asarray(coords[k]) for k in ("x0", "y0", "sx", "sy", "plane")], axis=1)
    same_as_prev = np.zeros(valid.size, bool)
    same_as_prev[1:] = valid[1:] & valid[:-1] & np.all(key[1:] == key[:-1], axis=1)
    head = valid & ~same_as_prev
    heads = np.nonzero(head)[0]
    run = np.cumsum(head) - 1                   # the run each visibility belongs to
    sums = np.zeros((heads.size, wv.shape[1]), np.complex128)
    np.add.at(sums, run[valid], np.asarray(wv, np.complex128)[valid])
    out = {k: np.asarray(coords[k])[heads] for k in ("x0", "y0", "sx", "sy", "plane")}
    out["valid"] = np.ones(heads.size, bool)
    return out, sums, heads


# ----------------------------------------------------------------------------
# W-stacking slices (Section 5: the data is split into slices by w, and each
# slice is gridded as its own problem)
# ----------------------------------------------------------------------------

def wslice_index(uvw: np.ndarray, w_first: float, inv_width: float, n_slices: int) -> np.ndarray:
    """Slice of each visibility, int64 [N]; n_slices for none.

    Reading (the paper fixes no rule): slices of equal width 1 / inv_width
    starting at w_first, slice = floor((w - w_first) * inv_width) in FP64; a
    visibility whose slice falls outside [0, n_slices), or whose w is not
    finite, belongs to no slice."""
    w = np.asarray(uvw, dtype=np.float64)[:, 2]
    with np.errstate(invalid="ignore"):
        t = (w - w_first) * inv_width
        inside = (t >= 0.0) & (t < n_slices)          # NaN fails both
    return np.where(inside, np.floor(np.where(inside, t, 0.0)), n_slices).astype(np.int64)


def wslice_partition(uvw: np.ndarray, w_first: float, inv_width: float, n_slices: int):
    """Stable partition of the stream by slice: (order, offsets) with
    order[offsets[s]:offsets[s + 1]] the input indices of slice s in input
    order (s < n_slices) and order[offsets[n_slices]:] those of no slice."""
    s = wslice_index(uvw, w_first, inv_width, n_slices)
    order = np.argsort(s, kind="stable")
    counts = np.bincount(s, minlength=n_slices + 1)
    offsets = np.concatenate([[0], np.cumsum(counts)[:-1]]).astype(np.int64)
    return order, offsets


def wslice_w_min(w_first: float, inv_width: float, s: int, w_min_rel: float) -> float:
    """w_min of slice s's GCF table.  Reading: the table's planes are relative
    to the slice's centre w_first + (s + 1/2) / inv_width (the stack corrects
    that w; the GCF only the offset from it), so its w_min moves with the
    centre."""
    return w_first + (s + 0.5) / inv_width + w_min_rel


def grid_wstack(vis: np.ndarray, uvw: np.ndarray, weights: Optional[np.ndarray], taps: np.ndarray,
                inv_cell_u: float, inv_cell_v: float, oversample: int, height: int, width: int,
                n_planes: int, w_min_rel: float, inv_dw: float, w_first: float, inv_width: float,
                n_slices: int):
    """Every slice gridded on its own into its own grid by the definition of
    :func:`grid_separable`, with the table ``taps`` whose plane rule is
    rint((w - wslice_w_min(s)) * inv_dw).  Returns (grids complex128
    [n_slices][P][H][W], visibilities dropped inside the slices by the
    coordinate and value rules, visibilities in no slice)."""
    vis = np.asarray(vis)
    n_pol = vis.shape[1]
    order, offsets = wslice_partition(uvw, w_first, inv_width, n_slices)
    grids = np.zeros((n_slices, n_pol, height, width), np.complex128)
    dropped = 0
    for s in range(n_slices):
        sel = order[offsets[s]:offsets[s + 1]]
        if sel.size == 0:
            continue
        g, d = grid_separable(vis[sel], np.asarray(uvw)[sel], None if weights is None else np.asarray(weights)[sel],
                              taps, inv_cell_u, inv_cell_v, oversample, height, width, n_planes,
                              wslice_w_min(w_first, inv_width, s, w_min_rel), inv_dw)
        grids[s] = g
        dropped += d
    return grids, dropped, int(order.size - offsets[n_slices])


def grid_aterm(vis: np.ndarray, uvw: np.ndarray, weights: Optional[np.ndarray], kernel_id: np.ndarray,
               taps: np.ndarray, inv_cell_u: float, inv_cell_v: float, oversample: int, height: int,
               width: int, n_planes: int, w_min: float, inv_dw: float, chunk: int = 1024):
    """Non-separable GCFs per visibility and per polarisation (Section 6: the
    A-projection GCFs depend on time, frequency, polarisation and possibly
    baseline, and are not separable):
        grid[p, y0+ky, x0+kx] += w[n,p] V[n,p] T[id[n], plane, sy, sx, p, ky, kx]
    with ``taps`` complex [n_ids][planes][O][O][P][S][S] and the indices of
    :func:`pixel_coords`.

    Readings (paper silent): each polarisation has its own GCF and none mixes
    polarisations (the diagonal of the Mueller matrix); a visibility whose id
    lies outside [0, n_ids) is dropped and counted like one off the grid.
    Returns (grid complex128 [P][H][W], n_dropped)."""
    taps = np.asarray(taps)
    n_ids, support = taps.shape[0], taps.shape[-1]
    vis = np.asarray(vis)
    n_pol = vis.shape[1]
    pc = pixel_coords(uvw, inv_cell_u, inv_cell_v, oversample, support, height, width, n_planes, w_min, inv_dw)
    ids = np.asarray(kernel_id, dtype=np.int64)
    valid = pc["valid"] & finite_values(vis, weights) & (ids >= 0) & (ids < n_ids)
    wv = weighted_vis(vis, weights)
    out = np.zeros((n_pol, height, width), np.complex128)
    flat = out.reshape(n_pol, -1)
    idx = np.nonzero(valid)[0]
    k = np.arange(support)
    for c0 in range(0, idx.size, chunk):
        sel = idx[c0:c0 + chunk]
        kern = taps[ids[sel], pc["plane"][sel], pc["sy"][sel], pc["sx"][sel]].astype(np.complex128)  # [n][P][S][S]
        rows = pc["y0"][sel][:, None] + k[None, :]
        cols = pc["x0"][sel][:, None] + k[None, :]
        cell = (rows[:, :, None] * width + cols[:, None, :]).ravel()
        for p in range(n_pol):
            contrib = (kern[:, p] * wv[sel, p][:, None, None]).ravel()
            flat[p] += np.bincount(cell, weights=contrib.real, minlength=height * width) \
                + 1j * np.bincount(cell, weights=contrib.imag, minlength=height * width)
    return out, int(np.count_nonzero(~valid))


def grid_table2d(vis: np.ndarray, uvw: np.ndarray, weights: Optional[np.ndarray],
                 taps2d: np.ndarray, inv_cell_u: float, inv_cell_v: float, oversample: int,
                 height: int, width: int, n_planes: int, w_min: float, inv_dw: float,
                 grid: Optional[np.ndarray] = None, chunk: int = 2048):
    """As :func:`grid_separable` with a non-separable table [planes][O][O][S][S]
    indexed [plane][sy][sx][ky][kx]."""
    taps2d = np.asarray(taps2d)
    support = taps2d.shape[-1]
    n_pol = vis.shape[1]
    pc = pixel_coords(uvw, inv_cell_u, inv_cell_v, oversample, support, height, width,
                      n_planes, w_min, inv_dw)
    pc["valid"] = pc["valid"] & finite_values(vis, weights)
    wv = weighted_vis(vis, weights)
    out = np.zeros((n_pol, height, width), np.complex128) if grid is None \
        else np.array(grid, dtype=np.complex128, copy=True)
    idx = np.nonzero(pc["valid"])[0]
    k = np.arange(support)
    flat = out.reshape(n_pol, -1)
    for c0 in range(0, idx.size, chunk):
        sel = idx[c0:c0 + chunk]
        kern = taps2d[pc["plane"][sel], pc["sy"][sel], pc["sx"][sel]].astype(np.complex128)
        rows = pc["y0"][sel][:, None] + k[None, :]
        cols = pc["x0"][sel][:, None] + k[None, :]
        cell = (rows[:, :, None] * width + cols[:, None, :]).ravel()
        for p in range(n_pol):
            contrib = (kern * wv[sel, p][:, None, None]).ravel()
            flat[p] += np.bincount(cell, weights=contrib.real, minlength=height * width) \
                + 1j * np.bincount(cell, weights=contrib.imag, minlength=height * width)
    return out, int(np.count_nonzero(~pc["valid"]))


def degrid_separable(grid: np.ndarray, uvw: np.ndarray, taps: np.ndarray, inv_cell_u: float,
                     inv_cell_v: float, oversample: int, n_planes: int = 1, w_min: float = 0.0,
                     inv_dw: float = 0.0) -> np.ndarray:
    """Adjoint of :func:`grid_separable` with unit weights (Section 6 names degridding
    as the natural next step):  V[n,p] = sum_{ky,kx} Tv Tu grid[p, y0+ky, x0+kx],
    complex128 [N][P]; dropped visibilities give 0."""
    n_pol, height, width = grid.shape
    support = taps.shape[-1]
    pc = pixel_coords(uvw, inv_cell_u, inv_cell_v, oversample, support, height, width,
                      n_planes, w_min, inv_dw)
    out = np.zeros((uvw.shape[0], n_pol), np.complex128)
    k = np.arange(support)
    for n in np.nonzero(pc["valid"])[0]:
        pl = pc["plane"][n]
        kern = np.outer(taps[pl, pc["sy"][n]], taps[pl, pc["sx"][n]])
        win = grid[:, pc["y0"][n] + k[:, None], pc["x0"][n] + k[None, :]]
        out[n] = np.sum(win * kern[None], axis=(1, 2))
    return out
