"""Pins for the FP64 oracle against facts that do not come from the oracle itself.

Each test names what fixes the expected value: a closed form, an independent
numerical route (an integral representation, an FFT, brute-force evaluation of
the analytic kernel), an invariant of the definition, or a physical identity.
"""
import math

import numpy as np
import pytest

from oracle import gridding as G
from synth import random_point_workload, tiny_kb_workload


def _i0_integral(x: float, n: int = 4096) -> float:
    """I0(x) = (1/pi) int_0^pi exp(x cos t) dt, trapezoid rule on a periodic integrand."""
    t = (np.arange(n) + 0.5) * (math.pi / n)
    return float(np.mean(np.exp(x * np.cos(t))))


# ---------------------------------------------------------------- kernel tables

def test_kb_against_integral_representation():
    """The Bessel function inside the KB window agrees with I0's integral form."""
    S, beta = 8, 8.6
    d = np.array([0.0, 0.3, 1.7, 2.5, 3.9])
    expect = np.array([_i0_integral(beta * math.sqrt(1 - (2 * x / S) ** 2)) for x in d]) / _i0_integral(beta)
    np.testing.assert_allclose(G.kaiser_bessel(d, S, beta), expect, rtol=1e-12)


def test_kb_special_cases():
    S = 8
    assert G.kaiser_bessel(0.0, S, 8.6) == pytest.approx(1.0, abs=1e-15)
    # zero at and beyond half the support (truncation), symmetric inside
    assert np.all(G.kaiser_bessel(np.array([4.0, -4.0, 4.5, 100.0]), S, 8.6) == 0.0)
    x = np.linspace(-3.9, 3.9, 41)
    np.testing.assert_array_equal(G.kaiser_bessel(x, S, 8.6), G.kaiser_bessel(-x, S, 8.6))
    # beta -> 0 is the boxcar of width S
    np.testing.assert_allclose(G.kaiser_bessel(x, S, 0.0), 1.0, rtol=0, atol=0)


def test_wkernel_zero_w_is_kb_within_fov_truncation():
    """The w = 0 W kernel is the DFT of the KB image response, so it must reproduce
    the KB window itself up to the field-of-view truncation of the taper (measured
    1.5e-3 relative at S=16; a dropped factor in the taper gives O(1) errors)."""
    S, O = 16, 8
    t0 = G.wkernel_table(S, O, [0.0])[0]
    kb = G.kaiser_bessel(G.tap_offsets(S, O), 8, 8.6)
    kb = kb / kb[0].sum()
    assert np.abs(t0.imag).max() < 1e-15
    assert np.abs(t0 - kb).max() / np.abs(kb).max() < 3e-3


def test_wkernel_dft_matches_fft_route():
    """Direct sum over the screen samples equals a zero-padded FFT of the same
    screen evaluated at delta = m/O (half-sample shift of the midpoint grid
    applied as a phase), i.e. the table is exactly a DFT of the screen."""
    S, O, M, wh = 16, 8, 64, 5.5
    nu = G.w_screen_samples(M)
    screen = G.kb_image_taper(nu, 8, 8.6) * np.exp(-1j * math.pi * wh * nu ** 2)
    spec = np.fft.fft(np.concatenate([screen, np.zeros(M * (O - 1))]))   # length M*O
    m = np.arange(-(S // 2) * O, (S // 2) * O)
    delta = m / O
    via_fft = spec[m % (M * O)] * np.exp(-2j * math.pi * delta * (0.5 / M - 0.5))
    direct = G.wkernel_1d(wh, delta, 8, 8.6, M)
    np.testing.assert_allclose(direct, via_fft, rtol=0, atol=1e-11 * np.abs(direct).max())


def test_wkernel_symmetries():
    """g_{-w}(delta) = conj g_w(delta) (real taper) and g_w(-delta) = g_w(delta)
    (even screen on a symmetric nu grid); on the table the mirror of (s, k) is
    (O - s, S - 1 - k) for s > 0 and (0, S - 2 - k) for s = 0."""
    S, O = 16, 8
    t = G.wkernel_table(S, O, [4.0, -4.0])
    np.testing.assert_allclose(t[1], np.conj(t[0]), rtol=0, atol=1e-15)
    tab = t[0]
    for s in range(O):
        for k in range(S):
            if s == 0:
                if k == S - 1:
                    assert tab[0, k] == 0.0   # delta = S/2 is outside the support
                    continue
                mk, ms = S - 2 - k, 0
            else:
                mk, ms = S - 1 - k, O - s
            assert abs(tab[s, k] - tab[ms, mk]) < 1e-14


def test_wkernel_normalisation():
    S, O = 32, 8
    t = G.wkernel_table(S, O, [0.0, 10.0])
    assert np.sum(t[0, 0]).real == pytest.approx(1.0, abs=1e-13)


def test_2d_table_limits():
    """At w = 0 the exact 2-D kernel is exactly the outer product of the separable
    one; as the field of view shrinks, the w != 0 kernel tends to it as well."""
    S, O = 8, 2
    sep = G.wkernel_table(S, O, [0.0, 3.0])
    two = G.wkernel_2d_table(S, O, [0.0, 3.0], fov=1e-3)
    outer0 = np.einsum("vk,uj->vukj", sep[0], sep[0])
    np.testing.assert_allclose(two[0], outer0, rtol=0, atol=1e-14)
    outer1 = np.einsum("vk,uj->vukj", sep[1], sep[1])
    assert np.abs(two[1] - outer1).max() < 1e-6 * np.abs(outer1).max()
    far = G.wkernel_2d_table(S, O, [3.0], fov=0.8)[0]
    assert np.abs(far - outer1).max() > 1e-3 * np.abs(outer1).max()


# ---------------------------------------------------------------- index conversion

def _coords(u, v, w=0.0, O=8, S=8, H=64, W=64, **kw):
    u, v = np.broadcast_arrays(np.atleast_1d(np.asarray(u, float)), np.atleast_1d(np.asarray(v, float)))
    uvw = np.stack([u, v, np.full(u.shape, w)], axis=1).astype(np.float64)
    return G.pixel_coords(uvw, 1.0, 1.0, O, S, H, W, **kw)


def test_pixel_coords_hand_cases():
    c = _coords(0.0, 0.0)
    assert c["fx"][0] == 32 * 8 and c["sx"][0] == 0 and c["x0"][0] == 32 - 4 + 1
    # round half to even on the oversampled grid: 2.5/8 px -> 2, 3.5/8 -> 4, -2.5/8 -> -2
    c = _coords(np.array([2.5, 3.5, -2.5, -3.5]) / 8, 0.0)
    np.testing.assert_array_equal(c["fx"] - 256, [2, 4, -2, -4])
    # one pixel plus three eighths
    c = _coords(1.375, -1.375)
    assert (c["fx"][0], c["sx"][0], c["x0"][0] + 3) == (256 + 11, 3, 33)
    assert (c["fy"][0], c["sy"][0]) == (256 - 11, 5)


def test_pixel_coords_mirror_exact():
    rng = np.random.default_rng(3)
    u = rng.uniform(-20, 20, 5000)
    u[:50] = (rng.integers(-100, 100, 50) + 0.5) / 8        # exact ties
    c1, c2 = _coords(u, u), _coords(-u, -u)
    np.testing.assert_array_equal(c1["fx"] + c2["fx"], 64 * 8)


def test_pixel_coords_drop_rules():
    S, W = 8, 64
    # footprint exactly touching each edge is kept; one pixel further is dropped
    lo = (0 + S // 2 - 1) - 32          # x0 = 0
    hi = (W - S + S // 2 - 1) - 32      # x0 + S = W
    c = _coords(np.array([lo, lo - 1, hi, hi + 1, np.nan, np.inf, 0.0]), 0.0)
    np.testing.assert_array_equal(c["valid"], [True, False, True, False, False, False, True])
    c = _coords(np.zeros(4), np.zeros(4), w=0.0, n_planes=4, w_min=-1.0, inv_dw=1.5)
    assert c["plane"][0] == 2 and c["valid"].all()
    uvw = np.array([[0, 0, -1.34], [0, 0, -1.33], [0, 0, 1.0], [0, 0, 1.34], [0, 0, np.nan]])
    c = G.pixel_coords(uvw, 1.0, 1.0, 8, 8, 64, 64, n_planes=4, w_min=-1.0, inv_dw=1.5)
    np.testing.assert_array_equal(c["plane"][:4], [-1, 0, 3, 4])
    np.testing.assert_array_equal(c["valid"], [False, True, True, False, False])


def test_finite_values_hand_cases():
    """The value half of the drop rule, by hand: a visibility is kept only when
    every real and imaginary part of its values, and every one of its weights,
    is finite; a bad value in one polarisation drops the whole visibility, and
    its finite neighbours are kept.  Holds for complex64 and complex128 input."""
    nan, inf = np.nan, np.inf
    vis = np.ones((8, 4), np.complex64) * np.complex64(1 - 2j)
    vis[1, 2] = complex(nan, 0.5)              # NaN in Re
    vis[2, 0] = complex(0.25, inf)             # +inf in Im
    vis[3, 3] = complex(-1.0, -inf)            # -inf in Im
    vis[5, 1] = complex(3.0e38, -3.0e38)       # large but finite: kept
    w = np.ones((8, 4), np.float32)
    w[4, 1] = nan                              # NaN in one of four weights
    w[6, 3] = -inf                             # -inf weight
    w[7, 0] = 0.0                              # a zero weight is a finite weight
    keep = [True, False, False, False, False, True, False, True]
    assert G.finite_values(vis, w).tolist() == keep
    # without weights only the values decide
    assert G.finite_values(vis, None).tolist() == [True, False, False, False, True, True, True, True]
    assert G.finite_values(vis.astype(np.complex128), w).tolist() == keep
    # single polarisation, and an empty stream
    assert G.finite_values(vis[:, :1], None).tolist() == [True, True, False, True, True, True, True, True]
    assert G.finite_values(vis[:0], w[:0]).shape == (0,)


def test_nonfinite_values_are_dropped_from_the_grid():
    """A visibility with a non-finite value or weight leaves the grid exactly as
    if it were absent (no NaN or inf reaches any cell), and is counted as
    dropped.  Expected grid: the definition summed by hand, in a Python loop
    over the visibilities known to be clean, without finite_values."""
    wl = _wl(n=24, P=4, H=40, W=48, S=8, O=8, seed=9, weights=True)
    bad = [2, 7, 8, 15]
    wl.vis[2, 1] = complex(np.nan, 0.0)
    wl.vis[7, 3] = complex(0.0, -np.inf)
    wl.weights[8, 0] = np.inf
    wl.weights[15, 2] = np.nan
    taps = G.kb_table(8, 8, 8.6)
    g, dropped = _grid(wl, taps)
    assert np.isfinite(g).all()
    c = G.pixel_coords(wl.uvw, 1, 1, 8, 8, 40, 48)
    assert c["valid"].all()                    # nothing else is dropped in this draw
    assert dropped == len(bad)
    ref = np.zeros((4, 40, 48), np.complex128)
    for n in range(24):
        if n in bad:
            continue
        k = np.outer(taps[0, c["sy"][n]], taps[0, c["sx"][n]])
        for p in range(4):
            val = complex(wl.vis[n, p]) * float(wl.weights[n, p])
            ref[p, c["y0"][n]:c["y0"][n] + 8, c["x0"][n]:c["x0"][n] + 8] += val * k
    np.testing.assert_allclose(g, ref, rtol=0, atol=1e-13 * np.abs(ref).max())


# ---------------------------------------------------------------- gridding

def _wl(n=60, P=2, H=40, W=48, S=8, O=8, seed=0, planes=1, kernel="kb", weights=True, margin=0):
    return random_point_workload(n, P, H, W, S, O, seed, n_planes=planes, margin=margin,
                                 weights=weights, kernel=kernel)


def _grid(wl, taps, **kw):
    return G.grid_separable(wl.vis, wl.uvw, wl.weights, taps, wl.inv_cell_u, wl.inv_cell_v,
                            wl.oversample, wl.height, wl.width, wl.n_planes, wl.w_min, wl.inv_dw, **kw)


def test_brute_force_analytic_kb():
    """Evaluating kb(x - px) kb(y - py) at every cell for every visibility, with
    no table and no footprint window, reproduces the table-based grid."""
    wl = _wl(n=40, P=2, H=24, W=32, S=8, O=8, seed=5)
    g, dropped = _grid(wl, G.kb_table(8, 8, 8.6))
    assert dropped == 0
    c = G.pixel_coords(wl.uvw, 1, 1, 8, 8, 24, 32)
    px, py = c["fx"] / 8.0, c["fy"] / 8.0
    ys, xs = np.mgrid[0:24, 0:32]
    ref = np.zeros((2, 24, 32), np.complex128)
    wv = wl.vis.astype(np.complex128) * wl.weights
    for n in range(40):
        k = G.kaiser_bessel(xs - px[n], 8, 8.6) * G.kaiser_bessel(ys - py[n], 8, 8.6)
        ref += wv[n][:, None, None] * k[None]
    np.testing.assert_allclose(g, ref, rtol=0, atol=1e-13 * np.abs(ref).max())


def test_delta_table_places_each_visibility_on_its_cell():
    S, O = 8, 8
    taps = np.zeros((1, O, S))
    taps[:, :, S // 2 - 1] = 1.0
    wl = _wl(n=30, P=1, S=S, O=O, seed=2, weights=False)
    g, _ = _grid(wl, taps)
    c = G.pixel_coords(wl.uvw, 1, 1, O, S, wl.height, wl.width)
    ref = np.zeros_like(g)
    np.add.at(ref[0], (c["fy"] >> 3, c["fx"] >> 3), wl.vis[:, 0].astype(np.complex128))
    np.testing.assert_array_equal(g, ref)


@pytest.mark.parametrize("kernel", ["kb", "wsep"])
def test_flux_conservation(kernel):
    S, O = 16, 8
    wl = _wl(n=200, P=4, H=64, W=80, S=S, O=O, seed=7, planes=(9 if kernel == "wsep" else 1),
             kernel=kernel, margin=4)
    taps = G.kb_table(S, O, 8.6) if kernel == "kb" else G.wkernel_table(S, O, wl.plane_w_hat())
    g, dropped = _grid(wl, taps)
    c = G.pixel_coords(wl.uvw, 1, 1, O, S, wl.height, wl.width, wl.n_planes, wl.w_min, wl.inv_dw)
    assert dropped == np.count_nonzero(~c["valid"]) and dropped > 0
    v = c["valid"]
    su = taps[c["plane"][v], c["sx"][v]].sum(axis=1)
    sv = taps[c["plane"][v], c["sy"][v]].sum(axis=1)
    expect = ((wl.vis[v].astype(np.complex128) * wl.weights[v]) * (su * sv)[:, None]).sum(axis=0)
    np.testing.assert_allclose(g.sum(axis=(1, 2)), expect, rtol=1e-12)


def test_linearity_superposition_permutation():
    S, O = 16, 8
    wl = _wl(n=150, P=4, H=64, W=64, S=S, O=O, seed=9, planes=5, kernel="wsep")
    taps = G.wkernel_table(S, O, wl.plane_w_hat())
    g, _ = _grid(wl, taps)
    # superposition: grid(A) + grid(B) = grid(A u B), and accumulation into an input grid
    import copy
    a, b = copy.copy(wl), copy.copy(wl)
    a.uvw, a.vis, a.weights = wl.uvw[:70], wl.vis[:70], wl.weights[:70]
    b.uvw, b.vis, b.weights = wl.uvw[70:], wl.vis[70:], wl.weights[70:]
    ga, _ = _grid(a, taps)
    gab, _ = _grid(b, taps, grid=ga)
    np.testing.assert_allclose(gab, g, rtol=0, atol=1e-13 * np.abs(g).max())
    # scaling (by factors that are exact in complex64)
    for f in (2j, -0.5):
        s = copy.copy(wl)
        s.vis = (wl.vis * f).astype(np.complex64)
        gs, _ = _grid(s, taps)
        np.testing.assert_allclose(gs, g * f, rtol=0, atol=1e-12 * np.abs(g).max())
    # permutation
    perm = np.random.default_rng(1).permutation(wl.n_vis)
    p = copy.copy(wl)
    p.uvw, p.vis, p.weights = wl.uvw[perm], wl.vis[perm], wl.weights[perm]
    gp, _ = _grid(p, taps)
    np.testing.assert_allclose(gp, g, rtol=0, atol=1e-13 * np.abs(g).max())


def test_hermitian_twin_symmetry():
    """Adding each visibility's twin (-u, -v, -w, conj V) makes the grid Hermitian
    about the centre cell: G[H/2 + j, W/2 + i] = conj G[H/2 - j, W/2 - i]."""
    S, O, H, W = 16, 8, 64, 64
    wl = _wl(n=120, P=2, H=H, W=W, S=S, O=O, seed=11, planes=7, kernel="wsep", weights=False)
    taps = G.wkernel_table(S, O, wl.plane_w_hat())
    import copy
    tw = copy.copy(wl)
    tw.uvw = np.concatenate([wl.uvw, -wl.uvw])
    tw.vis = np.concatenate([wl.vis, np.conj(wl.vis)])
    c1 = G.pixel_coords(wl.uvw, 1, 1, O, S, H, W, 7, wl.w_min, wl.inv_dw)
    c2 = G.pixel_coords(-wl.uvw, 1, 1, O, S, H, W, 7, wl.w_min, wl.inv_dw)
    assert np.all(c1["plane"] + c2["plane"] == 6)   # symmetric planes
    g, _ = _grid(tw, taps)
    mirrored = np.conj(g[:, (H - np.arange(1, H)) % H][:, :, (W - np.arange(1, W)) % W])
    np.testing.assert_allclose(g[:, 1:, 1:], mirrored, rtol=0, atol=1e-13 * np.abs(g).max())
    assert np.abs(g[:, 0, :]).max() == 0 and np.abs(g[:, :, 0]).max() == 0


def test_point_source_focuses_only_with_correct_w_correction():
    """Physical pin on the kernel sign, the w scaling and the u/v -> cell
    convention: visibilities of a point source at (l0, m0), gridded with
    W-projection and imaged by a direct transform at (l0, m0), add coherently
    (|I| ~ N) only if the W kernel undoes the source's w phase.  The same data
    with the kernel's w sign flipped, or with w ignored, stay incoherent."""
    rng = np.random.default_rng(4)
    S, O, Ng, fov = 16, 8, 64, 0.2
    du = 1.0 / fov                                    # cell size in wavelengths
    l0, m0 = 0.06, -0.045
    n0 = math.sqrt(1 - l0 * l0 - m0 * m0)
    N = 400
    half = (Ng / 2 - S / 2 - 2) * du
    w_max = (S - 8) / fov ** 2                          # largest w the support can correct
    uvw = np.stack([rng.uniform(-half, half, N), rng.uniform(-half, half, N),
                    rng.uniform(-w_max, w_max, N)], axis=1)
    vis = np.exp(-2j * math.pi * (uvw[:, 0] * l0 + uvw[:, 1] * m0 + uvw[:, 2] * (n0 - 1)))[:, None]
    n_planes = 129
    w_min, inv_dw = -w_max, (n_planes - 1) / (2 * w_max)
    w_planes = w_min + np.arange(n_planes) / inv_dw
    ys, xs = np.mgrid[0:Ng, 0:Ng]
    probe = np.exp(2j * math.pi * ((xs - Ng / 2) * du * l0 + (ys - Ng / 2) * du * m0))

    def image_at_source(w_hat_scale):
        taps = G.wkernel_table(S, O, w_planes * w_hat_scale)
        g, dropped = G.grid_separable(vis, uvw, None, taps, 1 / du, 1 / du, O, Ng, Ng,
                                      n_planes, w_min, inv_dw)
        assert dropped == 0
        return abs(np.sum(g[0] * probe))

    good = image_at_source(fov ** 2)
    flipped = image_at_source(-fov ** 2)
    ignored = image_at_source(0.0)
    # coherent sum: N times the normalised taper (c M t(nu)) on each axis at the source
    t = G.kb_image_taper(np.array([l0 / fov, m0 / fov]), 8, 8.6)
    cm = G.wkernel_norm(S, 8, 8.6, 4 * S) * 4 * S
    assert good == pytest.approx(N * cm * cm * t[0] * t[1], rel=0.02)
    assert flipped < 0.2 * good and ignored < 0.2 * good


def test_tiny_config_has_no_drops_and_numpy_c_agree(c_oracle):
    wl = tiny_kb_workload()
    taps = G.kb_table(8, 8, 8.6)
    g1, d1 = _grid(wl, taps)
    g2, d2 = c_oracle.grid_separable(wl.vis, wl.uvw, None, taps, wl.inv_cell_u, wl.inv_cell_v,
                                     8, 512, 512)
    assert d1 == d2 == 0
    np.testing.assert_allclose(g2, g1, rtol=0, atol=1e-12 * np.abs(g1).max())


def test_c_oracle_sampled_rows_and_coords(c_oracle):
    wl = _wl(n=300, P=4, H=64, W=72, S=16, O=8, seed=13, planes=5, kernel="wsep", margin=3)
    taps = G.wkernel_table(16, 8, wl.plane_w_hat())
    g, d = _grid(wl, taps)
    rows = [0, 5, 17, 40, 63]
    gr, dr = c_oracle.grid_separable(wl.vis, wl.uvw, wl.weights, taps, 1.0, 1.0, 8, 64, 72,
                                     5, wl.w_min, wl.inv_dw, rows=rows)
    assert d == dr
    np.testing.assert_allclose(gr, g[:, rows], rtol=0, atol=1e-12 * np.abs(g).max())
    cc = c_oracle.pixel_coords(wl.uvw, 1.0, 1.0, 8, 16, 64, 72, 5, wl.w_min, wl.inv_dw)
    cn = G.pixel_coords(wl.uvw, 1.0, 1.0, 8, 16, 64, 72, 5, wl.w_min, wl.inv_dw)
    np.testing.assert_array_equal(cc["valid"], cn["valid"])
    for k in ("x0", "y0", "sx", "sy", "plane"):
        np.testing.assert_array_equal(cc[k][cn["valid"]], cn[k][cn["valid"]])


def test_degrid_is_adjoint_of_grid():
    """<grid(V), G> = <V, degrid(G)> for unit weights."""
    S, O = 16, 8
    wl = _wl(n=50, P=2, H=32, W=40, S=S, O=O, seed=21, planes=3, kernel="wsep", weights=False)
    taps = G.wkernel_table(S, O, wl.plane_w_hat())
    g, _ = _grid(wl, taps)
    rng = np.random.default_rng(0)
    probe = rng.standard_normal(g.shape) + 1j * rng.standard_normal(g.shape)
    lhs = np.vdot(probe, g)
    dg = G.degrid_separable(probe, wl.uvw, taps, 1.0, 1.0, O, 3, wl.w_min, wl.inv_dw)
    rhs = np.vdot(dg, wl.vis.astype(np.complex128))
    # the adjoint of multiplication by the kernel is multiplication by its conjugate
    dgc = G.degrid_separable(probe, wl.uvw, np.conj(taps), 1.0, 1.0, O, 3, wl.w_min, wl.inv_dw)
    rhs_c = np.vdot(dgc, wl.vis.astype(np.complex128))
    assert lhs == pytest.approx(rhs_c, rel=1e-12)
    assert abs(lhs - rhs) > 1e-6 * abs(lhs)


def test_wkernel_2d_at_matches_table_entries():
    """The per-offset evaluation and the row-column table give the same taps."""
    S, O = 16, 4
    whs = [3.5, -2.0]
    t = G.wkernel_2d_table(S, O, whs, 0.5)
    d = G.tap_offsets(S, O)
    for p, wh in enumerate(whs):
        for sv in range(O):
            for su in range(O):
                np.testing.assert_allclose(G.wkernel_2d_at(wh, d[su], d[sv], 0.5, S), t[p, sv, su],
                                           atol=1e-13, rtol=0)


def test_continuous_w2d_grid_equals_table_grid_on_table_points():
    """Visibilities placed exactly on a plane centre and an oversampled phase:
    the continuous-kernel gridder and the 2-D table gridder agree, so the
    continuous reference uses the same cells, signs and offsets."""
    S, O, H, W, n_planes = 8, 4, 64, 64, 5
    rng = np.random.default_rng(11)
    n = 40
    w_min, inv_dw, whs = -100.0, (n_planes - 1) / 200.0, 0.03
    plane = rng.integers(0, n_planes, n)
    w = w_min + plane / inv_dw
    fx = rng.integers((S // 2 + 1) * O, (W - S // 2 - 1) * O, n)
    fy = rng.integers((S // 2 + 1) * O, (H - S // 2 - 1) * O, n)
    u = (fx - (W // 2) * O) / O
    v = (fy - (H // 2) * O) / O
    uvw = np.stack([u, v, w], axis=1)
    vis = (rng.standard_normal((n, 1)) + 1j * rng.standard_normal((n, 1))).astype(np.complex64)
    wh_planes = (w_min + np.arange(n_planes) / inv_dw) * whs
    table = G.wkernel_2d_table(S, O, wh_planes, 0.5)
    ref, drop_t = G.grid_table2d(vis, uvw, None, table, 1.0, 1.0, O, H, W, n_planes, w_min, inv_dw)
    got, drop_c = G.grid_w2d_continuous(vis, uvw, None, 1.0, 1.0, O, S, H, W, n_planes, w_min, inv_dw,
                                        whs, 0.5)
    assert drop_t == drop_c == 0
    np.testing.assert_allclose(got, ref, atol=1e-12 * np.abs(ref).max(), rtol=0)
    # off a table point the two differ (the continuous reference is not the table)
    uvw2 = uvw.copy()
    uvw2[:, 2] += 0.3 / inv_dw
    got2, _ = G.grid_w2d_continuous(vis, uvw2, None, 1.0, 1.0, O, S, H, W, n_planes, w_min, inv_dw,
                                    whs, 0.5)
    assert np.linalg.norm(got2 - ref) > 1e-3 * np.linalg.norm(ref)


def _coords_of(x0, y0, sx, sy, plane, valid):
    return {"x0": np.array(x0), "y0": np.array(y0), "sx": np.array(sx), "sy": np.array(sy),
            "plane": np.array(plane), "valid": np.array(valid, bool)}


def test_compress_hand_case():
    """Runs of equal (x0, y0, sx, sy, plane) among consecutive kept visibilities
    merge; a changed key or a dropped visibility starts a new run."""
    c = _coords_of([5, 5, 5, 6, 5, 5, 5, 5], [2, 2, 2, 2, 2, 2, 2, 2], [1, 1, 1, 1, 1, 1, 1, 2],
                [0, 0, 0, 0, 0, 0, 0, 0], [0, 0, 0, 0, 0, 0, 0, 0], [1, 1, 1, 1, 0, 1, 1, 1])
    wv = (np.arange(8) + 1j * np.arange(8)[::-1])[:, None] * np.array([[1.0, 10.0]])
    out, sums, heads = G.compress(c, wv)
    assert heads.tolist() == [0, 3, 5, 7]
    np.testing.assert_array_equal(sums, np.array([wv[0] + wv[1] + wv[2], wv[3], wv[5] + wv[6], wv[7]]))
    assert out["x0"].tolist() == [5, 6, 5, 5] and out["sx"].tolist() == [1, 1, 1, 2] and out["valid"].all()


def test_compress_matches_brute_force_and_keeps_the_grid():
    """On the 2 s-dump tracks (first 12 baselines): the run structure equals a
    plain loop over the stream, and gridding the compressed stream gives the
    grid of the full stream (FP64, 1e-12)."""
    from synth import compression_workload
    wl = compression_workload(n_baselines=12, n_pol=2, grid=512, support=8, n_planes=4)
    pc = G.pixel_coords(wl.uvw, wl.inv_cell_u, wl.inv_cell_v, 8, 8, 512, 512, 4, wl.w_min, wl.inv_dw)
    wv = G.weighted_vis(wl.vis, None)
    out, sums, heads = G.compress(pc, wv)
    keys = list(zip(*(pc[k].tolist() for k in ("x0", "y0", "sx", "sy", "plane"))))
    bf_heads, prev = [], None
    for i, (k, ok) in enumerate(zip(keys, pc["valid"].tolist())):
        if ok and k != prev:
            bf_heads.append(i)
        prev = k if ok else None
    assert heads.tolist() == bf_heads
    assert wl.n_vis / heads.size > 2.0                  # short 2 s dumps do merge
    taps = G.wkernel_table(8, 8, wl.plane_w_hat())
    full, _ = G.grid_separable(wl.vis, wl.uvw, None, taps, wl.inv_cell_u, wl.inv_cell_v, 8, 512, 512, 4,
                               wl.w_min, wl.inv_dw)
    comp = G.grid_coords(out, sums, taps, np.zeros((2, 512, 512), np.complex128))
    assert np.abs(comp - full).max() <= 1e-12 * np.abs(full).max()
