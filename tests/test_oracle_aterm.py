"""Pins of the oracle's gridding with per-visibility, per-polarisation
non-separable GCFs (Section 6, A-projection): a brute-force loop on a tiny
case, a delta table whose entries show the index order (id, plane, phases,
polarisation, row, column), the reduction to the pinned 2-D table gridder
when the GCF depends on neither id nor polarisation, and the drop rule for
ids out of range."""
import numpy as np

from oracle import gridding as G


def _case(seed, n, P, S, O, n_planes, n_ids, H=24, W=24):
    rng = np.random.default_rng(seed)
    uvw = np.stack([rng.uniform(-6, 6, n), rng.uniform(-6, 6, n), rng.uniform(-1, 1, n)], axis=1)
    vis = (rng.standard_normal((n, P)) + 1j * rng.standard_normal((n, P))).astype(np.complex64)
    wts = rng.uniform(0.5, 2.0, (n, P)).astype(np.float32)
    ids = rng.integers(0, n_ids, n).astype(np.int32)
    taps = (rng.standard_normal((n_ids, n_planes, O, O, P, S, S))
            + 1j * rng.standard_normal((n_ids, n_planes, O, O, P, S, S)))
    return uvw, vis, wts, ids, taps, H, W


def test_grid_aterm_brute_force():
    n, P, S, O, n_planes, n_ids = 40, 4, 4, 2, 3, 3
    uvw, vis, wts, ids, taps, H, W = _case(1, n, P, S, O, n_planes, n_ids)
    w_min, inv_dw = -1.0, 1.0
    got, dropped = G.grid_aterm(vis, uvw, wts, ids, taps, 1.0, 1.0, O, H, W, n_planes, w_min, inv_dw)
    pc = G.pixel_coords(uvw, 1.0, 1.0, O, S, H, W, n_planes, w_min, inv_dw)
    want = np.zeros((P, H, W), np.complex128)
    n_bad = 0
    for i in range(n):
        if not pc["valid"][i]:
            n_bad += 1
            continue
        for p in range(P):
            v = complex(vis[i, p]) * float(wts[i, p])
            for ky in range(S):
                for kx in range(S):
                    t = taps[ids[i], pc["plane"][i], pc["sy"][i], pc["sx"][i], p, ky, kx]
                    want[p, pc["y0"][i] + ky, pc["x0"][i] + kx] += v * t
    assert dropped == n_bad
    np.testing.assert_allclose(got, want, rtol=0, atol=1e-12)


def test_grid_aterm_delta_table_index_order():
    """T[id, plane, sy, sx, p] is one value c at cell (ky, kx) = (id + p, 2 id + 1 + plane): a
    visibility at uv = 0 (phases 0) lands at (y0 + ky, x0 + kx) of polarisation p with c V."""
    P, S, O, n_planes, n_ids, H, W = 4, 8, 1, 2, 3, 32, 32
    taps = np.zeros((n_ids, n_planes, O, O, P, S, S), np.complex128)
    for i in range(n_ids):
        for pl in range(n_planes):
            for p in range(P):
                taps[i, pl, 0, 0, p, i + p, 2 * i + 1 + pl] = (i + 1) + 1j * (p + 1) + 10 * pl
    cases = [(0, 0), (2, 1), (1, 0), (2, 0)]                # (id, plane)
    uvw = np.array([[0.0, 0.0, -0.5 + pl] for _, pl in cases])   # w_min -0.5, inv_dw 1: plane = rint(w + 0.5)
    vis = np.array([[1 + 2j, 3 - 1j, -2 + 0.5j, 4j]] * len(cases), np.complex64)
    ids = np.array([i for i, _ in cases], np.int32)
    got, dropped = G.grid_aterm(vis, uvw, None, ids, taps, 1.0, 1.0, O, H, W, n_planes, -0.5, 1.0)
    assert dropped == 0
    x0 = y0 = W // 2 - S // 2 + 1
    want = np.zeros((P, H, W), np.complex128)
    for n, (i, pl) in enumerate(cases):
        for p in range(P):
            c = (i + 1) + 1j * (p + 1) + 10 * pl
            want[p, y0 + i + p, x0 + 2 * i + 1 + pl] += c * complex(vis[n, p])
    np.testing.assert_array_equal(got, want)


def test_grid_aterm_reduces_to_the_2d_table():
    """A GCF that depends on neither the id nor the polarisation gives grid_table2d's grid."""
    n, P, S, O, n_planes, n_ids = 300, 4, 6, 4, 3, 5
    uvw, vis, wts, ids, _, H, W = _case(2, n, P, S, O, n_planes, n_ids, 40, 40)
    rng = np.random.default_rng(9)
    t2 = rng.standard_normal((n_planes, O, O, S, S)) + 1j * rng.standard_normal((n_planes, O, O, S, S))
    taps = np.broadcast_to(t2[None, :, :, :, None], (n_ids, n_planes, O, O, P, S, S))
    got, d1 = G.grid_aterm(vis, uvw, wts, ids, taps, 1.0, 1.0, O, H, W, n_planes, -1.0, 1.0)
    want, d2 = G.grid_table2d(vis, uvw, wts, t2, 1.0, 1.0, O, H, W, n_planes, -1.0, 1.0)
    assert d1 == d2
    np.testing.assert_allclose(got, want, rtol=0, atol=1e-11)


def test_grid_aterm_drops_ids_out_of_range():
    n, P, S, O, n_planes, n_ids = 200, 1, 4, 2, 1, 4
    uvw, vis, wts, ids, taps, H, W = _case(3, n, P, S, O, n_planes, n_ids)
    ok, d_ok = G.grid_aterm(vis, uvw, None, ids, taps, 1.0, 1.0, O, H, W, n_planes, 0.0, 0.0)
    bad = ids.copy()
    bad[::7] = n_ids                                       # out of range
    bad[3::11] = -1
    hit = (np.arange(n) % 7 == 0) | (np.arange(n) % 11 == 3)
    got, d_bad = G.grid_aterm(vis, uvw, None, bad, taps, 1.0, 1.0, O, H, W, n_planes, 0.0, 0.0)
    keep, d_keep = G.grid_aterm(vis[~hit], uvw[~hit], None, ids[~hit], taps, 1.0, 1.0, O, H, W, n_planes, 0.0, 0.0)
    np.testing.assert_allclose(got, keep, rtol=0, atol=1e-12)
    pc = G.pixel_coords(uvw, 1.0, 1.0, O, S, H, W, n_planes, 0.0, 0.0)
    assert d_bad == d_ok + int(np.count_nonzero(hit & pc["valid"]))
