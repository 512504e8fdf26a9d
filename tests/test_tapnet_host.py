"""Host-side logic of the tap-network trainer (no device work)."""
import math

import numpy as np
import pytest

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def T():
    from paper_1605_07023_amd import binding, tapnet
    import os
    if not os.path.exists(binding.library_path()):
        import __graft_entry__
        __graft_entry__.build()
    return tapnet


def test_blob_round_trip_and_layout(T):
    p = T.init_params(3)
    blob = T.params_to_blob(p, 12616, header=(0.5, 0.25, 2.0, 0.0))
    assert blob.dtype == np.float32 and blob.size == 12616
    assert list(blob[:3]) == [0.5, 0.25, 2.0]
    q = T.blob_to_params(blob)
    for k in p:
        np.testing.assert_allclose(q[k], p[k].astype(np.float32), rtol=0, atol=0)
    assert np.all(q["W1"][36:] == 0)                 # rows of the always-zero features
    # W stored [in][out] row-major after the header
    assert blob[T.OFFSETS["W2"] + 3 * 64 + 5] == np.float32(p["W2"][3, 5])
    assert T.OFFSETS["b4"] + 2 == 12614


def test_checkpoint_round_trip_on_host(T, tmp_path):
    net = T.TapNet("cpu", seed=1)
    net.m += 0.5
    net.v += 0.25
    net.step = 17
    net.meta = {"note": "x"}
    path = str(tmp_path / "ck.npz")
    net.save(path)
    back = T.TapNet.load(path, "cpu")
    assert back.step == 17 and back.meta == {"note": "x"}
    assert torch.equal(back.blob, net.blob) and torch.equal(back.m, net.m) and torch.equal(back.v, net.v)
    bad = str(tmp_path / "bad.npz")
    np.savez(bad, blob=np.zeros(5, np.float32), m=np.zeros(5), v=np.zeros(5), step=np.array([1]))
    with pytest.raises(ValueError):
        T.TapNet.load(bad, "cpu")


def test_nan_loss_aborts_training(T):
    assert T.check_loss(0.5, 3) == 0.5
    for bad in (float("nan"), float("inf")):
        with pytest.raises(T.TrainingDiverged):
            T.check_loss(bad, 10)


def test_plane_mappings(T):
    """Fine planes cover the coarse grid's rounding interval; the header maps a
    plane index to w_hat / w_hat_range."""
    w_min, inv_dw, n = -50.0, 31 / 100.0, 32
    wf, invf = T.fine_planes(w_min, inv_dw, n, 4096)
    lo_c, hi_c = w_min - 0.5 / inv_dw, w_min + (n - 0.5) / inv_dw
    assert math.isclose(wf - 0.5 / invf, lo_c, rel_tol=0, abs_tol=1e-12)
    assert math.isclose(wf + (4096 - 0.5) / invf, hi_c, rel_tol=0, abs_tol=1e-9)
    off, step = T.header_for_planes(w_min, inv_dw, 0.16, 16.0)
    for p in (0, 7, 31):
        w_hat = (w_min + p / inv_dw) * 0.16
        assert math.isclose(off + p * step, w_hat / 16.0, rel_tol=1e-12, abs_tol=1e-12)
