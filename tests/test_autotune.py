"""Host logic of the autotuner: the candidate space and the memo."""
import json

import pytest

pytest.importorskip("torch")


def test_candidate_space():
    from paper_1605_07023_amd import autotune as A
    c4 = A.candidates(4, 32, variants=(1,))
    pairs = {(t.cu, t.cv) for t in c4}
    # the paper's coarsening range, filtered by the register budget (cu*cv*P <= 64)
    assert (1, 1) in pairs and (4, 4) in pairs and (8, 2) in pairs and (8, 8) not in pairs
    assert all(t.cu * t.cv * 4 <= 64 and t.variant == 1 for t in c4)
    c1 = A.candidates(1, 8, variants=(1,))
    assert (8, 8) in {(t.cu, t.cv) for t in c1}
    m = A.candidates(4, 32, variants=(2,))
    assert {(t.vis_per_wg, t.wg_v) for t in m} == {(sl, rg) for sl in A.SEG_LENS for rg in (2, 3, 4, 6)}
    assert all(t.variant == 2 for t in m)
    # row groups per wave must divide the window's row groups (4-row groups at P = 4, 16-row at P = 1)
    for P, S in [(4, 16), (4, 32), (4, 56), (1, 16), (1, 32), (1, 56)]:
        w = 32 if S <= 16 else 48 if S <= 32 else 64
        assert all((w // (16 // P)) % rg == 0 for rg in A.row_group_options(P, S))
    assert A.candidates(4, 60, variants=(2,)) == []
    # tile orders: flat (0, 0) and a rectangle of at most 16 blocks along u
    shapes = {(t.wg_u, t.wg_v) for t in A.candidates(4, 32, variants=(1,)) if (t.cu, t.cv) == (4, 2)}
    assert shapes == {(0, 0), (9, 7)}


def test_memo_roundtrip_and_corruption(tmp_path):
    from paper_1605_07023_amd import autotune as A
    from paper_1605_07023_amd import binding as B
    p = tmp_path / "memo.json"
    m = A.Memo(str(p))
    k = A.memo_key("gfx950", 4, 32, "wsep", 0, 4096, (2,))
    assert m.get(k) is None
    m.put(k, B.GrTuning(0, 0, 0, 0, 2048, 2), 1.5)
    m.save()
    m2 = A.Memo(str(p))
    t = m2.get(k)
    assert (t.vis_per_wg, t.variant) == (2048, 2)
    assert A.memo_key("gfx950", 4, 32, "wsep", 0, 3000, (2,)) == k     # same grid side class
    p.write_text("{not json")
    assert A.Memo(str(p)).get(k) is None                               # corrupt -> defaults
    p.write_text(json.dumps({k: {"tuning": [1, 2]}}))
    assert A.Memo(str(p)).get(k) is None                               # malformed entry ignored


def test_memo_installs_into_the_library(tmp_path):
    """Entries saved with their library class go into the library's memo, where
    calls without a tuning read them; entries of other devices stay out."""
    from paper_1605_07023_amd import autotune as A
    from paper_1605_07023_amd import binding as B
    B.gr_tuning_memo_clear()
    p = tmp_path / "memo.json"
    m = A.Memo(str(p))
    k = B.GrKernel(B.GR_SEPARABLE, B.GR_F32, 1, 32, 8, 32, -1.0, 1.0, None)
    m.put(A.memo_key("devA", 4, 32, "wsep", 0, 4096, (1, 2)), B.GrTuning(8, 1, 0, 0, 0, 1), 2.0,
          A._c_class(4, k, 4096, 0))
    m.put(A.memo_key("devB", 4, 32, "wsep", 0, 2048, (1, 2)), B.GrTuning(4, 2, 0, 0, 0, 1), 2.0,
          A._c_class(4, k, 2048, 0))
    m.put(A.memo_key("devA", 4, 16, "wsep", 0, 4096, (2,)), B.GrTuning(0, 0, 0, 4, 2048, 2), 1.0)  # no class
    m.save()
    assert A.Memo(str(p)).install("devA") == 1
    got = B.gr_tuning_memo_get(4, k, 4096, 4096, 0)
    assert (got.cu, got.cv, got.variant) == (8, 1, 1)
    assert B.gr_tuning_memo_get(4, k, 2048, 2048, 0) is None
    B.gr_tuning_memo_clear()
