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
    assert [t.vis_per_wg for t in m] == list(A.SEG_LENS) and all(t.variant == 2 for t in m)
    assert A.candidates(4, 60, variants=(2,)) == []


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
