"""Recorded HBM traffic is reported only for the kernel sources it was
measured on (host logic, no GPU)."""
import json

from paper_2602_07860_amd import profiling


def test_traffic_lookup_matches_source_hash(tmp_path):
    p = tmp_path / "traffic.json"
    good = {"bytes_per_launch": 123.0, "source_sha256": profiling.source_hash()}
    stale = {"bytes_per_launch": 456.0, "source_sha256": "0" * 64}
    p.write_text(json.dumps({"k_bg_bwd@medium": good, "k_bg_bwd@large": stale}))
    assert profiling.lookup(str(p), "k_bg_bwd", "medium") == 123.0
    assert profiling.lookup(str(p), "k_bg_bwd", "large") is None
    assert profiling.lookup(str(p), "k_fg", "medium") is None
    assert profiling.lookup(str(tmp_path / "missing.json"), "k_bg_bwd", "medium") is None


def test_batch_class_is_coarse_and_stable():
    import torch
    from paper_2602_07860_amd import batch as BT
    from paper_2602_07860_amd import render as R
    from paper_2602_07860_amd import workloads as wl
    scs = wl.make_batch(seed=3, n=4)
    sts = [R.scene_tensors(sc, "cpu") for sc in scs]
    c1 = BT.batch_class(sts, "fast")
    assert c1 == BT.batch_class(list(reversed(sts)), "fast")
    assert c1 != BT.batch_class(sts, "recompute")
    assert c1.startswith("fast|n4|")


def test_source_hash_ignores_comments_only():
    from paper_2602_07860_amd import profiling as P
    a = 'int f(int x) { return x + 1; } // one\n/* two */\nconst char *s = "// not a comment";\n'
    b = 'int f(int x)  {\n  return x + 1;  // changed comment\n}\nconst char *s = "// not a comment";\n'
    c = 'int f(int x) { return x + 2; }\nconst char *s = "// not a comment";\n'
    d = 'int f(int x) { return x + 1; }\nconst char *s = "// other";\n'
    assert P.code_text(a) == P.code_text(b)
    assert P.source_hash([a]) == P.source_hash([b])
    assert P.source_hash([a]) != P.source_hash([c])
    assert P.source_hash([a]) != P.source_hash([d])
