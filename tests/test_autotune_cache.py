"""Host-side pieces of the autotuner: cache keys and the JSON cache (no GPU)."""
import workloads as W
from paper_2501_11962_amd import autotune as A


def test_shape_key_separates_systems():
    k1 = A.shape_key(W.cfg2(), 64)
    k2 = A.shape_key(W.cfg2(), 16)
    k3 = A.shape_key(W.cfg1(), 64)
    assert k1 != k2 and k1 != k3
    assert A.shape_key(W.cfg2(), 64) == k1  # deterministic


def test_cache_round_trip(tmp_path):
    p = str(tmp_path / "c.json")
    assert A.load_cache(p) == {}
    A.save_cache({"k": {"opts": {"col_width": 0.4, "waves": 2}, "ms": 1.0}}, p)
    assert A.load_cache(p)["k"]["opts"]["waves"] == 2
    open(p, "w").write("not json")
    assert A.load_cache(p) == {}


def test_search_space_contains_the_default():
    for k, v in A.DEFAULT.items():
        assert v in A.SPACE[k], k
