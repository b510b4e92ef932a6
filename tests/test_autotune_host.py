"""Host logic of the batch autotuner (paper_2606_02887_amd/autotune.py): rank classes,
cache keys and the JSON cache.  No GPU."""
import json

from paper_2606_02887_amd import autotune as AT


def test_rank_classes_follow_the_rank_padding():
    assert [AT.rank_class(r) for r in (1, 4, 5, 8, 9, 16, 17, 32, 33, 64)] == \
        [0, 0, 0, 0, 1, 1, 2, 2, 3, 3]


def test_workload_key_is_coarse_and_order_free():
    ns, rs = [500, 1200, 3000, 4800], [8, 16, 8, 32]
    k1 = AT.workload_key(ns, rs, 8, 1, "csr", "dev")
    k2 = AT.workload_key(ns[::-1], rs[::-1], 8, 1, "csr", "dev")
    assert k1 == k2
    # a few rows more or less land in the same power-of-two buckets
    assert AT.workload_key([510, 1190, 3010, 4790], rs, 8, 1, "csr", "dev") == k1
    assert AT.workload_key(ns, rs, 8, 0, "csr", "dev") != k1          # precision
    assert AT.workload_key(ns, rs, 4, 1, "csr", "dev") != k1          # restarts
    assert AT.workload_key(ns, rs, 8, 1, "dense", "dev") != k1        # format
    assert AT.workload_key([n * 8 for n in ns], rs, 8, 1, "csr", "dev") != k1
    assert k1.count("|q") == 3                                        # classes 0, 1, 2


def test_cache_round_trip_and_validation(tmp_path):
    path = str(tmp_path / "sub" / "tuning.json")
    assert AT.load_cache(path) == {}
    cfg = {"tiles_per_wg": [2, 4, 8, 4], "spmm_rows_per_wg": 32}
    AT.save_cache(path, {"k": cfg})
    assert AT.load_cache(path) == {"k": cfg}
    assert AT._valid(cfg)
    assert not AT._valid({"tiles_per_wg": [0, 4, 4, 4], "spmm_rows_per_wg": 16})
    assert not AT._valid({"tiles_per_wg": [4, 4, 4], "spmm_rows_per_wg": 16})
    assert not AT._valid({"tiles_per_wg": [4, 4, 4, 4]})
    with open(path, "w") as f:
        f.write("{not json")
    assert AT.load_cache(path) == {}
    json.dumps(AT.DEFAULT)
