"""Host logic of the batch autotuner (no GPU needed): the (size, skew)
buckets, the install rule and the table file."""
import numpy as np

from paper_1812_00283_amd import tune


def test_bucket_of_size_and_skew():
    assert tune.bucket_of(1, 1, 1.0) == "m4^0-flat"
    assert tune.bucket_of(4 ** 5, 10, 2.0) == "m4^5-flat"
    assert tune.bucket_of(4 ** 5 - 1, 10, 2.0) == "m4^4-flat"
    # skewed: the largest degree above 16x the mean degree
    assert tune.bucket_of(1000, 33, 2.0) == "m4^4-skewed"
    assert tune.bucket_of(1000, 32, 2.0) == "m4^4-flat"


def test_graph_buckets_per_graph():
    # graph 0: a star of 40 edges (skewed), graph 1: a perfect matching of 40 (flat), graph 2: empty
    star = np.stack([np.zeros(40, np.int32), np.arange(40, dtype=np.int32)], axis=1)
    match = np.stack([np.arange(40, dtype=np.int32), np.arange(40, dtype=np.int32)], axis=1)
    edges = np.concatenate([star, match])
    offsets = [0, 40, 80, 80]
    b = tune.graph_buckets(edges, offsets, [1, 40, 3], [40, 40, 3])
    # star: max degree 40, mean 2*40/41 < 2.5 -> skewed; matching: max 1, mean 1 -> flat
    assert b == ["m4^2-skewed", "m4^2-flat", "empty"]


class _Handle:
    def __init__(self):
        self.installed = None

    def set_graph_tuning(self, per_graph):
        self.installed = per_graph


def test_apply_table_installs_only_when_savings_outweigh_the_rebuild():
    table = {"m4^5-flat": {"tuning": {"window_mode": 3}, "est_saving_ms": 4.0},
             "m4^6-skewed": {"tuning": {}, "est_saving_ms": 0.0}}
    buckets = ["m4^5-flat", "m4^6-skewed", "empty"]
    h = _Handle()
    assert not tune.apply_table(h, table, buckets, min_saving_ms=10.0)
    assert h.installed is None
    assert tune.apply_table(h, table, buckets, min_saving_ms=3.0)
    assert h.installed == [{"window_mode": 3}, {}, {}]
    # nothing to install when every bucket keeps its defaults
    h2 = _Handle()
    assert not tune.apply_table(h2, {"m4^6-skewed": {"tuning": {}, "est_saving_ms": 50.0}}, ["m4^6-skewed"], 1.0)
    assert h2.installed is None


def test_table_file_round_trip(tmp_path):
    table = {"m4^5-flat": {"tuning": {"hash_window_wedges": 32768}, "graphs": 13, "est_saving_ms": 0.25}}
    p = tmp_path / "t.json"
    tune.save(table, str(p))
    assert tune.load_table(str(p)) == table
