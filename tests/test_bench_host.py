"""Host logic of the benchmark: which traversal kernel runs for a scene and the per-node
costs its roofline counts, and the tuner's default point lying inside its search space."""
import bench
from paper_2310_07182_amd import autotune


class _Scene:
    def __init__(self, wide, quant, ntri):
        self._i = dict(wide=wide, quant=quant, ntri=ntri)

    def info(self):
        return self._i


def test_traversal_kind_follows_the_library_choice():
    assert bench.traversal_kind(_Scene(1, 1, 1000)) == "quant"
    assert bench.traversal_kind(_Scene(1, 0, 1000)) == "queue"
    assert bench.traversal_kind(_Scene(1, 1, (1 << 26) + 1)) == "wide"
    assert bench.traversal_kind(_Scene(0, 1, 1000)) == "pair"
    assert bench.traversal_kind(_Scene(1, 1, 1000), "pair") == "pair"


def test_node_costs_per_kind():
    assert bench.node_costs(_Scene(1, 1, 10)) == (bench.NODE4Q_BYTES, bench.OPS_PER_NODE4Q) == (64, 137)
    assert bench.node_costs(_Scene(1, 0, 10)) == (bench.NODE4_BYTES, bench.OPS_PER_NODE4) == (128, 137)
    assert bench.node_costs(_Scene(0, 0, 10)) == (bench.NODE_BYTES, bench.OPS_PER_NODE) == (64, 58)
    for kind in ("pair", "wide", "queue", "quant"):
        assert bench.kernel_label(_Scene(1, 1, 10), kind)


def test_tuner_default_inside_search_space():
    d = autotune.DEFAULT
    assert d["refill"] in autotune.REFILLS
    assert d["waves_per_cu"] in autotune.WAVES_PER_CU
    assert d["leaf_gate"] in autotune.LEAF_GATES
    assert d["group"] in autotune.GROUPS
