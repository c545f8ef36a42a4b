"""Host logic of the benchmark: which traversal kernel runs for a scene and the per-node
costs its roofline counts, the tuner's default point lying inside its search space, and
the image-quality measures of the quality study (PSNR, tile variance ratio)."""
import numpy as np

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


def test_psnr_closed_form():
    ref = np.full((4, 6, 3), 0.5)
    img = ref + 0.1                                  # every difference 0.1: MSE 0.01, 20 dB
    assert abs(bench.psnr_db(img, ref) - 20.0) < 1e-9
    img = ref.copy()
    img[0, 0, 0] += 0.3                              # one value off: MSE 0.09 / 72
    assert abs(bench.psnr_db(img, ref) - 10.0 * np.log10(72 / 0.09)) < 1e-9
    assert bench.psnr_db(ref, ref) == float("inf")


def test_tile_variance_ratio_closed_forms():
    rng = np.random.default_rng(3)
    W, H, K = 8, 8, 32
    h, w = 8 * 40, 8 * 60
    # independent pixel errors: ratio 1 (within its sampling error over 2400 tiles)
    iid = rng.normal(size=(h, w))
    assert abs(bench.tile_variance_ratio(iid, (W, H)) - 1.0) < 0.1
    # one error shared by each group of K pixels of a tile (interleaved: every (WH/K)-th
    # slot), groups independent: ratio K
    slots = np.arange(W * H).reshape(H, W)
    grp = np.tile(slots % (W * H // K), (h // H, w // W))
    tile_id = (np.arange(h)[:, None] // H) * (w // W) + (np.arange(w)[None, :] // W)
    g = rng.normal(size=(tile_id.max() + 1, W * H // K))
    shared = g[tile_id, grp]
    assert abs(bench.tile_variance_ratio(shared, (W, H)) / K - 1.0) < 0.1
    # an error constant over whole tiles: ratio W*H; channels are averaged first
    const = np.repeat(np.repeat(rng.normal(size=(h // H, w // W)), H, axis=0), W, axis=1)
    assert abs(bench.tile_variance_ratio(np.stack([const] * 3, axis=2), (W, H)) - W * H) < 1e-6
    # partial tiles at the image edge are left out
    assert abs(bench.tile_variance_ratio(const[:, : w - 3], (W, H)) - W * H) < 1e-6
