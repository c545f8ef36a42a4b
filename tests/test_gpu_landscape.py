"""GPU parity on the full-size landscape workload (63.6M triangles, 1920x1080,
1 spp, 3 bounces, tile 8x8, K=8), all three modes: sampled tiles against the
oracle, element by element; whole-image properties elsewhere."""
import sys
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

from paper_2310_07182_amd import scenes
from tests.parity import compare_render

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def land(orc):
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2310_07182_amd import api
    _say("[gpu] landscape: generating the scene")
    s = scenes.landscape()
    _say(f"[gpu] landscape: {s['tris'].shape[0]} triangles; building the library and oracle BVHs")
    with ThreadPoolExecutor(2) as ex:
        fo = ex.submit(orc.OracleScene, s)
        sc = api.Scene(s)
        _say("[gpu] landscape: library scene uploaded", sc.info())
        osc = fo.result()
    _say("[gpu] landscape: oracle scene built")
    yield api, torch, s, sc, osc
    del sc, osc


@pytest.mark.timeout(1200)
@pytest.mark.parametrize("mode", ["reuse", "incoherent", "sorted"])
def test_landscape_full_size_sampled_tiles(land, mode):
    api, torch, s, sc, osc = land
    cfg = scenes.CONFIGS["landscape"]
    w, h, B, tile, k = cfg["w"], cfg["h"], cfg["bounces"], cfg["tile"], cfg["k"]
    seed = 2310071822
    _say(f"[gpu] landscape render {w}x{h} B={B} mode={mode}")
    g = api.render(sc, w, h, 1, B, mode, tile, k, None, seed, rays=True)
    torch.cuda.synchronize()
    ntx, nty = (w + tile[0] - 1) // tile[0], (h + tile[1] - 1) // tile[1]
    rng = np.random.default_rng(321)
    pick = rng.choice(ntx * nty, (ntx * nty) // 100, replace=False)   # 1% of the tiles
    pick = np.concatenate([pick, [0, ntx - 1, ntx * nty - 1, ntx * (nty // 2) + ntx // 2]])
    mask = np.zeros(ntx * nty, np.uint8)
    mask[pick] = 1
    o = osc.render(w, h, 1, B, mode=mode, tile=tile, k=k, seed=seed, tile_mask=mask, rays=True)
    pm = np.zeros((h, w), bool)
    for t in np.where(mask)[0]:
        ty, tx = divmod(int(t), ntx)
        pm[ty * tile[1]:(ty + 1) * tile[1], tx * tile[0]:(tx + 1) * tile[0]] = True
    res = compare_render(g, o, tile, mode, pixel_mask=pm)
    _say("  ", res)
    hp = g["hit_prim"].cpu().numpy()
    assert np.array_equal(g["rays_per_bounce"].cpu().numpy(), (hp != -2).reshape(B + 1, -1).sum(1))
    # the camera sees terrain and sky: primary rays both hit and miss
    assert (hp[0] >= 0).any() and (hp[0] == -1).any()
    assert np.all(hp[0] != -2)
