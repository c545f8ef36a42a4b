"""Serving on the GPU: requests that arrive while others are in flight are
admitted and batched with them (continuous batching), and every result matches
the CPU oracle's render of the same request (tests/parity.py bar) and is bit for
bit the one the same request gives rendered alone; the same under a tight HBM
budget that makes requests queue.  The autotuner returns parameters from its
space whose frame time is not above the default's."""
import sys

import pytest

from paper_2310_07182_amd import autotune, scenes, serve
from tests.parity import compare_render

pytestmark = pytest.mark.gpu

RES = ((64, 64), (96, 72), (50, 37), (128, 64))
SPPS = (1, 2)


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def env(orc):
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2310_07182_amd import api
    src = {name: getattr(scenes, name)() for name in ("tiny", "mixed_small", "furnace")}
    sc = {name: api.Scene(s) for name, s in src.items()}
    osc = {name: orc.OracleScene(s) for name, s in src.items()}
    return torch, api, sc, osc


def _check_alone(torch, api, sc, osc, reqs, kept):
    for r in reqs:
        ref = api.render(sc[r.scene], r.w, r.h, r.spp, r.bounces, r.mode, (8, 8), 8, None, r.seed)
        torch.cuda.synchronize()
        o = kept[r.rid]
        for key in ("radiance", "hit_prim", "hit_t"):
            assert torch.equal(ref[key].view(torch.int32), getattr(o, key).view(torch.int32)), (r, key)
        orr = osc[r.scene].render(r.w, r.h, r.spp, r.bounces, mode=r.mode, tile=(8, 8), k=8, seed=r.seed)
        compare_render(dict(radiance=o.radiance, hit_prim=o.hit_prim, hit_t=o.hit_t), orr, (8, 8), r.mode,
                       check_rays=False)


@pytest.mark.parametrize("mode", ["reuse", "incoherent"])
def test_serving_mix_equals_alone(env, mode):
    torch, api, sc, osc = env
    reqs = serve.make_requests(12, 400.0, list(sc), mode, seed=21, bounces=3, resolutions=RES, spps=SPPS)
    arena = api.Batch.base_bytes(4) + 4 * max(api.batch_job_bytes(r.w, r.h, r.spp, r.bounces, mode) for r in reqs)
    be = serve.BatchBackend(sc, 4, arena, keep=[r.rid for r in reqs])
    _say(f"[gpu] serving {mode}: {len(reqs)} requests")
    st = serve.serve(reqs, be, 1 << 40)
    torch.cuda.synchronize()
    assert st.max_in_flight >= 2
    assert all(r.finished >= r.admitted >= r.arrival for r in st.records)
    _check_alone(torch, api, sc, osc, reqs, be.kept)
    s = st.summary()
    assert s["secondary_rays"] > 0


def test_serving_tight_budget_equals_alone(env):
    torch, api, sc, osc = env
    reqs = serve.make_requests(8, None, list(sc), "reuse", seed=22, bounces=2, resolutions=RES, spps=SPPS)
    be = serve.BatchBackend(sc, 8, api.Batch.base_bytes(8) + 8 * max(
        api.batch_job_bytes(r.w, r.h, r.spp, r.bounces, "reuse") for r in reqs), keep=[r.rid for r in reqs])
    budget = be.resident_bytes() + 2 * max(serve.output_bytes(r) for r in reqs)
    _say("[gpu] serving under a two-request budget")
    st = serve.serve(reqs, be, budget)
    torch.cuda.synchronize()
    assert st.refused_admissions > 0 and st.peak_budget_bytes <= budget
    _check_alone(torch, api, sc, osc, reqs, be.kept)


def test_autotune_render_returns_a_candidate(env):
    torch, api, sc, osc = env
    _say("[gpu] autotune mixed_small 320x240")
    w, h, B = 320, 240, 3
    best, cost, log = autotune.tune_render(sc["mixed_small"], w, h, 1, B, "reuse", reps=3)
    space = dict(autotune.search_space("reuse"))
    assert best["group"] in space["group"] and best["waves_per_cu"] in space["waves_per_cu"]
    assert best["refill"] in space["refill"] and cost > 0
    assert len(log) == 1 + sum(len(v) - 1 for v in space.values())

    # on a repeat, the tuned choice is not slower than the default (10% allowance for noise)
    def frame_ms(p):
        (tile, k) = p["group"]
        cfg = api.RenderConfig(w, h, 1, B, "reuse", tile, k, None, p["refill"], p["waves_per_cu"], p["leaf_gate"])
        r = api.Renderer(sc["mixed_small"], cfg)
        r.render(1)
        return autotune._median_ms(lambda: r.render(1), 9)

    d, t = frame_ms(autotune.DEFAULT), frame_ms(best)
    _say(f"   default {d:.3f} ms, tuned {t:.3f} ms ({best})")
    assert t <= 1.10 * d, (t, d, best)
