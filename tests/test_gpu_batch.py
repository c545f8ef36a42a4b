"""Batched rendering on the GPU: every job's outputs match the CPU oracle's
render of the same job (tests/parity.py bar: bit-exact ids, hit distances and
radiance) and are bit-identical to the same job rendered alone with pt_render,
whether the batch is stepped with jobs joining at different times (continuous
batching), run as a static schedule, or replayed as a captured hipGraph;
admission refuses jobs beyond the slots or the arena."""
import sys

import numpy as np
import pytest

from paper_2310_07182_amd import scenes
from tests.parity import compare_render

pytestmark = pytest.mark.gpu


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


JOBS = [
    # scene, w, h, spp, bounces, mode, seed
    ("tiny", 64, 64, 1, 2, "reuse", 11),
    ("mixed_small", 96, 72, 2, 3, "reuse", 12),
    ("mixed_small", 50, 37, 1, 4, "incoherent", 13),
    ("furnace", 16, 16, 3, 3, "reuse", 14),
    ("tiny", 33, 71, 2, 1, "incoherent", 15),
    ("mixed_small", 128, 64, 1, 0, "reuse", 16),
]
TILE, K = (8, 8), 8


def _alone(torch, api, sc, spec):
    name, w, h, spp, B, mode, seed = spec
    r = api.render(sc[name], w, h, spp, B, mode, TILE, K, None, seed)
    torch.cuda.synchronize()
    return {k: v.clone() for k, v in r.items() if k in ("radiance", "hit_prim", "hit_t")}


def _same(torch, ref, out, tag):
    for key in ("radiance", "hit_prim", "hit_t"):
        a, b = ref[key], getattr(out, key)
        assert torch.equal(a.view(torch.int32), b.view(torch.int32)), (tag, key)


_orc_cache = {}


def _matches_oracle(osc, out, spec):
    """The batched job against the oracle's render of the same job."""
    name, w, h, spp, B, mode, seed = spec
    if spec not in _orc_cache:
        _orc_cache[spec] = osc[name].render(w, h, spp, B, mode=mode, tile=TILE, k=K, seed=seed)
    g = dict(radiance=out.radiance, hit_prim=out.hit_prim, hit_t=out.hit_t)
    return compare_render(g, _orc_cache[spec], TILE, mode, check_rays=False)


def _new_batch(api, max_jobs, specs, sc, extra=0, traversal=0):
    b = api.Batch(max_jobs, 1, tile=TILE, k=K)
    need = api.Batch.base_bytes(max_jobs)
    outs = []
    for spec in specs:
        name, w, h, spp, B, mode, seed = spec
        o = api.JobOutputs(w, h, spp, B, b.device)
        need += b.job_bytes(b.job_struct(sc[name], w, h, spp, B, mode, seed, o))
        outs.append(o)
    del b
    return api.Batch(max_jobs, need + extra, tile=TILE, k=K, traversal=traversal), outs


def test_batch_stepped_with_staggered_arrivals_equals_alone(env):
    torch, api, sc, osc = env
    refs = [_alone(torch, api, sc, spec) for spec in JOBS]
    b, outs = _new_batch(api, 4, JOBS, sc)
    pending = list(range(len(JOBS)))
    live = {}
    steps = 0
    while pending or live:
        # admit one new job every other step while slots and arena allow
        if pending and steps % 2 == 0:
            i = pending[0]
            name, w, h, spp, B, mode, seed = JOBS[i]
            jid = b.submit(b.job_struct(sc[name], w, h, spp, B, mode, seed, outs[i]))
            if jid is not None:
                live[jid] = i
                pending.pop(0)
        active = b.step()
        steps += 1
        torch.cuda.synchronize()
        for jid in list(live):
            if b.done(jid):
                b.release(jid)
                del live[jid]
        assert active <= 4
        assert steps < 500
    _say(f"[gpu] stepped batch: {steps} steps")
    for i, spec in enumerate(JOBS):
        _same(torch, refs[i], outs[i], spec)
        _say("  ", spec, _matches_oracle(osc, outs[i], spec))


@pytest.mark.parametrize("use_graph,traversal", [(False, "auto"), (True, "auto"), (False, "pair"), (True, "wide"),
                                                (False, "queue")])
def test_batch_static_run_equals_alone(env, use_graph, traversal):
    torch, api, sc, osc = env
    refs = [_alone(torch, api, sc, spec) for spec in JOBS]
    b, outs = _new_batch(api, len(JOBS), JOBS, sc, extra=1 << 20, traversal=traversal)
    for i, (name, w, h, spp, B, mode, seed) in enumerate(JOBS):
        assert b.submit(b.job_struct(sc[name], w, h, spp, B, mode, seed, outs[i])) is not None
    for rep in range(3):
        for o in outs:
            o.radiance.fill_(-7.0)
            o.hit_prim.fill_(-7)
            o.hit_t.fill_(-7.0)
        _say(f"[gpu] static batch run graph={use_graph} traversal={traversal} rep={rep}")
        b.run(use_graph=use_graph)
        torch.cuda.synchronize()
        for i, spec in enumerate(JOBS):
            _same(torch, refs[i], outs[i], (spec, rep))
            _matches_oracle(osc, outs[i], spec)


def test_batch_admission_limits(env):
    torch, api, sc, osc = env
    spec = ("tiny", 64, 64, 1, 2, "reuse", 1)
    b, outs = _new_batch(api, 2, [spec, spec], sc)
    name, w, h, spp, B, mode, seed = spec
    ids = [b.submit(b.job_struct(sc[name], w, h, spp, B, mode, seed, outs[i])) for i in range(2)]
    assert None not in ids
    extra = api.JobOutputs(w, h, spp, B, b.device)
    assert b.submit(b.job_struct(sc[name], w, h, spp, B, mode, seed, extra)) is None     # no slot
    from paper_2310_07182_amd import capi
    with pytest.raises(capi.PtError):
        b.release(ids[0])                                                             # not finished
    while b.step():
        pass
    torch.cuda.synchronize()
    assert b.done(ids[0]) and b.done(ids[1])
    b.release(ids[0])
    big = ("tiny", 1024, 1024, 1, 2, "reuse", 1)
    bo = api.JobOutputs(1024, 1024, 1, 2, b.device)
    assert b.submit(b.job_struct(sc["tiny"], 1024, 1024, 1, 2, "reuse", 1, bo)) is None  # arena full
    with pytest.raises(capi.PtError):
        b.submit(b.job_struct(sc["tiny"], 64, 64, 1, 2, "sorted", 1, outs[0]))         # unsupported mode
