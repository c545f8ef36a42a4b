"""Autotuner for the launch parameters of the path tracer.

Tuned, by measuring on the device:
  * the reuse group: tile (W, H) and group size K, limited to K <= W*H/8 -- larger
    groups trace faster (fewer distinct directions per tile, the trend of the paper's
    tile/K table) but leave visible structured noise (the paper reports it for K = 32
    on 8x8 tiles), so the bound keeps one distinct direction per eight pixels at least;
  * waves per CU of the persistent traversal grid;
  * the refill threshold of the traversal: the number of idle lanes at which a wave
    takes new rays from the ray queue (the queue tile one refill fetches);
  * the leaf gate: how few lanes may still be looking for a leaf when a wave stops
    walking inner nodes and tests the leaves its lanes hold.

The search is coordinate descent: one parameter at a time, over its candidate list,
keeping the best value before moving to the next.  The objective is the measured
time of the caller's unit of work (a frame, or a whole batch).
"""
from __future__ import annotations

GROUPS = (((4, 4), 2), ((8, 8), 2), ((8, 8), 4), ((8, 8), 8), ((16, 8), 16), ((16, 16), 32))
WAVES_PER_CU = (16, 20, 24)
REFILLS = (8, 12, 16, 24, 32, 48)
LEAF_GATES = (4, 6, 8, 12, 16)
MAX_GROUP_FRACTION = 8      # K <= W*H / 8


def group_allowed(tile, k, fraction=MAX_GROUP_FRACTION) -> bool:
    w, h = tile
    return k >= 1 and (w * h) % k == 0 and k * fraction <= w * h


def coordinate_descent(evaluate, dims, start):
    """evaluate(params) -> cost (lower is better); dims: [(name, candidates)];
    start: the initial parameters.  Returns (best, best_cost, log of (params, cost))."""
    def key(p):
        return tuple(sorted((k, repr(v)) for k, v in p.items()))

    best = dict(start)
    best_cost = evaluate(dict(best))
    log = [(dict(best), best_cost)]
    seen = {key(best)}
    for name, values in dims:
        for v in values:
            cand = dict(best)
            cand[name] = v
            if key(cand) in seen:
                continue
            seen.add(key(cand))
            c = evaluate(dict(cand))
            log.append((cand, c))
            if c < best_cost:
                best, best_cost = cand, c
    return best, best_cost, log


def search_space(mode, groups=GROUPS, waves=WAVES_PER_CU, refills=REFILLS, leaf_gates=LEAF_GATES):
    dims = []
    if mode == "reuse":
        dims.append(("group", tuple(g for g in groups if group_allowed(*g))))
    dims.append(("waves_per_cu", tuple(waves)))
    dims.append(("refill", tuple(refills)))
    dims.append(("leaf_gate", tuple(leaf_gates)))
    return dims


DEFAULT = dict(group=((8, 8), 8), waves_per_cu=24, refill=16, leaf_gate=8)


def _median_ms(run, reps):
    import torch
    st = torch.cuda.current_stream()
    times = []
    for _ in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(st)
        run()
        b.record(st)
        torch.cuda.synchronize()
        times.append(a.elapsed_time(b))
    times.sort()
    return times[len(times) // 2]


def tune_render(scene, w, h, spp, bounces, mode, reps=3, seed=1, **space):
    """Best parameters for repeated frames of one configuration (pt_render)."""
    from . import api

    def evaluate(p):
        (tile, k) = p["group"]
        cfg = api.RenderConfig(w, h, spp, bounces, mode, tile, k, None, p["refill"], p["waves_per_cu"],
                               p["leaf_gate"])
        r = api.Renderer(scene, cfg)
        r.render(seed)                                   # warm-up
        return _median_ms(lambda: r.render(seed), reps)

    return coordinate_descent(evaluate, search_space(mode, **space), DEFAULT)


def tune_batch(scenes, requests, arena_bytes, max_jobs=None, reps=2, **space):
    """Best parameters for a static batch of requests (pt_batch_run as a captured graph)."""
    from . import api
    mode = requests[0].mode
    max_jobs = max_jobs or len(requests)
    outs = [api.JobOutputs(r.w, r.h, r.spp, r.bounces, "cuda:0") for r in requests]

    def evaluate(p):
        (tile, k) = p["group"]
        b = api.Batch(max_jobs, arena_bytes, tile=tile, k=k, refill=p["refill"], waves_per_cu=p["waves_per_cu"],
                      leaf_gate=p["leaf_gate"])
        for r, o in zip(requests, outs):
            if b.submit(b.job_struct(scenes[r.scene], r.w, r.h, r.spp, r.bounces, r.mode, r.seed, o)) is None:
                raise RuntimeError("batch arena too small for the tuning set")
        b.run(use_graph=True)                            # capture + first replay
        ms = _median_ms(lambda: b.run(use_graph=True), reps)
        del b
        return ms

    return coordinate_descent(evaluate, search_space(mode, **space), DEFAULT)
