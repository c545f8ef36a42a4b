"""Benchmark: secondary-ray trace speed of the reuse path tracer on one MI355X.

One step = one frame of the whole hot path (primary rays, then B bounces of
trace -> shade -> next direction) over the indoor workload (1920x1080, 1 spp,
4 bounces, ~1M triangles, tile 8x8 / K = 8), inputs resident in HBM.

Headline (value): secondary Mrays/s in reuse mode = rays traced at bounces
1..B / summed traversal-kernel time of those bounces (HIP events on the
library's stream), the definition of the paper's Table 1.  The same figure for
the incoherent and sorted modes, end-to-end rates and p50/p99 frame latency
are reported beside it.  The roofline object describes the traversal kernel:
algorithmic operations and bytes per launch (nodes visited x 64 B of the quantized
four-wide nodes, 128 B of the float four-wide nodes, 64 B of child-pair nodes, + triangles tested x 48 B + 32 B ray + 8 B hit, per ray, counted by the
counting variant of the kernel in an untimed frame) divided by its average launch
time.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# algorithmic bytes per unit of traversal work: a node as the kernel reads it, a triangle as
# 36 bytes of vertices + its 4-byte id (the kernel's float4 layout reads 48), the ray and the hit
NODE_BYTES, TRI_BYTES, RAY_BYTES, HIT_BYTES = 64, 40, 32, 8
# 32-bit VALU lane operations per unit of traversal work (counted from the kernel source):
# a node visit = two slab tests (6 sub, 6 mul, 10 min/max, 1 mul, 2 cmp, 1 and = 26 each)
# plus the near/far choice (~6); a triangle test = 9 sub, 12 mul, 9 sub of the shear and
# edge functions, 6 sign tests, 2 add, 3 mul + 2 add for T, the division (~10),
# 3 compares and 18 component selects.
OPS_PER_NODE, OPS_PER_TRI = 58, 74
# a four-wide node visit: four slab tests (4 x 26), the five compare-exchanges of the sorting
# network on (distance, code) (5 x 5) and ~8 for the pushes and the choice of the next node
OPS_PER_NODE4, NODE4_BYTES = 137, 128
# a quantized four-wide node visit: per node a = step / d (3 mul), b = (p - o) / d (3 sub,
# 3 mul), b moved outward for near and far planes (6 fused multiply-adds) and the choice of
# near/far plane bytes by the ray's signs (3 cmp, 6 select) = 24; per child 6 byte
# conversions, 6 fused multiply-adds, 3 max, 2 min, 1 mul, the cull min and 1 cmp = 20; then
# the sorting network (25) and the pushes (8).  Bytes read: the whole 64-byte node.
OPS_PER_NODE4Q, NODE4Q_BYTES = 137, 64
# MI355X vector ALU: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz, one 32-bit op per lane and cycle
# (no packed FP32, an FMA counted once) = 39.3 T ops/s.
VALU_PEAK_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12


PROFILE_SUMMARY = os.path.join(ROOT, "profiles", "k_trace_{config}_1080p.md")
# sources whose change makes the committed counter summaries stale (the kernels, the host code
# that launches them, the build flags and the BVH builder, which sets the work per ray)
KERNEL_SOURCES = ("paper_2310_07182_amd/csrc/kernels.hip", "paper_2310_07182_amd/csrc/kernels.h",
                  "paper_2310_07182_amd/csrc/capi.hip", "paper_2310_07182_amd/build.py",
                  "paper_2310_07182_amd/csrc/bvh_build.cpp")


def measured_traffic(mode, config):
    """Bytes per secondary traversal launch from the committed rocprofv3 FETCH_SIZE/WRITE_SIZE
    summary, or None when it covers another workload or the kernel sources changed since."""
    import hashlib
    path = PROFILE_SUMMARY.format(config=config)
    if not os.path.exists(path):
        return None
    digest = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(os.path.join(ROOT, p), "rb") as f:
            digest.update(f.read())
    with open(path) as f:
        for line in f:
            if line.startswith("traffic_bytes_per_launch "):
                fields = dict(kv.split("=", 1) for kv in line.split()[1:])
                if fields.get("source_sha256") != digest.hexdigest() or mode not in fields:
                    return None
                return float(fields[mode])
    return None


def traversal_kind(sc, trav="auto"):
    """The traversal kernel that runs: the one asked for, else the one the library picks."""
    if trav != "auto":
        return trav
    inf = sc if isinstance(sc, dict) else sc.info()
    if inf["wide"] and inf["ntri"] <= (1 << 26):
        return "quant" if inf["quant"] else "queue"
    return "wide" if inf["wide"] else "pair"


def kernel_label(sc, trav="auto"):
    return {"quant": "k_trace_q (closest hit over quantized four-wide nodes, per-wave triangle-test queue)",
            "queue": "k_trace_q (closest hit over four-wide nodes, per-wave triangle-test queue)",
            "wide": "k_trace (closest hit over four-wide nodes)",
            "pair": "k_trace (closest hit over child-pair nodes)"}[traversal_kind(sc, trav)]


def node_costs(sc, trav="auto"):
    """(bytes, ops) of one node visit of the traversal kernel that runs."""
    k = traversal_kind(sc, trav)
    if k == "quant":
        return NODE4Q_BYTES, OPS_PER_NODE4Q
    if k in ("queue", "wide"):
        return NODE4_BYTES, OPS_PER_NODE4
    return NODE_BYTES, OPS_PER_NODE


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def bench_mode(api, sc, cfg, mode, steps, warmup, seed0, nee=False, trav="auto", tile=None, k=None,
               frame_groups=False, reuse_max_bounce=None, latency_frames=0):
    """Timed frames of one mode: W untimed frames, then exactly `steps` timed frames (the
    value), then `latency_frames` more for the frame-latency percentiles."""
    import torch
    node_bytes, ops_node = node_costs(sc, trav)
    tile = tuple(cfg["tile"]) if tile is None else tuple(tile)
    k = cfg["k"] if k is None else k
    rc = api.RenderConfig(cfg["w"], cfg["h"], 1, cfg["bounces"], mode, tile, k, nee=nee, traversal=trav,
                          frame_groups=frame_groups, reuse_max_bounce=reuse_max_bounce)
    # untimed counting frame: nodes / triangles per ray and rays per bounce
    rs = api.Renderer(sc, rc, stats=True, touched=True)
    rs.render(seed0)
    torch.cuda.synchronize()
    stats = rs.stats.cpu().numpy().astype(np.float64)
    rays_stats = rs.ray_count.cpu().numpy().reshape(-1).astype(np.float64)
    # compulsory bytes per bounce: the distinct nodes and triangles the bounce touched, plus
    # each ray read and hit written once (a lower bound on the launch's memory traffic)
    tn, tt = rs.touched_counts()
    compulsory = [float(tn[b] * node_bytes + tt[b] * TRI_BYTES + rays_stats[b] * (RAY_BYTES + HIT_BYTES))
                  for b in range(len(tn))]
    del rs
    timer = api.Timer(capacity=64 * (steps + warmup + 2))
    r = api.Renderer(sc, rc, timer=timer)
    for i in range(warmup):
        r.render(seed0 + 1 + i)
    torch.cuda.synchronize()
    timer.reset()
    st = torch.cuda.current_stream()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    rays = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(steps):
        ev[i][0].record(st)
        r.render(seed0 + 1000 + i)
        ev[i][1].record(st)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    frame_ms = np.array([a.elapsed_time(b) for a, b in ev])
    ms, kind, bounce = timer.read()
    # more frames, after the timed region, for the latency percentiles only
    lat_ms = list(frame_ms)
    if latency_frames > 0:
        r2 = api.Renderer(sc, rc)
        evl = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
               for _ in range(latency_frames)]
        for i in range(latency_frames):
            evl[i][0].record(st)
            r2.render(seed0 + 50000 + i)
            evl[i][1].record(st)
        torch.cuda.synchronize()
        # percentiles over these frames alone: the timed frames carry the timer's events
        lat_ms = [a.elapsed_time(b) for a, b in evl]
        del r2
    lat_ms = np.array(lat_ms)
    # rays of the last frame (identical statistics every frame; counted on the device)
    rays = r.ray_count.cpu().numpy().reshape(-1).astype(np.float64)
    B = cfg["bounces"]
    trace = kind == 0
    sec = trace & (bounce >= 1)
    per_frame_sec_ms = ms[sec].sum() / steps
    per_frame_trace_ms = ms[trace].sum() / steps
    sec_rays = rays[1:].sum()
    mrays = sec_rays / (per_frame_sec_ms * 1e-3) / 1e6
    e2e = sec_rays / (frame_ms.mean() * 1e-3) / 1e6
    # algorithmic bytes of the traversal kernel (secondary bounces)
    nodes_per_ray = stats[1:, 0].sum() / max(rays_stats[1:].sum(), 1)
    tris_per_ray = stats[1:, 1].sum() / max(rays_stats[1:].sum(), 1)
    bytes_per_ray = nodes_per_ray * node_bytes + tris_per_ray * TRI_BYTES + RAY_BYTES + HIT_BYTES
    launches = int(sec.sum())
    avg_launch_ms = ms[sec].mean()
    bytes_per_launch = bytes_per_ray * sec_rays / B
    ops_per_ray = nodes_per_ray * ops_node + tris_per_ray * OPS_PER_TRI
    ops_per_launch = ops_per_ray * sec_rays / B
    kinds = {int(kk): float(ms[kind == kk].sum() / steps) for kk in np.unique(kind)}
    # per bounce: mean traversal and shade launch time; per frame: the secondary trace rate
    trace_us = [float(ms[trace & (bounce == bb)].mean() * 1e3) for bb in range(B + 1)]
    shade_us = [float(ms[(kind == 2) & (bounce == bb)].mean() * 1e3) for bb in range(B + 1)]
    per_frame_sec = ms[sec].reshape(steps, -1).sum(axis=1)
    frame_rates = sec_rays / (per_frame_sec * 1e-3) / 1e6
    shadow = {}
    if nee:
        srays = r.shadow_count.cpu().numpy().astype(np.float64).sum()
        sms = ms[kind == 7].sum() / steps
        shadow = dict(shadow_rays_per_frame=int(srays), shadow_trace_ms_per_frame=float(sms),
                      shadow_mrays_s=float(srays / (sms * 1e-3) / 1e6) if sms > 0 else 0.0)
    return dict(mode=mode, tile=list(tile), k=k, frame_groups=bool(frame_groups), reuse_max_bounce=reuse_max_bounce,
                secondary_mrays_s=mrays, end_to_end_secondary_mrays_s=e2e,
                secondary_mrays_s_frame_sd=float(frame_rates.std()),
                trace_us_per_bounce=trace_us, shade_us_per_bounce=shade_us,
                frame_ms_mean=float(frame_ms.mean()), frame_ms_p50=float(np.percentile(lat_ms, 50)),
                frame_ms_p99=float(np.percentile(lat_ms, 99)), latency_frames=int(len(lat_ms)), wall_s=wall,
                trace_ms_per_frame=float(per_frame_trace_ms), secondary_trace_ms_per_frame=float(per_frame_sec_ms),
                rays_per_bounce=[int(v) for v in rays], nodes_per_ray=float(nodes_per_ray),
                tris_per_ray=float(tris_per_ray), bytes_per_ray=float(bytes_per_ray),
                avg_trace_launch_ms=float(avg_launch_ms), trace_launches=launches,
                bytes_per_launch=float(bytes_per_launch), ops_per_ray=float(ops_per_ray),
                compulsory_bytes_per_bounce=compulsory,
                compulsory_bytes_per_launch=float(np.mean(compulsory[1:])) if len(compulsory) > 1 else 0.0,
                ops_per_launch=float(ops_per_launch), ms_by_kind=kinds, **shadow)


def cpu_baseline(scene, cfg, name, budget_s=15.0, seed=2310071821):
    """The oracle, single-threaded, on a bounded sample of the same frame: a
    band of reuse tiles (reuse mode), timed on this host."""
    import oracle
    t0 = time.perf_counter()
    osc = oracle.OracleScene(scene)
    build_s = time.perf_counter() - t0
    w, h, B, tile, k = cfg["w"], cfg["h"], cfg["bounces"], tuple(cfg["tile"]), cfg["k"]
    ntx, nty = (w + tile[0] - 1) // tile[0], (h + tile[1] - 1) // tile[1]
    rng = np.random.default_rng(7)
    order = rng.permutation(ntx * nty)
    # calibrate: grow the sample until it takes a tenth of the budget, then size it
    mask = np.zeros(ntx * nty, np.uint8)
    n = 64
    while True:
        mask[:] = 0
        mask[order[:n]] = 1
        t0 = time.perf_counter()
        osc.render(w, h, 1, B, mode="reuse", tile=tile, k=k, seed=seed, tile_mask=mask)
        dt = time.perf_counter() - t0
        if dt >= 0.1 * budget_s or n >= ntx * nty:
            break
        n = min(ntx * nty, n * 4)
    n = int(min(ntx * nty, max(64, n * budget_s / max(dt, 1e-6))))
    mask[:] = 0
    mask[order[:n]] = 1
    t0 = time.perf_counter()
    r = osc.render(w, h, 1, B, mode="reuse", tile=tile, k=k, seed=seed, tile_mask=mask)
    dt = time.perf_counter() - t0
    sec = float(r["rays_per_bounce"][1:].sum())
    return dict(value=sec / dt / 1e6, unit="secondary Mrays/s", cores=1, kind="oracle",
                sample=f"{n} of {ntx * nty} {tile[0]}x{tile[1]} reuse tiles of the {w}x{h} {name} frame "
                       f"(B={B}), single thread, {dt:.1f} s; BVH build {build_s:.1f} s excluded",
                seconds=dt, tiles_per_s=n / dt)


def cpu_worker(args):
    """Child process of the all-cores baseline: the oracle renders tile band `--cpu-part`
    of `--cpu-parts` (tiles t with t mod parts == part) `--cpu-reps` times from the agreed
    start time and prints its timing.  Never touches the GPU."""
    import oracle
    from paper_2310_07182_amd import scenes
    cfg = scenes.CONFIGS[args.config]
    osc = oracle.OracleScene(cfg["scene"]())
    w, h, B, tile, k = cfg["w"], cfg["h"], cfg["bounces"], tuple(cfg["tile"]), cfg["k"]
    ntx, nty = (w + tile[0] - 1) // tile[0], (h + tile[1] - 1) // tile[1]
    mask = (np.arange(ntx * nty) % args.cpu_parts == args.cpu_part).astype(np.uint8)
    while time.time() < args.cpu_start:
        time.sleep(0.005)
    t0 = time.time()
    rays = 0
    for rep in range(args.cpu_reps):
        r = osc.render(w, h, 1, B, mode="reuse", tile=tile, k=k, seed=2310071900 + rep, tile_mask=mask)
        rays += int(r["rays_per_bounce"][1:].sum())
    print(json.dumps(dict(t0=t0, t1=time.time(), rays=rays, tiles=int(mask.sum()) * args.cpu_reps)), flush=True)


def cpu_baseline_all_cores(cfg, name, single, budget_s=10.0):
    """The same oracle as independent processes, one per host core, over interleaved tile
    bands of the frame (no reuse group spans two processes); value = all secondary rays
    traced / wall time from the first start to the last finish."""
    import subprocess
    cores = len(os.sched_getaffinity(0))
    w, h, tile = cfg["w"], cfg["h"], tuple(cfg["tile"])
    ntiles = ((w + tile[0] - 1) // tile[0]) * ((h + tile[1] - 1) // tile[1])
    band = ntiles / cores
    reps = max(1, int(round(budget_s * single["tiles_per_s"] / band)))
    start = time.time() + 20.0                         # scene generation and BVH build first
    procs = [subprocess.Popen([sys.executable, os.path.abspath(__file__), "--cpu-worker", "--config", name,
                               "--cpu-part", str(i), "--cpu-parts", str(cores), "--cpu-reps", str(reps),
                               "--cpu-start", repr(start)], stdout=subprocess.PIPE, text=True)
             for i in range(cores)]
    res = []
    for p in procs:
        out, _ = p.communicate()
        if p.returncode != 0:
            raise RuntimeError(f"oracle worker failed with {p.returncode}")
        res.append(json.loads(out.strip().splitlines()[-1]))
    t0, t1 = min(r["t0"] for r in res), max(r["t1"] for r in res)
    rays = sum(r["rays"] for r in res)
    late = max(r["t0"] for r in res) - start
    return dict(value=rays / (t1 - t0) / 1e6, unit="secondary Mrays/s", cores=cores, kind="oracle",
                sample=f"{cores} oracle processes, one per host core, each rendering an interleaved band of "
                       f"{int(band)} of the {ntiles} {tile[0]}x{tile[1]} reuse tiles of the {w}x{h} {name} frame "
                       f"{reps} times (different seeds); {t1 - t0:.1f} s wall from first start to last finish "
                       f"(latest start {late:+.1f} s after the agreed time); BVH builds excluded",
                single_core_value=single["value"], single_core_sample=single["sample"])


MIX_SCENES = ("tiny", "indoor", "landscape", "mid")
MALL_BYTES = 256 << 20          # MI355X Infinity Cache


def measure_ceilings(api):
    """Read bandwidth and dependent-load latency of the level holding a 4 GiB (HBM),
    128 MiB (MALL) and 2 MiB (L2 of each XCD) buffer, with the library's probe kernels."""
    import torch
    buf = torch.empty(4 << 30, dtype=torch.uint8, device="cuda:0")
    out = {}
    for level, nbytes, passes, steps in (("hbm", 4 << 30, 3, 20000), ("mall", 128 << 20, 60, 50000),
                                         ("l2", 2 << 20, 4000, 100000)):
        r = api.probe_memory(nbytes, passes, steps, buf)
        out[level] = {"bytes": nbytes, "read_GBps": round(r["read_gbps"], 1), "dependent_load_ns": round(r["chase_ns"], 1)}
    del buf
    torch.cuda.empty_cache()
    return out


def load_scenes(api, scenes, names):
    out = {}
    for n in names:
        t0 = time.perf_counter()
        sd = getattr(scenes, n)()
        t1 = time.perf_counter()
        out[n] = api.Scene(sd, device="cuda:0")
        log(f"[bench] scene {n}: {sd['tris'].shape[0]} triangles, generated {t1 - t0:.1f} s, "
            f"BVH + upload {time.perf_counter() - t1:.1f} s, {out[n].arena.numel() / 1e9:.2f} GB on the device")
    return out


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
    return float(np.median(times)), [round(t, 3) for t in times]


def bench_batched(api, serve, autotune, scs, args, tune=True):
    """Batched workload: 64 jobs over the resident scenes, mixed resolution and spp,
    4 bounces; per-job pt_render calls vs one batch (merged launches, captured graph)
    with the default and (tune) the autotuned launch parameters."""
    import torch
    out = {}
    for mode in args.modes.split(","):
        if mode == "sorted":
            continue                                   # batches trace reuse and incoherent jobs
        reqs = serve.make_requests(args.jobs, None, list(scs), mode, seed=2310071823)
        rend = [api.Renderer(scs[r.scene], api.RenderConfig(r.w, r.h, r.spp, r.bounces, mode, (8, 8), 8))
                for r in reqs]

        def per_job():
            for rr, r in zip(rend, reqs):
                rr.render(r.seed)
        per_job()
        torch.cuda.synchronize()
        per_ms, per_all = _median_ms(per_job, args.reps)
        rays = int(sum(int((rr.hit_prim[1:] != -2).sum()) for rr in rend))
        del rend
        torch.cuda.empty_cache()
        need = api.Batch.base_bytes(len(reqs)) + sum(
            api.batch_job_bytes(r.w, r.h, r.spp, r.bounces, mode, (16, 16), 32) for r in reqs)
        need = int(need * 1.05) + (64 << 20)           # room for any tuned group's super tiles

        def batch_ms(p, graph=True):
            (tile, k) = p["group"]
            b = api.Batch(len(reqs), need, tile=tile, k=k, refill=p["refill"], waves_per_cu=p["waves_per_cu"],
                          leaf_gate=p["leaf_gate"])
            outs = [api.JobOutputs(r.w, r.h, r.spp, r.bounces, "cuda:0") for r in reqs]
            for r, o in zip(reqs, outs):
                assert b.submit(b.job_struct(scs[r.scene], r.w, r.h, r.spp, r.bounces, mode, r.seed, o)) is not None
            b.run(use_graph=graph)
            torch.cuda.synchronize()
            res = _median_ms(lambda: b.run(use_graph=graph), args.reps)
            del b, outs
            return res

        default = dict(autotune.DEFAULT)
        d_ms, d_all = batch_ms(default)
        e_ms, _ = batch_ms(default, graph=False)
        if not tune:
            out[mode] = dict(jobs=len(reqs), secondary_rays=rays,
                             per_job_ms=round(per_ms, 3), per_job_mrays_s=round(rays / per_ms / 1e3, 1),
                             batch_graph_ms=round(d_ms, 3), batch_graph_mrays_s=round(rays / d_ms / 1e3, 1),
                             batch_stepped_no_graph_ms=round(e_ms, 3), speedup_vs_per_job=round(per_ms / d_ms, 3),
                             runs_ms=dict(per_job=per_all, batch=d_all))
            log(f"[batched] {mode}: {json.dumps(out[mode])}")
            continue
        t0 = time.perf_counter()
        best, _, tlog = autotune.coordinate_descent(lambda p: batch_ms(p)[0], autotune.search_space(mode), default)
        tune_s = time.perf_counter() - t0
        b_ms, b_all = batch_ms(best)
        out[mode] = dict(jobs=len(reqs), secondary_rays=rays,
                         per_job_ms=round(per_ms, 3), per_job_mrays_s=round(rays / per_ms / 1e3, 1),
                         batch_graph_ms=round(d_ms, 3), batch_graph_mrays_s=round(rays / d_ms / 1e3, 1),
                         batch_stepped_no_graph_ms=round(e_ms, 3),
                         tuned=dict(group=list(best["group"]), waves_per_cu=best["waves_per_cu"],
                                    refill=best["refill"], leaf_gate=best["leaf_gate"]),
                         tuned_ms=round(b_ms, 3), tuned_mrays_s=round(rays / b_ms / 1e3, 1),
                         speedup_vs_per_job=round(per_ms / b_ms, 3), tuning_s=round(tune_s, 1),
                         tuning_log=[[str(p["group"]), p["waves_per_cu"], p["refill"], p["leaf_gate"], round(c, 3)]
                                     for p, c in tlog],
                         runs_ms=dict(per_job=per_all, batch=d_all, tuned=b_all))
        log(f"[batched] {mode}: {json.dumps(out[mode])}")
    return out


def bench_serve(api, serve, scs, args):
    """Serving workload: Poisson arrivals of mixed requests, admission by the HBM budget,
    continuous batching; latency = finish - arrival."""
    import torch
    res = {}
    max_jobs = args.max_jobs
    big = max(api.batch_job_bytes(w, h, max(serve.SPPS), 4, "reuse") for w, h in serve.RESOLUTIONS)
    scene_bytes = sum(int(s.arena.numel()) for s in scs.values())
    budget = int(args.budget_gb * 1e9)
    arena = min(max_jobs * big + api.Batch.base_bytes(max_jobs), (budget - scene_bytes) // 2)
    for mode in args.modes.split(","):
        if mode == "sorted":
            continue
        backend = serve.BatchBackend(scs, max_jobs, arena)
        # warm the allocator and the kernels with a short burst
        serve.serve(serve.make_requests(16, None, list(scs), mode, seed=7), backend, budget)
        torch.cuda.synchronize()
        for rate in [float(x) for x in args.rates.split(",")]:
            reqs = serve.make_requests(args.requests, rate, list(scs), mode, seed=2310071824 + int(rate))
            log(f"[serve] {mode} rate {rate}/s: {len(reqs)} requests, warm-up {args.serve_warmup}")
            st = serve.serve(reqs, backend, budget)
            torch.cuda.synchronize()
            summ = st.summary(warmup=args.serve_warmup)
            res[f"{mode}@{rate:g}"] = {k: (round(v, 3) if isinstance(v, float) else v) for k, v in summ.items()}
            log(f"[serve] {mode} rate {rate}/s: {json.dumps(res[f'{mode}@{rate:g}'])}")
        del backend
        torch.cuda.empty_cache()
    return res, dict(budget_gb=args.budget_gb, scene_gb=round(scene_bytes / 1e9, 3), arena_gb=round(arena / 1e9, 3),
                     max_jobs=max_jobs)


TABLE3_TILES = ((8, 8), (16, 8), (16, 16), (32, 8))
TABLE3_KS = (8, 16, 32, 64)


def _ldr(x):
    # display transform for PSNR: clamp to [0, 1], gamma 1/2.2
    return x.clamp(0.0, 1.0).pow(1.0 / 2.2)


def psnr_db(img, ref):
    """PSNR in dB of an image against a reference, both display values in [0, 1] (numpy
    arrays of one shape): 10 log10(1 / mean squared difference over every pixel and channel)."""
    mse = float(np.mean((np.asarray(img, np.float64) - np.asarray(ref, np.float64)) ** 2))
    return 10.0 * np.log10(1.0 / mse) if mse > 0 else float("inf")


def tile_variance_ratio(err, tile):
    """Structured noise at the period of the reuse tiles: the variance of the error averaged
    over each W x H tile, times W*H, over the variance of the per-pixel error (channels
    averaged first; whole tiles only).  Independent pixel errors give 1; errors shared by
    groups of K pixels inside each tile give K, the correlation that the paper reports as
    visible noise for large groups (Sec. 5.3), which a per-pixel PSNR does not see."""
    e = np.asarray(err, np.float64)
    if e.ndim == 3:
        e = e.mean(axis=2)
    W, H = tile
    h, w = (e.shape[0] // H) * H, (e.shape[1] // W) * W
    e = e[:h, :w]
    e = e - e.mean()
    tm = e.reshape(h // H, H, w // W, W).mean(axis=(1, 3))
    return float(tm.var() * (W * H) / e.var())


def bench_quality(api, sc, cfg, args):
    """Image quality and the tile/group sweep (the protocols of the paper's Table 2 and
    Table 3): PSNR after `--quality-frames` frames (1 spp each, a new seed per frame, so
    the interleaved grouping changes every frame) against an incoherent reference of
    `--quality-ref` frames; secondary trace speed of every (W,H) x K with K <= W*H."""
    import torch
    w, h, B = cfg["w"], cfg["h"], cfg["bounces"]

    def average(mode, tile, k, frames, seed0, nee=False):
        r = api.Renderer(sc, api.RenderConfig(w, h, 1, B, mode, tile, k, nee=nee))
        acc = torch.zeros((h, w, 3), dtype=torch.float64, device="cuda:0")
        for i in range(frames):
            r.render(seed0 + i)
            acc += r.radiance.double()
        torch.cuda.synchronize()
        return acc / frames

    def trace_speed(mode, tile, k, nee=False):
        timer = api.Timer(4096)
        r = api.Renderer(sc, api.RenderConfig(w, h, 1, B, mode, tile, k, nee=nee), timer=timer)
        for i in range(3):
            r.render(11 + i)
        torch.cuda.synchronize()
        timer.reset()
        for i in range(10):
            r.render(100 + i)
        torch.cuda.synchronize()
        ms, kind, bounce = timer.read()
        rays = r.ray_count.cpu().numpy().reshape(-1).astype(np.float64)
        sec = (kind == 0) & (bounce >= 1)
        return rays[1:].sum() / (ms[sec].sum() / 10 * 1e-3) / 1e6

    t0 = time.perf_counter()
    ref = _ldr(average("incoherent", (8, 8), 8, args.quality_ref, 7_000_000))
    log(f"[quality] reference: {args.quality_ref} frames in {time.perf_counter() - t0:.1f} s")

    ref_np = ref.cpu().numpy()

    def psnr(img):
        return psnr_db(_ldr(img).cpu().numpy(), ref_np)

    def structure(img, tile):
        return tile_variance_ratio(_ldr(img).cpu().numpy() - ref_np, tile)

    out = {"reference_frames": args.quality_ref, "frames": args.quality_frames,
           "display": "clamp to [0,1], gamma 1/2.2, PSNR over all pixels and channels",
           "incoherent": {"psnr_db": round(psnr(average("incoherent", (8, 8), 8, args.quality_frames, 1)), 3),
                          "secondary_mrays_s": round(trace_speed("incoherent", (8, 8), 8), 1)}}
    rows = []
    for tile in TABLE3_TILES:
        for k in TABLE3_KS:
            if k > tile[0] * tile[1]:
                continue
            q = psnr(average("reuse", tile, k, args.quality_frames, 1))
            v = trace_speed("reuse", tile, k)
            rows.append({"tile": list(tile), "k": k, "psnr_db": round(q, 3), "secondary_mrays_s": round(v, 1),
                         "speedup_vs_incoherent": round(v / out["incoherent"]["secondary_mrays_s"], 3)})
            log(f"[quality] reuse {tile} K={k}: {rows[-1]}")
    out["reuse"] = rows
    # ablations: direct world-space reuse with one direction per 8x8 tile (Sec. 3.1) and
    # tangent-space reuse in non-interleaved groups (Sec. 3.3)
    abl = []
    for mode, tile, k in (("reuse_world", (8, 8), 64), ("reuse_world", (8, 8), 8), ("reuse_plain", (8, 8), 8),
                          ("reuse_plain", (8, 8), 64)):
        q = psnr(average(mode, tile, k, args.quality_frames, 1))
        v = trace_speed(mode, tile, k)
        abl.append({"mode": mode, "tile": list(tile), "k": k, "psnr_db": round(q, 3), "secondary_mrays_s": round(v, 1),
                    "speedup_vs_incoherent": round(v / out["incoherent"]["secondary_mrays_s"], 3)})
        log(f"[quality] {mode} {tile} K={k}: {abl[-1]}")
    out["ablations"] = abl
    # next-event estimation (the future-work extension): same expectation, less noise
    nee_rows = []
    for mode in ("incoherent", "reuse"):
        q = psnr(average(mode, (8, 8), 8, args.quality_frames, 1, nee=True))
        v = trace_speed(mode, (8, 8), 8, nee=True)
        nee_rows.append({"mode": mode, "nee": True, "tile": [8, 8], "k": 8, "psnr_db": round(q, 3),
                         "secondary_mrays_s": round(v, 1)})
        log(f"[quality] {mode} + NEE: {nee_rows[-1]}")
    out["nee"] = nee_rows
    # structured noise (Sec. 5.3: K = 32 in 8x8 tiles leaves visible noise after many frames):
    # the tile variance ratio of the error after 128 and after `--quality-long` frames
    srows = []
    for mode, tile, k in (("incoherent", (8, 8), 8), ("reuse", (8, 8), 8), ("reuse", (8, 8), 32),
                          ("reuse", (8, 8), 64), ("reuse", (16, 16), 32), ("reuse_plain", (8, 8), 8),
                          ("reuse_world", (8, 8), 8)):
        row = {"mode": mode, "tile": list(tile), "k": k}
        for frames in (args.quality_frames, args.quality_long):
            img = average(mode, tile, k, frames, 1)
            row[f"psnr_db_{frames}"] = round(psnr(img), 3)
            row[f"tile_variance_ratio_{frames}"] = round(structure(img, tile), 3)
        srows.append(row)
        log(f"[quality] structure {mode} {tile} K={k}: {row}")
    out["structure"] = srows
    return out


def bench_quality_short(api, sc, cfg, ref_frames=1024, frames=128, long_frames=1024):
    """A short form of the quality study for the default run (indoor, 1 spp per frame, a new
    seed per frame): PSNR after `frames` frames against an incoherent reference of
    `ref_frames` frames, for incoherent tracing and reuse in 8x8 tiles with K = 8, 32, 64
    (Table 2 and Table 3 protocols), and the tile variance ratio of the error (structured,
    tile-periodic noise; Sec. 5.3's K = 32 case) after `frames` and `long_frames` frames."""
    import torch
    w, h, B = cfg["w"], cfg["h"], cfg["bounces"]

    def average(mode, tile, k, n, seed0):
        r = api.Renderer(sc, api.RenderConfig(w, h, 1, B, mode, tile, k))
        acc = torch.zeros((h, w, 3), dtype=torch.float64, device="cuda:0")
        for i in range(n):
            r.render(seed0 + i)
            acc += r.radiance.double()
        torch.cuda.synchronize()
        return acc / n

    t0 = time.perf_counter()
    ref_np = _ldr(average("incoherent", (8, 8), 8, ref_frames, 7_000_000)).cpu().numpy()
    rows = []
    for mode, k in (("incoherent", 8), ("reuse", 8), ("reuse", 32), ("reuse", 64)):
        row = {"mode": mode, "tile": [8, 8], "k": k}
        for n in (frames, long_frames):
            img = _ldr(average(mode, (8, 8), k, n, 1)).cpu().numpy()
            row[f"psnr_db_{n}"] = round(psnr_db(img, ref_np), 3)
            row[f"tile_variance_ratio_{n}"] = round(tile_variance_ratio(img - ref_np, (8, 8)), 3)
        rows.append(row)
        log(f"[quality] {row}")
    return {"workload": f"indoor {w}x{h}, 1 spp per frame, {B} bounces, a new seed per frame; reference: "
                        f"{ref_frames} incoherent frames (other seeds); display: clamp to [0,1], gamma 1/2.2",
            "tile_variance_ratio": "variance of the error averaged over each 8x8 tile, times 64, over the "
                                   "variance of the per-pixel error: 1 for independent pixel errors, up to K "
                                   "for errors shared by the K pixels of a group",
            "rows": rows, "seconds": round(time.perf_counter() - t0, 1)}


def _csv_rows(path):
    import csv
    with open(path, newline="") as f:
        return list(csv.DictReader(f))


def summarize_profile(config, prof_dir, out_path, modes, bounces, counters):
    """Writes the text summary of a profiled `bench.py --config CONFIG --profile` run: the
    kernel-trace table, traversal launch times per mode and bounce, the counters per launch
    and the machine-readable lines the bench reads.  prof_dir holds pf_CONFIG_kt (kernel
    trace, stats and log) and pf_CONFIG_pmcI (one counter run each, in `counters` order)."""
    import glob
    import hashlib
    B1 = bounces + 1
    nm = len(modes)
    trace_name = "k_trace_q<false, false, true>"

    def trace_rows(rows, key="Kernel_Name"):
        return [r for r in rows if trace_name in r[key]]

    def mapping(n_dispatch):
        # 20 warm-up frames, then per mode 3 frames of B+1 launches; frames 1 and 2 are profiled
        assert n_dispatch == (20 + 3 * nm) * B1, (n_dispatch, (20 + 3 * nm) * B1)
        out = {}
        for i, m in enumerate(modes):
            for fr in (1, 2):
                for b in range(B1):
                    out.setdefault((m, b), []).append((20 + 3 * i + fr) * B1 + b)
        return out

    kt_dir = os.path.join(prof_dir, f"pf_{config}_kt")
    kt = _csv_rows(glob.glob(os.path.join(kt_dir, "*kernel_trace.csv"))[0])
    stats = _csv_rows(glob.glob(os.path.join(kt_dir, "*kernel_stats.csv"))[0])
    tr = trace_rows(kt)
    tr.sort(key=lambda r: int(r["Dispatch_Id"]))
    mp = mapping(len(tr))
    dur = {k: np.mean([(int(tr[i]["End_Timestamp"]) - int(tr[i]["Start_Timestamp"])) / 1e3 for i in v])
           for k, v in mp.items()}
    counts = {}
    with open(os.path.join(prof_dir, f"pf_{config}_kt.log")) as f:
        for line in f:
            if "[profile] counts " in line:
                c = json.loads(line.split("[profile] counts ", 1)[1])
                counts[c["mode"]] = c
    # counters: per run, per (mode, bounce) mean over the profiled frames; copy calibration
    ctr = {}
    calib = {}
    for j, names in enumerate(counters, start=1):
        rows = _csv_rows(glob.glob(os.path.join(prof_dir, f"pf_{config}_pmc{j}", "*counter_collection.csv"))[0])
        per = {}
        for r in rows:
            per.setdefault((int(r["Dispatch_Id"]), r["Kernel_Name"]), {})[r["Counter_Name"]] = float(r["Counter_Value"])
        disp = sorted(per.items(), key=lambda kv: kv[0][0])
        tdisp = [v for (d, name), v in disp if trace_name in name]
        m2 = mapping(len(tdisp))
        for nme in names.split():
            for k, idx in m2.items():
                ctr.setdefault(nme, {})[k] = float(np.mean([tdisp[i].get(nme, np.nan) for i in idx]))
            if nme in ("FETCH_SIZE", "WRITE_SIZE"):
                calib[nme] = max(v.get(nme, 0.0) for (d, name), v in disp if "copyBuffer" in name)
    gib_kib = float(1 << 20)
    fac = {k: gib_kib / v for k, v in calib.items() if v > 0}
    digest = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(os.path.join(ROOT, p), "rb") as f:
            digest.update(f.read())
    sha = digest.hexdigest()
    L = []
    L.append(f"# {trace_name.split('<')[0]} (closest-hit traversal over quantized four-wide nodes, per-wave triangle-test "
             f"queue), {config} 1920x1080, 1 spp, {bounces} bounces")
    L.append("")
    L.append("Workload: the seeded scene; one counting frame per mode (a separate counting instantiation of the "
             "kernel), 20 warm-up frames, then per mode one warm-up and two profiled frames "
             f"({B1} traversal launches each: bounce 0 = primary rays, 1..{bounces} = secondary), then a 1 GiB "
             "device-to-device copy that calibrates the byte counters.")
    L.append("")
    L.append("Commands (from the repository root, `export TMPDIR=/tmp` first), then this summary:")
    L.append("")
    L.append("```")
    pd = os.path.normpath(os.path.relpath(prof_dir, ROOT)) if os.path.isabs(prof_dir) else os.path.normpath(prof_dir)
    L.append(f"rocprofv3 --kernel-trace --stats --output-format csv -d {pd}/pf_{config}_kt -o kt -- "
             f"python -u bench.py --config {config} --profile > {pd}/pf_{config}_kt.log 2>&1")
    for j, names in enumerate(counters, start=1):
        L.append(f"timeout -s KILL 300 rocprofv3 --pmc {names} --output-format csv -d {pd}/pf_{config}_pmc{j} "
                 f"-o pmc -- python -u bench.py --config {config} --profile")
    L.append(f"python bench.py --summarize-profile {pd} --config {config}")
    L.append("```")
    L.append("")
    L.append("## Kernel trace summary (rocprofv3 --stats, all kernels of the run)")
    L.append("")
    L.append("| kernel | calls | total ms | avg us | min us | max us |")
    L.append("|---|---|---|---|---|---|")
    for r in stats[:14]:
        nm_ = r["Name"].replace("pt::(anonymous namespace)::", "").split("(")[0].replace("void ", "")
        L.append(f"| {nm_} | {r['Calls']} | {int(r['TotalDurationNs']) / 1e6:.3f} | {float(r['AverageNs']) / 1e3:.1f} | "
                 f"{int(r['MinNs']) / 1e3:.1f} | {int(r['MaxNs']) / 1e3:.1f} |")
    L.append("")
    L.append("## Traversal launch duration per mode and bounce (kernel trace, mean of the two profiled frames, us)")
    L.append("")
    L.append("| mode | " + " | ".join(f"b{b}" for b in range(B1)) + f" | mean b1..b{bounces} |")
    L.append("|---|" + "---|" * (B1 + 1))
    mean_sec = {}
    for m in modes:
        mean_sec[m] = float(np.mean([dur[(m, b)] for b in range(1, B1)]))
        L.append(f"| {m} | " + " | ".join(f"{dur[(m, b)]:.1f}" for b in range(B1)) + f" | {mean_sec[m]:.1f} |")
    L.append("")
    if fac:
        L.append("Byte calibration from the 1 GiB copy: " + ", ".join(
            f"{k} reads {calib[k]:.0f} KiB for 1,048,576 KiB (factor {fac[k]:.4f})" for k in sorted(fac)) +
            ". MB below = KiB x factor x 1024 / 1e6. FETCH_SIZE counts L2 misses served by the fabric (MALL hits "
            "included), an upper bound on HBM reads.")
        L.append("")
    cols = []

    def g(nme, k):
        return ctr.get(nme, {}).get(k, float("nan"))

    L.append("## Counters per traversal launch (mean of the two profiled frames)")
    L.append("")
    table = []
    traffic, lane_ops = {}, {}
    for m in modes:
        tb, lo = [], []
        for b in range(B1):
            k = (m, b)
            rd = g("FETCH_SIZE", k) * fac.get("FETCH_SIZE", float("nan")) * 1024
            wr = g("WRITE_SIZE", k) * fac.get("WRITE_SIZE", float("nan")) * 1024
            util = g("SQ_THREAD_CYCLES_VALU", k) / (64.0 * g("SQ_ACTIVE_INST_VALU", k))
            gui = g("GRBM_GUI_ACTIVE", k) / 8.0
            row = {"fabric read MB": rd / 1e6, "write MB": wr / 1e6,
                   "L2 hit": g("TCC_HIT_sum", k) / (g("TCC_HIT_sum", k) + g("TCC_MISS_sum", k)),
                   "VALU Minstr": g("SQ_INSTS_VALU", k) / 1e6, "VALU lane util": util,
                   "VALU issue": g("SQ_INSTS_VALU", k) * 4.0 / 1024.0 / gui,
                   "SALU Minstr": g("SQ_INSTS_SALU", k) / 1e6,
                   "TA busy": g("TA_TA_BUSY_sum", k) / 256.0 / gui, "TD busy": g("TD_TD_BUSY_sum", k) / 256.0 / gui,
                   "L1 lines / mem instr": g("TCP_TOTAL_CACHE_ACCESSES_sum", k) / g("SQ_INSTS_VMEM", k)}
            table.append((m, b, row))
            if b >= 1:
                tb.append(rd + wr)
                lo.append(g("SQ_INSTS_VALU", k) * 64.0 * util)
        traffic[m] = float(np.mean(tb))
        lane_ops[m] = float(np.mean(lo))
    # columns the counter runs of this workload cover
    cols = [c for c in table[0][2] if not all(np.isnan(r[c]) for _, _, r in table)]
    L.append("| mode | bounce | " + " | ".join(cols) + " |")
    L.append("|---|---|" + "---|" * len(cols))
    for m, b, row in table:
        L.append(f"| {m} | {b} | " + " | ".join(f"{row[c]:.3f}" if row[c] < 10 else f"{row[c]:.1f}" for c in cols) + " |")
    L.append("")
    L.append("VALU lane util = SQ_THREAD_CYCLES_VALU / (64 x SQ_ACTIVE_INST_VALU), the fraction of the 64 lanes active "
             "per VALU instruction. VALU issue = VALU instructions x 4 cycles / 1024 SIMDs / (GRBM_GUI_ACTIVE / 8). "
             "TA / TD busy = busy cycles summed over the 256 CUs / 256 / the same cycles. L1 lines / mem instr = "
             "TCP_TOTAL_CACHE_ACCESSES / SQ_INSTS_VMEM. Counters come from separate runs of the same sequence.")
    L.append("")
    L.append("## Roofline per secondary traversal launch (mean over bounces 1..%d)" % bounces)
    L.append("")
    L.append("Algorithmic bytes per ray = nodes x node bytes + triangles x 40 B + 32 B ray + 8 B hit, nodes and "
             "triangles per secondary ray from the counting frame; frac = algorithmic bytes per launch / mean launch "
             "time / 8 TB/s. Executed lane-ops = SQ_INSTS_VALU x 64 x lane util (all VALU work, overhead included), "
             "against 256 CUs x 64 lanes x 2.4 GHz = 39.3 T lane-op/s.")
    L.append("")
    L.append("| mode | nodes / ray | tris / ray | alg. bytes / ray | rays / launch | alg. bytes / launch | mean launch us | "
             "alg. GB/s | frac of 8 TB/s | counted traffic / launch | traffic GB/s | executed lane-ops / launch | "
             "executed frac of VALU |")
    L.append("|---|---|---|---|---|---|---|---|---|---|---|---|---|")
    for m in modes:
        c = counts.get(m)
        t = mean_sec[m] * 1e-6
        if c:
            abl = c["bytes_per_ray"] * c["rays_per_launch"]
            L.append(f"| {m} | {c['nodes_per_ray']:.2f} | {c['tris_per_ray']:.2f} | {c['bytes_per_ray']:.1f} | "
                     f"{c['rays_per_launch']:.0f} | {abl:.4g} | {mean_sec[m]:.1f} | {abl / t / 1e9:.0f} | "
                     f"{abl / t / 1e9 / HBM_PEAK_GBS:.3f} | {traffic[m]:.4g} | {traffic[m] / t / 1e9:.0f} | "
                     f"{lane_ops[m]:.4g} | {lane_ops[m] / t / 1e12 / VALU_PEAK_TOPS:.3f} |".replace("nan", "-"))
    L.append("")
    L.append("Machine-readable lines read by bench.py (source digest of kernels.hip, kernels.h, capi.hip, build.py and bvh_build.cpp "
             "when the counters were taken):")
    L.append("")
    L.append("```")
    L.append("traffic_bytes_per_launch " + " ".join(f"{m}={traffic[m]:.6g}" for m in modes) + f" source_sha256={sha}")
    if not any(np.isnan(v) for v in lane_ops.values()):
        L.append("valu_lane_ops_per_launch " + " ".join(f"{m}={lane_ops[m]:.6g}" for m in modes) +
                 f" source_sha256={sha}")
    L.append("mean_launch_us " + " ".join(f"{m}={mean_sec[m]:.1f}" for m in modes) + f" source_sha256={sha}")
    L.append("```")
    with open(out_path, "w") as f:
        f.write("\n".join(L) + "\n")
    return out_path


PROFILE_COUNTERS = {
    "indoor": ("FETCH_SIZE", "WRITE_SIZE",
               "SQ_WAVES SQ_INSTS_VALU SQ_INSTS_VMEM_RD SQ_INSTS_SALU SQ_INSTS_LDS SQ_WAVE_CYCLES SQ_BUSY_CYCLES "
               "SQ_WAIT_INST_ANY",
               "TCC_HIT_sum TCC_MISS_sum TCP_TOTAL_CACHE_ACCESSES_sum TCP_TCC_READ_REQ_sum GRBM_GUI_ACTIVE",
               "SQ_THREAD_CYCLES_VALU SQ_ACTIVE_INST_VALU",
               "TA_TA_BUSY_sum TD_TD_BUSY_sum TCP_TOTAL_CACHE_ACCESSES_sum SQ_INSTS_VMEM GRBM_GUI_ACTIVE"),
    "landscape": ("FETCH_SIZE", "WRITE_SIZE", "SQ_THREAD_CYCLES_VALU SQ_ACTIVE_INST_VALU"),
}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--config", default="all",
                    help="all (indoor, then landscape: the default run) or one of the scene configs")
    ap.add_argument("--no-deploy", action="store_true",
                    help="leave out the short batched and serving run of the default workload")
    ap.add_argument("--latency-frames", type=int, default=200,
                    help="frames rendered after the timed ones, for the p50/p99 frame latency")
    ap.add_argument("--modes", default="reuse,incoherent,sorted")
    ap.add_argument("--traversal", default="auto", choices=["auto", "pair", "wide", "queue", "quant"],
                    help="traversal kernel of the frame runs (pt_group.traversal); auto = the library's choice")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=15.0)
    ap.add_argument("--profile", action="store_true",
                    help="short fixed sequence for rocprofv3: per mode one warm-up and two frames, "
                         "then a 1 GiB device copy that calibrates the HBM byte counters")
    ap.add_argument("--batched", action="store_true",
                    help="batched workload: 64 mixed jobs, per-job launches vs merged graph launches, autotuned")
    ap.add_argument("--serve", action="store_true",
                    help="serving workload: Poisson arrivals, HBM-budget admission, continuous batching")
    ap.add_argument("--scenes", default=",".join(MIX_SCENES), help="resident scenes of --batched / --serve")
    ap.add_argument("--jobs", type=int, default=64)
    ap.add_argument("--reps", type=int, default=3)
    ap.add_argument("--rates", default="20,50,100")
    ap.add_argument("--requests", type=int, default=600)
    ap.add_argument("--serve-warmup", type=int, default=100)
    ap.add_argument("--budget-gb", type=float, default=200.0)
    ap.add_argument("--max-jobs", type=int, default=64)
    ap.add_argument("--nee", action="store_true",
                    help="next-event estimation at Lambert points (shadow rays), reported beside the paths")
    ap.add_argument("--quality", action="store_true",
                    help="PSNR against a many-frame reference and the (W,H) x K speed sweep")
    ap.add_argument("--quality-frames", type=int, default=128)
    ap.add_argument("--quality-ref", type=int, default=4096)
    ap.add_argument("--quality-long", type=int, default=2048,
                    help="frames of the long runs of the structured-noise rows")
    ap.add_argument("--summarize-profile", metavar="DIR",
                    help="write profiles/k_trace_CONFIG_1080p.md from the rocprofv3 runs of --profile under DIR")
    ap.add_argument("--cpu-worker", action="store_true", help=argparse.SUPPRESS)
    ap.add_argument("--cpu-part", type=int, default=0, help=argparse.SUPPRESS)
    ap.add_argument("--cpu-parts", type=int, default=1, help=argparse.SUPPRESS)
    ap.add_argument("--cpu-reps", type=int, default=1, help=argparse.SUPPRESS)
    ap.add_argument("--cpu-start", type=float, default=0.0, help=argparse.SUPPRESS)
    args = ap.parse_args()
    if args.cpu_worker:
        cpu_worker(args)
        return
    if args.summarize_profile:
        from paper_2310_07182_amd import scenes
        name = "indoor" if args.config == "all" else args.config
        out = PROFILE_SUMMARY.format(config=name)
        summarize_profile(name, args.summarize_profile, out, args.modes.split(","),
                          scenes.CONFIGS[name]["bounces"], PROFILE_COUNTERS[name])
        print(out)
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU only: the library has no multi-GPU path (asked for {args.gpus}); "
              "run with --gpus 1", file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_2310_07182_amd import api, scenes

    if args.batched or args.serve:
        from paper_2310_07182_amd import autotune, serve
        scs = load_scenes(api, scenes, args.scenes.split(","))
        line = {"metric": "batched and served secondary Mrays/s, p50/p99 request latency", "n_gpus": 1,
                "data": "synthetic (seeded procedural scenes)", "dtype": "f32",
                "config": {"workload": f"mixed jobs over resident scenes {args.scenes}: resolutions "
                                       f"{[f'{w}x{h}' for w, h in serve.RESOLUTIONS]}, spp {list(serve.SPPS)}, "
                                       "4 bounces, tile 8x8 / K=8 unless tuned"}}
        if args.batched:
            line["batched"] = bench_batched(api, serve, autotune, scs, args)
        if args.serve:
            line["serving"], line["serving_setup"] = bench_serve(api, serve, scs, args)
        print(json.dumps(line), flush=True)
        return
    if not (args.quality or args.profile):
        line = bench_frames(api, scenes, args, torch)
        print(json.dumps(line), flush=True)
        return
    if args.config == "all":
        args.config = "indoor"
    cfg = dict(scenes.CONFIGS[args.config])
    t0 = time.perf_counter()
    scene = cfg["scene"]()
    gen_s = time.perf_counter() - t0
    t0 = time.perf_counter()
    sc = api.Scene(scene, device="cuda:0")
    build_s = time.perf_counter() - t0
    log(f"[bench] {args.config}: {scene.ntri} triangles, generated in {gen_s:.1f} s, BVH+upload {build_s:.1f} s, "
        f"info {sc.info()}")
    if args.quality:
        line = {"metric": "PSNR (dB) after N frames vs a many-frame reference; secondary Mrays/s per (W,H) x K",
                "n_gpus": 1, "data": "synthetic (seeded procedural scene)", "dtype": "f32",
                "config": {"workload": f"{args.config}: {cfg['w']}x{cfg['h']}, 1 spp per frame, {cfg['bounces']} bounces, "
                                       f"{scene.ntri} triangles"},
                "quality": bench_quality(api, sc, cfg, args)}
        print(json.dumps(line), flush=True)
        return
    if args.profile:
        # warm the GPU up (clocks, caches) with 20 untimed frames before the profiled sequence
        rw = api.Renderer(sc, api.RenderConfig(cfg["w"], cfg["h"], 1, cfg["bounces"], "incoherent", tuple(cfg["tile"]),
                                               cfg["k"], traversal=args.traversal))
        for j in range(20):
            rw.render(7 + j)
        torch.cuda.synchronize()
        del rw
        log("[profile] 20 warm-up frames")
        # counting frame per mode (a separate, counting instantiation of the traversal kernel):
        # nodes and triangles per secondary ray and rays per launch, the algorithmic bytes of the summary
        node_bytes, _ = node_costs(sc, args.traversal)
        for i, mode in enumerate(args.modes.split(",")):
            rs = api.Renderer(sc, api.RenderConfig(cfg["w"], cfg["h"], 1, cfg["bounces"], mode, tuple(cfg["tile"]),
                                                   cfg["k"], traversal=args.traversal), stats=True)
            rs.render(2310071821 + 10 * i)
            torch.cuda.synchronize()
            st = rs.stats.cpu().numpy().astype(np.float64)
            rc_ = rs.ray_count.cpu().numpy().reshape(-1).astype(np.float64)
            npr, tpr = st[1:, 0].sum() / rc_[1:].sum(), st[1:, 1].sum() / rc_[1:].sum()
            bpr = npr * node_bytes + tpr * TRI_BYTES + RAY_BYTES + HIT_BYTES
            log("[profile] counts " + json.dumps({"mode": mode, "nodes_per_ray": npr, "tris_per_ray": tpr,
                                                  "node_bytes": node_bytes, "bytes_per_ray": bpr,
                                                  "rays_per_launch": rc_[1:].sum() / cfg["bounces"]}))
            del rs
        for i, mode in enumerate(args.modes.split(",")):
            r = api.Renderer(sc, api.RenderConfig(cfg["w"], cfg["h"], 1, cfg["bounces"], mode, tuple(cfg["tile"]),
                                                  cfg["k"], traversal=args.traversal))
            for j in range(3):
                r.render(2310071821 + 10 * i + j)
                torch.cuda.synchronize()
            log(f"[profile] {mode}: 3 frames ({cfg['bounces'] + 1} traversal launches each)")
        x = torch.empty(1 << 28, dtype=torch.float32, device="cuda:0")
        y = torch.empty_like(x)
        torch.cuda.synchronize()
        y.copy_(x)
        torch.cuda.synchronize()
        log("[profile] copy of 1 GiB done")
        return


# Rows of the default run: (label, mode, tile, K, frame_groups, reuse_max_bounce); None = the
# config's own tile / K / every bounce.  The first row is the headline.
INDOOR_POINTS = (("reuse", "reuse", None, None, False, None),
                 ("incoherent", "incoherent", None, None, False, None),
                 ("sorted", "sorted", None, None, False, None),
                 ("reuse_frame_groups", "reuse", None, None, True, None),
                 ("reuse_first_bounce", "reuse", None, None, False, 1),
                 ("reuse_4x4_k2", "reuse", (4, 4), 2, False, None))
LANDSCAPE_POINTS = (("reuse", "reuse", None, None, False, None),
                    ("incoherent", "incoherent", None, None, False, None),
                    ("sorted", "sorted", None, None, False, None),
                    ("reuse_frame_groups", "reuse", None, None, True, None))


def profile_figures(mode, config):
    """Per secondary traversal launch, from the committed rocprofv3 summary of this kernel and
    workload: counted traffic (FETCH_SIZE + WRITE_SIZE, calibrated bytes) and executed VALU
    lane operations (SQ_THREAD_CYCLES_VALU-based); None for figures taken from other sources."""
    import hashlib
    path = PROFILE_SUMMARY.format(config=config)
    out = {}
    if not os.path.exists(path):
        return out
    digest = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(os.path.join(ROOT, p), "rb") as f:
            digest.update(f.read())
    with open(path) as f:
        for line in f:
            parts = line.split()
            if len(parts) < 2 or parts[0] not in ("traffic_bytes_per_launch", "valu_lane_ops_per_launch",
                                                  "mean_launch_us"):
                continue
            fields = dict(kv.split("=", 1) for kv in parts[1:])
            if fields.get("source_sha256") == digest.hexdigest() and mode in fields:
                out[parts[0]] = float(fields[mode])
    return out


def roofline(head, sc, trav, ceil, config, level):
    """The traversal kernel's roofline over the secondary bounces of the headline mode.
    Primary bound: algorithmic bytes (nodes x node bytes + triangles x 40 B + 32 B ray + 8 B
    hit per traced ray, node and triangle counts from the counting frame) per launch over the
    mean launch time, against the 8 TB/s HBM peak.  Second bound: the VALU, algorithmic lane
    operations per launch over the launch time against 256 CUs x 64 lanes x 2.4 GHz."""
    t = head["avg_trace_launch_ms"] * 1e-3
    gbs = head["bytes_per_launch"] / t / 1e9
    ops = head["ops_per_launch"] / t / 1e12
    prof = profile_figures(head["mode"], config) if trav == "auto" else {}
    traffic = prof.get("traffic_bytes_per_launch")
    counted_ops = prof.get("valu_lane_ops_per_launch")
    rays_per_launch = head["bytes_per_launch"] / head["bytes_per_ray"]
    return {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(gbs / HBM_PEAK_GBS, 4), "traffic": round(traffic) if traffic else None,
            "kernel": kernel_label(sc, trav) + ", secondary bounces",
            "unit_of_work": "one traced secondary ray",
            "bytes_per_ray_formula": f"nodes x {node_costs(sc, trav)[0]} B + triangles x {TRI_BYTES} B + "
                                     f"{RAY_BYTES} B ray + {HIT_BYTES} B hit",
            "nodes_per_ray": round(head["nodes_per_ray"], 2), "tris_per_ray": round(head["tris_per_ray"], 2),
            "algorithmic_bytes_per_ray": round(head["bytes_per_ray"], 1),
            "rays_per_launch": round(rays_per_launch),
            "algorithmic_bytes_per_launch": round(head["bytes_per_launch"]),
            "mean_launch_us": round(head["avg_trace_launch_ms"] * 1e3, 1),
            "compulsory_bytes_per_launch": round(head["compulsory_bytes_per_launch"]),
            "traffic_over_compulsory": round(traffic / head["compulsory_bytes_per_launch"], 2) if traffic else None,
            "traffic_GBps": round(traffic / t / 1e9, 1) if traffic else None,
            "working_set_level": level, "measured_ceiling_GBps": ceil[level]["read_GBps"] if ceil else None,
            "algorithmic_frac_of_measured_ceiling": round(gbs / ceil[level]["read_GBps"], 4) if ceil else None,
            "valu": {"achieved": round(ops, 3), "peak": round(VALU_PEAK_TOPS, 2), "unit": "T lane-op/s",
                     "frac": round(ops / VALU_PEAK_TOPS, 4), "ops_per_ray": round(head["ops_per_ray"], 1),
                     "op": "32-bit VALU lane operation (compare/min/max/select counted like add/mul), "
                           "hand-counted per node visit and triangle test",
                     "executed_lane_ops_per_launch": round(counted_ops) if counted_ops else None,
                     "executed_frac": round(counted_ops / t / 1e12 / VALU_PEAK_TOPS, 4) if counted_ops else None}}


def _mode_summary(v, nee=False):
    return {"mode": v["mode"], "tile": v["tile"], "k": v["k"], "frame_groups": v["frame_groups"],
            "reuse_max_bounce": v["reuse_max_bounce"],
            "secondary_mrays_s": round(v["secondary_mrays_s"], 3),
            "secondary_mrays_s_frame_sd": round(v["secondary_mrays_s_frame_sd"], 2),
            "end_to_end_secondary_mrays_s": round(v["end_to_end_secondary_mrays_s"], 3),
            "frame_ms_p50": round(v["frame_ms_p50"], 4), "frame_ms_p99": round(v["frame_ms_p99"], 4),
            "latency_frames": v["latency_frames"],
            "trace_us_per_bounce": [round(x, 1) for x in v["trace_us_per_bounce"]],
            "shade_us_per_bounce": [round(x, 1) for x in v["shade_us_per_bounce"]],
            "ms_by_kind": {TIMER_KIND_NAMES.get(kk, str(kk)): round(x, 4) for kk, x in v["ms_by_kind"].items()},
            "rays_per_bounce": v["rays_per_bounce"], "nodes_per_ray": round(v["nodes_per_ray"], 2),
            "tris_per_ray": round(v["tris_per_ray"], 2),
            "compulsory_bytes_per_bounce": [round(x) for x in v["compulsory_bytes_per_bounce"]],
            **({"shadow_mrays_s": round(v["shadow_mrays_s"], 3),
                "shadow_rays_per_frame": v["shadow_rays_per_frame"]} if nee else {})}


TIMER_KIND_NAMES = {0: "trace", 1: "raygen", 2: "shade", 3: "key", 4: "sort", 6: "other",
                    7: "shadow_trace", 8: "shadow_accumulate"}


def bench_config(api, scenes, name, points, args, torch):
    cfg = dict(scenes.CONFIGS[name])
    t0 = time.perf_counter()
    scene = cfg["scene"]()
    gen_s = time.perf_counter() - t0
    t0 = time.perf_counter()
    sc = api.Scene(scene, device="cuda:0")
    build_s = time.perf_counter() - t0
    log(f"[bench] {name}: {scene.ntri} triangles, generated in {gen_s:.1f} s, BVH+upload {build_s:.1f} s, "
        f"info {sc.info()}")
    # the same untimed warm-up before every mode's own warm-up, so the first mode does not meet
    # a GPU whose clocks are still ramping up
    rw = api.Renderer(sc, api.RenderConfig(cfg["w"], cfg["h"], 1, cfg["bounces"], "incoherent", tuple(cfg["tile"]),
                                           cfg["k"], traversal=args.traversal))
    for j in range(20):
        rw.render(7 + j)
    torch.cuda.synchronize()
    del rw
    results = {}
    for i, (label, mode, tile, k, fg, rmax) in enumerate(points):
        log(f"[bench] {name} {label}: warmup {args.warmup}, steps {args.steps}, then {args.latency_frames} latency frames")
        results[label] = bench_mode(api, sc, cfg, mode, args.steps, args.warmup, 2310071821 + 100000 * i, args.nee,
                                    args.traversal, tile, k, fg, rmax, args.latency_frames)
        log(f"[bench] {name} {label}: {json.dumps(results[label])}")
    level = "mall" if sc.arena.numel() <= MALL_BYTES else "hbm"
    info = dict(scene=scene, sc=sc, sc_info=sc.info(), cfg=cfg, level=level, ntri=int(scene.ntri),
                gen_s=gen_s, build_s=build_s)
    return results, info


def bench_deploy(api, scenes, args, resident):
    """A short run of the deployment patterns over the resident scenes (indoor and landscape
    from the frame runs, plus tiny and mid): 64 mixed jobs as per-job pt_render calls and as
    one batch (merged launches, captured graph, default launch parameters), and a Poisson
    serving run at 100 requests/s with continuous batching, for reuse and incoherent jobs."""
    import types
    from paper_2310_07182_amd import autotune, serve
    scs = dict(resident)
    for n in ("tiny", "mid"):
        scs[n] = api.Scene(getattr(scenes, n)(), device="cuda:0")
    a = types.SimpleNamespace(modes="reuse,incoherent", jobs=64, reps=3, rates="100", requests=400, serve_warmup=50,
                              budget_gb=200.0, max_jobs=64)
    log("[bench] deployment: batched")
    batched = bench_batched(api, serve, autotune, scs, a, tune=False)
    log("[bench] deployment: serving")
    serving, setup = bench_serve(api, serve, scs, a)
    keep = ("requests", "latency_ms_p50", "latency_ms_p99", "mrays_s", "requests_per_s", "max_in_flight",
            "refused_admissions")
    return {"workload": f"{a.jobs} mixed jobs / {a.requests} Poisson requests at 100/s over resident scenes "
                        f"{sorted(scs)}: resolutions {[f'{w}x{h}' for w, h in serve.RESOLUTIONS]}, spp "
                        f"{list(serve.SPPS)}, 4 bounces, tile 8x8 / K=8; first {a.serve_warmup} requests excluded",
            "batched": {m: {k: v[k] for k in ("jobs", "secondary_rays", "per_job_ms", "batch_graph_ms",
                                               "batch_stepped_no_graph_ms", "batch_graph_mrays_s", "speedup_vs_per_job")}
                        for m, v in batched.items()},
            "serving": {m: {k: v[k] for k in keep if k in v} for m, v in serving.items()},
            "serving_setup": setup}


def bench_sort_yardstick(api, torch, n, reps=20):
    """The sorted modes' radix sort (pt_sort_pairs: 4 passes of 8-bit digits) beside the vendor
    library's device radix sort (rocPRIM radix_sort_pairs in libptsortref.so) on n seeded
    uniform 30-bit keys with their indices as values; median microseconds of reps sorts each."""
    import ctypes as C
    from paper_2310_07182_amd import build as B
    L = C.CDLL(B.SORTREF_LIB)
    L.ptref_sort_workspace_bytes.argtypes = [C.c_uint32, C.c_int, C.POINTER(C.c_size_t)]
    L.ptref_sort_pairs.argtypes = [C.c_void_p, C.c_size_t, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                   C.c_uint32, C.c_int, C.c_void_p]
    rng = np.random.default_rng(2310071825)
    k0 = torch.from_numpy(rng.integers(0, 1 << 30, n, dtype=np.int64).astype(np.int32)).to("cuda:0")
    v0 = torch.arange(n, dtype=torch.int32, device="cuda:0")
    k1, v1 = torch.empty_like(k0), torch.empty_like(v0)
    kr, vr = torch.empty_like(k0), torch.empty_like(v0)
    st = torch.cuda.current_stream()
    out = {"n": n, "keys": "uniform 30-bit, seeded; values = indices", "reps": reps}

    def ours():
        k1.copy_(k0)
        v1.copy_(v0)
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(st)
        api.sort_pairs(k1, v1)
        b.record(st)
        return a, b

    for bits in (30, 32):
        need = C.c_size_t(0)
        assert L.ptref_sort_workspace_bytes(n, bits, C.byref(need)) == 0
        ws = torch.empty(max(int(need.value), 256), dtype=torch.uint8, device="cuda:0")

        def lib_sort():
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(st)
            rc = L.ptref_sort_pairs(ws.data_ptr(), ws.numel(), k0.data_ptr(), kr.data_ptr(), v0.data_ptr(),
                                    vr.data_ptr(), n, bits, st.cuda_stream)
            b.record(st)
            assert rc == 0, rc
            return a, b

        times = []
        for i in range(reps + 2):
            a, b = lib_sort()
            torch.cuda.synchronize()
            if i >= 2:
                times.append(a.elapsed_time(b) * 1e3)
        out[f"rocprim_{bits}bit_us"] = round(float(np.median(times)), 1)
    times = []
    for i in range(reps + 2):
        a, b = ours()
        torch.cuda.synchronize()
        if i >= 2:
            times.append(a.elapsed_time(b) * 1e3)
    out["ours_us"] = round(float(np.median(times)), 1)
    # both sorts are stable: equal keys and equal values
    out["same_result"] = bool(torch.equal(k1, kr) and torch.equal(v1, vr))
    return out


def bench_frames(api, scenes, args, torch):
    """The default run: every configured workload, its modes and extra points, the memory
    ceilings, the roofline of the traversal kernel and the CPU oracle baseline."""
    if args.config == "all":
        plan = [("indoor", INDOOR_POINTS), ("landscape", LANDSCAPE_POINTS)]
    else:
        plan = [(args.config, tuple((m, m, None, None, False, None) for m in args.modes.split(",")))]
    out = {}
    for name, points in plan:
        res, info = bench_config(api, scenes, name, points, args, torch)
        out[name] = (res, info)
    quality = None
    if args.config == "all" and not args.no_deploy:
        log("[bench] short quality study")
        quality = bench_quality_short(api, out[plan[0][0]][1]["sc"], out[plan[0][0]][1]["cfg"])
    deploy = None
    if args.config == "all" and not args.no_deploy:
        deploy = bench_deploy(api, scenes, args, {n: info["sc"] for n, (res, info) in out.items()})
    for name, (res, info) in out.items():
        if name != plan[0][0]:
            del info["sc"], info["scene"]
    torch.cuda.empty_cache()
    yard = None
    res_first = out[plan[0][0]][0]
    srt = next((v for v in res_first.values() if v["mode"] == "sorted" and not v.get("frame_groups")), None)
    if srt is not None:
        nb = len(srt["rays_per_bounce"]) - 1
        n_live = int(round(float(np.mean(srt["rays_per_bounce"][1:]))))
        log(f"[bench] sort yardstick, {n_live} keys")
        yard = bench_sort_yardstick(api, torch, n_live)
        yard["in_frame_us_per_bounce"] = {
            "keys": round(srt["ms_by_kind"].get(3, 0.0) * 1e3 / nb, 1),
            "sort": round(srt["ms_by_kind"].get(4, 0.0) * 1e3 / nb, 1),
            "workload": f"{plan[0][0]} sorted mode: live rays of a bounce, 30-bit keys, 4 passes of 8-bit digits"}
        log(f"[bench] sort yardstick: {yard}")
    log("[bench] memory ceilings")
    ceil = measure_ceilings(api)
    log(f"[bench] ceilings: {ceil}")
    name0 = plan[0][0]
    res0, info0 = out[name0]
    head = next(iter(res0.values()))
    cfg0 = info0["cfg"]
    cpu = None
    if not args.no_cpu_baseline:
        log("[bench] cpu baseline (oracle, bounded sample)")
        single = cpu_baseline(info0["scene"], cfg0, name0, args.cpu_budget)
        log(f"[bench] cpu baseline, one core: {single}")
        log("[bench] cpu baseline on every host core")
        cpu = cpu_baseline_all_cores(cfg0, name0, single)
        log(f"[bench] cpu baseline, all cores: {cpu}")

    def workload(name, info):
        c = info["cfg"]
        return (f"{name}: {c['w']}x{c['h']}, 1 spp, {c['bounces']} bounces, {info['ntri']} triangles, "
                f"tile {c['tile'][0]}x{c['tile'][1]}, K={c['k']}")

    line = {
        "metric": "secondary Mrays/s (reuse vs incoherent vs sorted) + p99 frame latency",
        "value": round(head["secondary_mrays_s"], 3),
        "unit": "Mrays/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(head["frame_ms_mean"], 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (seeded procedural scenes standing in for the paper's archived scenes)",
        "config": {"workload": workload(name0, info0), "mode": head["mode"], "parallelism": "single GPU",
                   "nee": bool(args.nee), "traversal": traversal_kind(info0["sc_info"], args.traversal),
                   "metric_definition": "rays traced at bounces 1..B / summed traversal-kernel time of those "
                                        "bounces (HIP events on the library's stream), per frame of exactly "
                                        "`steps` timed frames; p50/p99 frame latency over "
                                        f"{args.latency_frames} frames rendered after them without "
                                        "the per-kernel timer"},
        "modes": {lab: _mode_summary(v, args.nee) for lab, v in res0.items()},
        "p99_frame_ms": round(head["frame_ms_p99"], 4),
        "roofline": roofline(head, info0["sc_info"], args.traversal, ceil, name0, info0["level"]),
    }
    for name, (res, info) in out.items():
        if name == name0:
            continue
        h = next(iter(res.values()))
        line[name] = {"workload": workload(name, info), "value": round(h["secondary_mrays_s"], 3),
                      "p99_frame_ms": round(h["frame_ms_p99"], 4),
                      "modes": {lab: _mode_summary(v, args.nee) for lab, v in res.items()},
                      "roofline": roofline(h, info["sc_info"], args.traversal, ceil, name, info["level"])}
    if quality is not None:
        line["quality"] = quality
    if deploy is not None:
        line["deployment"] = deploy
    if yard is not None:
        line["sort_yardstick"] = yard
    line["ceilings"] = ceil
    line["cpu_baseline"] = None if cpu is None else {k: cpu[k] for k in ("value", "unit", "cores", "kind", "sample",
                                                                         "single_core_value", "single_core_sample")}
    return line


if __name__ == "__main__":
    main()
