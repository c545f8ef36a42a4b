"""Serving: continuous batching of render requests over device-resident scenes.

Requests arrive over time (Poisson arrivals for the serving workload, all at once
for a static batch).  The request loop keeps the scenes, their BVHs and the path
state of every request in flight on the device, admits waiting requests first
come first served while a slot of the batch, room in its arena and the HBM budget
allow, and advances every request in flight by one bounce per step with one
merged launch per kernel (pt_batch_step).  A finished request frees its slot and
memory at once, so requests that arrive while others run join the next step.

The loop itself is plain host logic over a small backend interface, so that the
admission and accounting rules run on the CPU in tests with a simulated backend;
`BatchBackend` is the GPU backend over `api.Batch`.
"""
from __future__ import annotations

import collections
import time
from dataclasses import dataclass, field

import numpy as np

# the mixed job population of the batched and serving workloads
RESOLUTIONS = ((256, 256), (512, 512), (1280, 720), (1920, 1080))
SPPS = (1, 2, 4)


@dataclass
class Request:
    rid: int
    arrival: float          # seconds after the start of the run
    scene: str
    w: int
    h: int
    spp: int
    bounces: int
    mode: str
    seed: int


def make_requests(n, rate, scenes, mode, seed, bounces=4, resolutions=RESOLUTIONS, spps=SPPS):
    """n requests with exponential inter-arrival times of mean 1/rate (rate None: all
    arrive at 0), scene, resolution and spp drawn uniformly, seeded."""
    rng = np.random.default_rng(seed)
    if rate is None:
        arrivals = np.zeros(n)
    else:
        arrivals = np.cumsum(rng.exponential(1.0 / float(rate), n))
    sc = rng.integers(0, len(scenes), n)
    res = rng.integers(0, len(resolutions), n)
    spp = rng.integers(0, len(spps), n)
    seeds = rng.integers(1, 1 << 62, n)
    return [Request(i, float(arrivals[i]), scenes[sc[i]], resolutions[res[i]][0], resolutions[res[i]][1],
                    int(spps[spp[i]]), int(bounces), mode, int(seeds[i])) for i in range(n)]


def output_bytes(r: Request) -> int:
    """Device bytes of a request's outputs: radiance [h][w][3] f32, hit prim and t
    [B+1][spp][h][w] i32/f32."""
    px = r.w * r.h
    return px * 3 * 4 + 2 * (r.bounces + 1) * r.spp * px * 4


@dataclass
class Record:
    rid: int
    arrival: float
    admitted: float = float("nan")
    finished: float = float("nan")
    rays: object = 0            # secondary rays traced (int, or a device scalar until the end)


@dataclass
class ServeStats:
    records: list
    wall_s: float
    steps: int
    max_in_flight: int
    max_waiting: int
    peak_budget_bytes: int
    refused_admissions: int = 0
    extra: dict = field(default_factory=dict)

    def summary(self, warmup: int = 0) -> dict:
        recs = [r for r in self.records if r.rid >= warmup]
        lat = np.array([r.finished - r.arrival for r in recs]) * 1e3
        wait = np.array([r.admitted - r.arrival for r in recs]) * 1e3
        rays = float(sum(float(r.rays) for r in recs))
        t0 = min(r.arrival for r in recs)
        t1 = max(r.finished for r in recs)
        return dict(requests=len(recs), latency_ms_p50=float(np.percentile(lat, 50)),
                    latency_ms_p99=float(np.percentile(lat, 99)), latency_ms_mean=float(lat.mean()),
                    queue_wait_ms_p99=float(np.percentile(wait, 99)), secondary_rays=rays,
                    mrays_s=rays / max(t1 - t0, 1e-9) / 1e6, window_s=t1 - t0,
                    requests_per_s=len(recs) / max(t1 - t0, 1e-9), steps=self.steps,
                    max_in_flight=self.max_in_flight, max_waiting=self.max_waiting,
                    peak_budget_gb=self.peak_budget_bytes / 1e9, refused_admissions=self.refused_admissions)


def serve(requests, backend, budget_bytes, clock=time.perf_counter, sleep=time.sleep, idle_sleep=1e-4,
          on_finish=None) -> ServeStats:
    """Run the request loop until every request has finished.

    backend: submit(req) -> handle or None (no slot or arena room now), step() -> jobs
    advanced, done(handle) -> bool, release(handle, req) -> secondary rays, resident_bytes()
    -> bytes held whatever the load (scenes, arena).  budget_bytes bounds resident bytes
    plus the outputs of the requests in flight; a request that can never fit is an error.
    """
    reqs = sorted(requests, key=lambda r: (r.arrival, r.rid))
    resident = int(backend.resident_bytes())
    if resident > budget_bytes:
        raise ValueError(f"scenes and arena ({resident} B) exceed the HBM budget ({budget_bytes} B)")
    for r in reqs:
        if resident + output_bytes(r) > budget_bytes:
            raise ValueError(f"request {r.rid} ({output_bytes(r)} B of outputs) can never fit the HBM budget")
    recs = {r.rid: Record(r.rid, r.arrival) for r in reqs}
    waiting = collections.deque()
    live = {}                   # handle -> request
    used = resident
    peak = used
    nxt = 0
    steps = max_live = max_wait = refused = 0
    t0 = clock()
    finished = 0
    while finished < len(reqs):
        now = clock() - t0
        while nxt < len(reqs) and reqs[nxt].arrival <= now:
            waiting.append(reqs[nxt])
            nxt += 1
        max_wait = max(max_wait, len(waiting))
        # admission, first come first served: the head waits until it fits
        while waiting:
            r = waiting[0]
            need = output_bytes(r)
            if used + need > budget_bytes:
                refused += 1
                break
            h = backend.submit(r)
            if h is None:
                refused += 1
                break
            waiting.popleft()
            live[h] = r
            used += need
            peak = max(peak, used)
            recs[r.rid].admitted = clock() - t0
        if waiting and not live:
            raise RuntimeError(f"request {waiting[0].rid} cannot be admitted even with nothing in flight "
                               "(batch arena too small for it)")
        max_live = max(max_live, len(live))
        advanced = backend.step() if live else 0
        if advanced:
            steps += 1
        for h in [h for h in live if backend.done(h)]:
            r = live.pop(h)
            rec = recs[r.rid]
            rec.finished = clock() - t0
            rec.rays = backend.release(h, r)
            used -= output_bytes(r)
            finished += 1
            if on_finish is not None:
                on_finish(r, h)
        if not advanced:
            if live:
                sleep(idle_sleep)          # every step of the jobs in flight is enqueued
            elif nxt < len(reqs):
                gap = reqs[nxt].arrival - (clock() - t0)
                if gap > 0:
                    sleep(min(gap, 0.01))
    wall = clock() - t0
    return ServeStats([recs[r.rid] for r in sorted(reqs, key=lambda r: r.rid)], wall, steps, max_live, max_wait,
                      peak, refused)


class BatchBackend:
    """GPU backend of the request loop: an `api.Batch` over device-resident scenes;
    a request's outputs are torch tensors allocated at admission and dropped at release
    (kept for the request ids in `keep`)."""

    def __init__(self, scenes: dict, max_jobs: int, arena_bytes: int, tile=(8, 8), k=8, refill=0, waves_per_cu=0,
                 device="cuda:0", keep=()):
        import torch
        from . import api
        self.torch, self.api = torch, api
        self.scenes = scenes
        self.batch = api.Batch(max_jobs, arena_bytes, tile=tile, k=k, refill=refill, waves_per_cu=waves_per_cu,
                               device=device)
        self.device = self.batch.device
        self.keep = set(keep)
        self.kept = {}
        self.outs = {}
        self.count = None

    def resident_bytes(self) -> int:
        return sum(int(s.arena.numel()) for s in self.scenes.values()) + int(self.batch.arena.numel())

    def submit(self, r: Request):
        o = self.api.JobOutputs(r.w, r.h, r.spp, r.bounces, self.device)
        job = self.batch.job_struct(self.scenes[r.scene], r.w, r.h, r.spp, r.bounces, r.mode, r.seed, o)
        jid = self.batch.submit(job, keep=o)
        if jid is None:
            return None
        self.outs[jid] = o
        return jid

    def step(self) -> int:
        return self.batch.step()

    def done(self, h) -> bool:
        return self.batch.done(h)

    def release(self, h, r: Request):
        o = self.outs.pop(h)
        self.batch.release(h)
        # secondary rays traced = hit records at bounces >= 1 that are not "no ray" (-2);
        # summed on the device, read once at the end
        n = (o.hit_prim[1:] != -2).sum()
        if r.rid in self.keep:
            self.kept[r.rid] = o
        return n
