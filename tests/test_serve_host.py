"""Host logic of serving and autotuning, on the CPU: request generation, the
request loop's admission and accounting against a simulated backend, and the
coordinate-descent search."""
import math

import numpy as np
import pytest

from paper_2310_07182_amd import autotune, serve


class Clock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t

    def sleep(self, dt):
        self.t += max(dt, 1e-6)


class FakeBackend:
    """Each job needs spp * (bounces + 1) steps; a step takes step_s of simulated time.
    Slots and an arena of fixed size bound the jobs in flight, as in pt_batch."""

    def __init__(self, clock, max_jobs=4, arena=10**9, step_s=1e-3, resident=10**6):
        self.clock, self.max_jobs, self.arena, self.step_s, self.resident = clock, max_jobs, arena, step_s, resident
        self.live = {}
        self.used_arena = 0
        self.next = 0
        self.admit_order = []
        self.max_live = 0

    def need(self, r):
        return r.w * r.h * r.spp * 96

    def resident_bytes(self):
        return self.resident

    def submit(self, r):
        if len(self.live) >= self.max_jobs or self.used_arena + self.need(r) > self.arena:
            return None
        h = self.next
        self.next += 1
        self.live[h] = [r, r.spp * (r.bounces + 1)]
        self.used_arena += self.need(r)
        self.admit_order.append(r.rid)
        self.max_live = max(self.max_live, len(self.live))
        return h

    def step(self):
        act = [v for v in self.live.values() if v[1] > 0]
        if not act:
            return 0
        self.clock.t += self.step_s
        for v in act:
            v[1] -= 1
        return len(act)

    def done(self, h):
        return self.live[h][1] == 0

    def release(self, h, r):
        assert self.live[h][1] == 0
        del self.live[h]
        self.used_arena -= self.need(r)
        return r.w * r.h * r.spp * r.bounces


def test_requests_are_seeded_and_follow_the_mix():
    names = ["a", "b", "c", "d"]
    r1 = serve.make_requests(20000, 50.0, names, "reuse", seed=3)
    r2 = serve.make_requests(20000, 50.0, names, "reuse", seed=3)
    assert r1 == r2
    arr = np.array([r.arrival for r in r1])
    gaps = np.diff(arr)
    assert np.all(gaps >= 0)
    # exponential gaps of mean 1/rate: mean and the coefficient of variation (1 for an exponential)
    assert abs(gaps.mean() * 50.0 - 1.0) < 0.03
    assert abs(gaps.std() / gaps.mean() - 1.0) < 0.05
    for attr, values in (("scene", names), ("spp", serve.SPPS), ("w", [w for w, _ in serve.RESOLUTIONS])):
        counts = np.array([sum(getattr(r, attr) == v for r in r1) for v in values])
        assert np.all(np.abs(counts / len(r1) - 1.0 / len(values)) < 0.02), (attr, counts)
    assert all((r.w, r.h) in serve.RESOLUTIONS for r in r1)
    assert all(r.bounces == 4 and r.mode == "reuse" for r in r1)
    assert all(r.arrival == 0.0 for r in serve.make_requests(10, None, names, "reuse", seed=1))


def test_output_bytes():
    r = serve.Request(0, 0.0, "a", 1920, 1080, 4, 4, "reuse", 1)
    assert serve.output_bytes(r) == 1920 * 1080 * 12 + 2 * 5 * 4 * 1920 * 1080 * 4


def test_single_request_latency_is_its_steps():
    clk = Clock()
    be = FakeBackend(clk, step_s=2e-3)
    r = serve.Request(0, 0.0, "a", 64, 64, 2, 3, "reuse", 1)
    st = serve.serve([r], be, 10**12, clock=clk, sleep=clk.sleep)
    rec = st.records[0]
    assert math.isclose(rec.finished - rec.arrival, 2 * 4 * 2e-3, rel_tol=1e-9)
    assert rec.rays == 64 * 64 * 2 * 3
    assert st.steps == 8


def test_continuous_batching_overlaps_and_respects_limits():
    clk = Clock()
    be = FakeBackend(clk, max_jobs=3, step_s=1e-3)
    reqs = serve.make_requests(200, 400.0, ["a"], "reuse", seed=5, resolutions=((64, 64), (32, 32)), spps=(1, 2))
    budget = be.resident + 3 * serve.output_bytes(max(reqs, key=serve.output_bytes))
    st = serve.serve(reqs, be, budget, clock=clk, sleep=clk.sleep)
    assert be.max_live == 3 and st.max_in_flight == 3          # requests overlap, never beyond the slots
    assert st.peak_budget_bytes <= budget
    assert be.admit_order == sorted(be.admit_order)           # first come, first served
    for rec, r in zip(st.records, reqs):
        assert rec.arrival <= rec.admitted <= rec.finished
        # a request needs at least its own steps once admitted
        assert rec.finished - rec.admitted >= r.spp * (r.bounces + 1) * 1e-3 - 1e-12
    s = st.summary(warmup=20)
    assert s["requests"] == 180 and s["latency_ms_p99"] >= s["latency_ms_p50"] > 0


def test_budget_admission_queues_requests():
    clk = Clock()
    be = FakeBackend(clk, max_jobs=64, step_s=1e-3)
    reqs = [serve.Request(i, 0.0, "a", 64, 64, 1, 1, "reuse", i) for i in range(10)]
    one = serve.output_bytes(reqs[0])
    st = serve.serve(reqs, be, be.resident + 2 * one, clock=clk, sleep=clk.sleep)
    assert be.max_live == 2 and st.refused_admissions > 0
    fin = sorted(rec.finished for rec in st.records)
    # two at a time, two steps each
    assert math.isclose(fin[-1], 5 * 2 * 1e-3, rel_tol=1e-9)


def test_arena_admission_and_impossible_requests():
    clk = Clock()
    be = FakeBackend(clk, max_jobs=8, arena=64 * 64 * 96 * 2)
    reqs = [serve.Request(i, 0.001 * i, "a", 64, 64, 1, 2, "reuse", i) for i in range(6)]
    st = serve.serve(reqs, be, 10**12, clock=clk, sleep=clk.sleep)
    assert be.max_live == 2 and len(st.records) == 6
    with pytest.raises(ValueError):
        serve.serve([serve.Request(0, 0.0, "a", 1920, 1080, 4, 4, "reuse", 1)], FakeBackend(clk), 10**6 + 1000,
                    clock=clk, sleep=clk.sleep)
    with pytest.raises(RuntimeError):
        serve.serve([serve.Request(0, 0.0, "a", 256, 256, 1, 1, "reuse", 1)], FakeBackend(clk, arena=1000), 10**12,
                    clock=clk, sleep=clk.sleep)


def test_idle_gaps_wait_for_arrivals():
    clk = Clock()
    be = FakeBackend(clk, step_s=1e-3)
    reqs = [serve.Request(0, 0.0, "a", 8, 8, 1, 1, "reuse", 1), serve.Request(1, 5.0, "a", 8, 8, 1, 1, "reuse", 2)]
    st = serve.serve(reqs, be, 10**12, clock=clk, sleep=clk.sleep)
    assert st.records[1].admitted >= 5.0
    assert math.isclose(st.records[1].finished - st.records[1].arrival, 2e-3, abs_tol=2e-3)


def test_coordinate_descent_finds_separable_minimum():
    space = [("a", (1, 2, 3, 4)), ("b", (10, 20, 30))]
    calls = []

    def cost(p):
        calls.append(dict(p))
        return (p["a"] - 3) ** 2 + (p["b"] - 20) ** 2

    best, c, log = autotune.coordinate_descent(cost, space, dict(a=1, b=10))
    assert best == dict(a=3, b=20) and c == 0
    assert len(log) == len(calls) == 1 + 3 + 2


def test_group_bound_and_search_space():
    assert autotune.group_allowed((8, 8), 8) and not autotune.group_allowed((8, 8), 16)
    assert autotune.group_allowed((4, 4), 2) and not autotune.group_allowed((4, 4), 4)
    assert not autotune.group_allowed((8, 8), 3)
    dims = dict(autotune.search_space("reuse"))
    assert all(autotune.group_allowed(*g) for g in dims["group"])
    assert autotune.DEFAULT["group"] in dims["group"]
    assert "group" not in dict(autotune.search_space("incoherent"))


def test_coordinate_descent_never_repeats_a_point():
    space = [("a", (1, 2, 3)), ("b", (1, 2))]
    seen = []

    def cost(p):
        key = (p["a"], p["b"])
        assert key not in seen
        seen.append(key)
        return -p["a"] * 10 - p["b"]           # the best moves away from the start at once

    best, c, log = autotune.coordinate_descent(cost, space, dict(a=2, b=1))
    assert best == dict(a=3, b=2) and len(log) == 1 + 2 + 1
