"""Serving scheduler on the host (no GPU): HBM-budget admission, failure
handling, continuous batching and retirement of replaced factors.

A host-only engine stands in for the device: builds sleep, deblurs finish after
a fixed delay, and the engine keeps its own count of live workspace bytes
(taken when a build starts, given back when a survey is freed or a build
fails), which must never exceed the budget.
"""
import threading
import time

import pytest

from paper_2512_16642_amd import serve


class HostEngine:
    def __init__(self, sizes, build_s, fail_keys=(), deblur_s=0.002, max_batch_sources=64):
        self.sizes = dict(sizes)
        self.build_s = dict(build_s)
        self.fail_keys = set(fail_keys)
        self.deblur_s = deblur_s
        self.max_batch_sources = max_batch_sources
        self.live = 0
        self.max_live = 0
        self.lock = threading.Lock()
        self.n = 0
        self.batches = []           # (handle, [rids])
        self.freed = {}             # handle -> time freed
        self.deblur_end = {}        # handle -> last deblur completion time
        self.slots_in_use = set()
        self.max_slots = 0

    def workspace_bytes(self, key):
        return self.sizes[key]

    def build(self, key, slot):
        with self.lock:
            assert slot not in self.slots_in_use
            self.slots_in_use.add(slot)
            self.max_slots = max(self.max_slots, len(self.slots_in_use))
            self.live += self.sizes[key]
            self.max_live = max(self.max_live, self.live)
            self.n += 1
            h = (key, self.n)
        time.sleep(self.build_s[key])
        with self.lock:
            self.slots_in_use.discard(slot)
            if key in self.fail_keys:
                self.live -= self.sizes[key]
                raise RuntimeError("non-positive pivot")
        return h

    def deblur(self, h, reqs):
        assert sum(r.ns for r in reqs) <= self.max_batch_sources
        self.batches.append((h, [r.rid for r in reqs]))
        end = time.perf_counter() + self.deblur_s
        self.deblur_end[h] = max(self.deblur_end.get(h, 0.0), end)
        return (end, h, reqs)

    def ready(self, t):
        return time.perf_counter() >= t[0]

    def result(self, t, i):
        return (t[1], t[2][i].rid)

    def free(self, h):
        assert h not in self.freed
        self.freed[h] = time.perf_counter()
        with self.lock:
            self.live -= self.sizes[h[0]]


def test_admission_never_exceeds_budget():
    sizes = {0: 40, 1: 30, 2: 50, 3: 20}
    eng = HostEngine(sizes, {k: 0.01 + 0.004 * k for k in sizes})
    budget = 100
    srv = serve.Server(eng, budget_bytes=budget, build_slots=3, tick_s=1e-4)
    reqs = [serve.Request(i, "build", 0.001 * i, i % 4) for i in range(24)]
    srv.run(reqs)
    assert all(r.status == "done" for r in reqs)
    assert eng.max_live <= budget
    assert srv.adm.peak <= budget
    assert max(u for _, u in srv.trace) <= budget
    assert eng.max_slots <= 3
    # the four surveys need 140 > 100 bytes: least recently used factors were evicted
    assert srv.evictions > 0
    assert srv.adm.used == sum(sizes[k] for k in srv.resident) == eng.live
    srv.close()
    assert srv.adm.used == 0 and eng.live == 0


def test_budget_binds_builds_wait():
    # two 60-byte builds under a 100-byte budget cannot overlap although slots are free
    eng = HostEngine({0: 60, 1: 60}, {0: 0.03, 1: 0.03})
    srv = serve.Server(eng, budget_bytes=100, build_slots=2, tick_s=1e-4)
    reqs = [serve.Request(0, "build", 0.0, 0), serve.Request(1, "build", 0.0, 1)]
    srv.run(reqs)
    assert eng.max_live == 60
    # survey 0 is resident after the first build: the second waits, then evicts it
    assert reqs[1].t_done - reqs[0].t_done >= 0.025
    assert set(srv.resident) == {1} and srv.evictions == 1
    srv.close()


def test_oversized_build_rejected():
    eng = HostEngine({0: 10, 1: 500}, {0: 0.001, 1: 0.001})
    srv = serve.Server(eng, budget_bytes=100, build_slots=2, tick_s=1e-4)
    reqs = [serve.Request(0, "build", 0.0, 1), serve.Request(1, "build", 0.0, 0)]
    srv.run(reqs)
    assert reqs[0].status == "rejected" and reqs[1].status == "done"
    srv.close()


def test_failed_build_releases_budget_and_rejects_its_deblurs():
    eng = HostEngine({0: 40, 1: 40}, {0: 0.005, 1: 0.01}, fail_keys={1})
    srv = serve.Server(eng, budget_bytes=100, build_slots=2, tick_s=1e-4)
    srv.preload([0])
    reqs = [serve.Request(0, "build", 0.0, 1),
            serve.Request(1, "deblur", 0.001, 1, ns=4),       # waits for the build, then rejected
            serve.Request(2, "deblur", 0.002, 0, ns=4),
            serve.Request(3, "deblur", 0.05, 1, ns=4)]        # key 1 neither resident nor building
    srv.run(reqs)
    assert reqs[0].status == "failed"
    assert reqs[1].status == "rejected" and reqs[3].status == "rejected"
    assert reqs[2].status == "done"
    assert srv.adm.used == 40 == eng.live
    srv.close()


def test_deblurs_are_merged_and_mapped_back():
    eng = HostEngine({0: 10, 1: 10}, {0: 0.001, 1: 0.001}, deblur_s=0.01, max_batch_sources=64)
    srv = serve.Server(eng, budget_bytes=100, build_slots=1, keep_results=True, tick_s=1e-4)
    srv.preload([0, 1])
    reqs = [serve.Request(i, "deblur", 0.0, i % 2, ns=1 + (7 * i) % 30) for i in range(12)]
    srv.run(reqs)
    assert all(r.status == "done" for r in reqs)
    # merged: fewer launches than requests, each within the cap, each request exactly once
    assert len(eng.batches) < len(reqs)
    seen = sorted(rid for _, rids in eng.batches for rid in rids)
    assert seen == list(range(12))
    for r in reqs:
        h, rid = srv.results[r.rid]
        assert rid == r.rid and h[0] == r.key
    srv.close()


def test_replaced_factors_retire_after_their_deblurs():
    eng = HostEngine({0: 30}, {0: 0.005}, deblur_s=0.05)
    srv = serve.Server(eng, budget_bytes=100, build_slots=1, tick_s=1e-4)
    srv.preload([0])
    first = srv.resident[0].handle
    reqs = [serve.Request(0, "deblur", 0.0, 0, ns=8), serve.Request(1, "build", 0.001, 0)]
    srv.run(reqs)
    assert srv.resident[0].handle != first
    assert eng.freed[first] >= eng.deblur_end[first]
    assert srv.adm.peak == 60 and srv.adm.used == 30
    srv.close()


def test_poisson_requests_reproducible():
    a = serve.poisson_requests(5.0, 20.0, 0.02, 8, seed=2400)
    b = serve.poisson_requests(5.0, 20.0, 0.02, 8, seed=2400)
    assert [(r.kind, r.arrival, r.key, r.ns, r.seed) for r in a] == \
           [(r.kind, r.arrival, r.key, r.ns, r.seed) for r in b]
    assert 60 <= len(a) <= 140
    assert all(1 <= r.ns <= 256 for r in a if r.kind == "deblur")
    assert all(0.0 < r.arrival < 5.0 for r in a)


@pytest.mark.parametrize("cap", [16, 64])
def test_request_above_batch_cap_rejected(cap):
    eng = HostEngine({0: 10}, {0: 0.001}, max_batch_sources=cap)
    srv = serve.Server(eng, budget_bytes=100, build_slots=1, tick_s=1e-4)
    srv.preload([0])
    reqs = [serve.Request(0, "deblur", 0.0, 0, ns=cap + 1), serve.Request(1, "deblur", 0.0, 0, ns=cap)]
    srv.run(reqs)
    assert reqs[0].status == "rejected" and reqs[1].status == "done"
    srv.close()
