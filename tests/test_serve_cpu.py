"""Scheduler logic of the render server, driven by a sleep-based fake executor (no GPU):
admission against the memory budget, continuous batching, overlap across slots, failure
isolation and memory release."""
import threading
import time

import numpy as np
import pytest

from paper_2605_31419_amd import scenes as S
from paper_2605_31419_amd.serve import FakeExecutor, Request, Server, run_poisson

POSE = np.zeros(12, np.float32)


def _req(i, w=320, h=240):
    return Request(i, S.intrinsics_for(w, h), POSE)


def test_all_requests_complete_with_stats():
    ex = FakeExecutor(per_pixel_s=2e-9)
    srv = Server(ex, n_slots=2, mem_budget=1 << 30)
    srv.start()
    try:
        qs = S.serving_queries(1, 60, qps=2000.0)
        st = run_poisson(srv, qs)
    finally:
        srv.stop()
    assert st["completed"] == 60 and st["errors"] == 0
    assert 0 < st["p50_ms"] <= st["p99_ms"]
    assert srv.used == 0
    assert sum(len(b) for b in ex.batches) == 60


def test_memory_budget_is_never_exceeded():
    ex = FakeExecutor(per_pixel_s=1e-8)
    one = 20 * 640 * 480
    srv = Server(ex, n_slots=4, mem_budget=one)          # room for one 640x480 query at a time
    srv.start()
    try:
        for i in range(12):
            srv.submit(_req(i, 640, 480))
        srv.drain()
    finally:
        srv.stop()
    assert srv.peak_used <= one
    assert ex.max_active == 1
    assert len(srv.completed) == 12 and srv.used == 0


def test_continuous_batching_overlaps_and_batches():
    ex = FakeExecutor(per_pixel_s=5e-8)
    srv = Server(ex, n_slots=3, mem_budget=1 << 30, max_batch_views=4)
    srv.start()
    try:
        for i in range(40):
            srv.submit(_req(i))
        srv.drain()
    finally:
        srv.stop()
    assert ex.max_active >= 2                              # batches ran concurrently
    assert max(len(b) for b in ex.batches) > 1             # arrivals during a run were batched
    assert max(len(b) for b in ex.batches) <= 4
    assert sorted(r for b in ex.batches for r in b) == list(range(40))


def test_requests_arriving_during_a_run_are_admitted_as_memory_frees():
    ex = FakeExecutor(per_pixel_s=2e-7)                    # 320x240: ~15 ms per request
    per = 20 * 320 * 240
    srv = Server(ex, n_slots=2, mem_budget=2 * per, max_batch_views=1)
    srv.start()
    try:
        first = [srv.submit(_req(i)) for i in range(2)]
        time.sleep(0.003)
        later = [srv.submit(_req(10 + i)) for i in range(3)]
        assert all(r.admitted == 0.0 for r in later)       # no memory left yet
        srv.drain()
    finally:
        srv.stop()
    assert all(r.admitted >= min(f.done for f in first) for r in later)
    assert srv.peak_used <= 2 * per


def test_failures_are_isolated_and_release_memory():
    ex = FakeExecutor(per_pixel_s=1e-9, fail_ids=[3, 7])
    srv = Server(ex, n_slots=2, mem_budget=1 << 30, max_batch_views=1)
    srv.start()
    try:
        for i in range(10):
            srv.submit(_req(i))
        srv.drain()
    finally:
        srv.stop()
    errs = sorted(r.rid for r in srv.completed if r.error)
    assert errs == [3, 7]
    assert srv.used == 0


class _Raising(FakeExecutor):
    def run(self, slot, batch):
        if any(r.rid == 5 for r in batch):
            raise RuntimeError("device lost")
        super().run(slot, batch)


def test_executor_exception_fails_only_its_batch():
    ex = _Raising(per_pixel_s=1e-9)
    srv = Server(ex, n_slots=1, mem_budget=1 << 30, max_batch_views=1)
    srv.start()
    try:
        for i in range(8):
            srv.submit(_req(i))
        srv.drain()
    finally:
        srv.stop()
    bad = [r for r in srv.completed if r.error]
    assert [r.rid for r in bad] == [5] and "device lost" in bad[0].error
    assert srv.used == 0


def test_oversized_request_is_rejected_immediately():
    ex = FakeExecutor()
    srv = Server(ex, n_slots=1, mem_budget=1000)
    srv.start()
    try:
        r = srv.submit(_req(0))
        assert r.event.is_set() and "budget" in r.error
    finally:
        srv.stop()


class _Slots(FakeExecutor):
    """Fake executor whose slots hold `ws` bytes each and fit at most `views` views."""

    def __init__(self, ws, views, **kw):
        super().__init__(**kw)
        self.ws, self.views = ws, views

    def setup(self, n_slots, budget, max_views, max_pixels):
        return n_slots * self.ws, min(max_views, self.views)

    def batch_fits(self, intrs):
        return len(intrs) <= self.views


def test_slot_workspaces_are_charged_for_the_servers_lifetime():
    per = 20 * 320 * 240
    ex = _Slots(ws=10 * per, views=2, per_pixel_s=1e-8)
    srv = Server(ex, n_slots=2, mem_budget=22 * per, max_batch_views=8)
    srv.start()
    try:
        assert srv.used == 20 * per and srv.max_views == 2
        reqs = [srv.submit(_req(i)) for i in range(10)]
        big = srv.submit(_req(99, 640, 480))              # 4 per: above the 2 per left
        srv.drain()
        assert srv.used == 20 * per
    finally:
        srv.stop()
    assert srv.used == 0
    assert big.error and "slots hold" in big.error
    assert all(r.error is None for r in reqs)
    assert srv.peak_used <= 22 * per
    assert max(len(b) for b in ex.batches) <= 2


def test_concurrent_submitters_keep_the_books():
    """Race check of the scheduler (a stand-in for a thread sanitizer, which does not apply to
    Python code): 8 submitting threads, 4 slots, random service times.  Every request
    completes exactly once, the charged memory stays within [0, budget] at every batch, and
    the books balance at the end."""
    import random

    per = 20 * 320 * 240
    budget = 6 * per
    seen = []

    class Checking(FakeExecutor):
        def run(self, slot, batch):
            with srv.cv:
                seen.append(srv.used)
                assert 0 <= srv.used <= budget
            time.sleep(random.uniform(0, 2e-3))
            super().run(slot, batch)

    ex = Checking(per_pixel_s=1e-9)
    srv = Server(ex, n_slots=4, mem_budget=budget, max_batch_views=3)
    srv.start()
    out = []
    lock = threading.Lock()

    def submitter(k):
        for i in range(50):
            r = srv.submit(_req(1000 * k + i))
            with lock:
                out.append(r)
            time.sleep(random.uniform(0, 1e-4))

    try:
        ts = [threading.Thread(target=submitter, args=(k,)) for k in range(8)]
        for t in ts:
            t.start()
        for t in ts:
            t.join()
        srv.drain()
    finally:
        srv.stop()
    assert len(out) == 400 and all(r.event.is_set() and r.error is None for r in out)
    ids = [r.rid for r in srv.completed]
    assert len(ids) == len(set(ids)) == 400
    assert srv.used == 0 and srv.peak_used <= budget and max(seen) <= budget
    assert sorted(r for b in ex.batches for r in b) == sorted(ids)
