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
