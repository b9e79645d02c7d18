"""Serving scheduler on the CPU: the real admission / arena / batching logic
driven by a fake executor whose batches complete after a programmed delay."""
import ctypes
import os
import time

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2012_13257_amd", "libgmmsched_test.so")

OK, EINVAL, ENOMEM, EAGAIN, EHIP, ENOTFOUND = 0, -1, -2, -3, -4, -5
QUEUED, RUNNING, DONE, FAILED = 0, 1, 2, 3


class Status(ctypes.Structure):
    _fields_ = [("state", ctypes.c_int32), ("err", ctypes.c_int32), ("t_submit_ns", ctypes.c_int64),
                ("t_admit_ns", ctypes.c_int64), ("t_done_ns", ctypes.c_int64)]


@pytest.fixture(scope="module")
def L():
    if not os.path.exists(LIB):
        from paper_2012_13257_amd.build import build_sched_test
        build_sched_test()
    lib = ctypes.CDLL(LIB)
    lib.gmm_fake_create.restype = ctypes.c_void_p
    lib.gmm_fake_create.argtypes = [ctypes.c_uint64, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                    ctypes.c_int]
    lib.gmm_fake_submit.argtypes = [ctypes.c_void_p, ctypes.c_uint64, ctypes.c_int64, ctypes.c_int,
                                    ctypes.POINTER(ctypes.c_uint64)]
    lib.gmm_fake_submit_many.argtypes = [ctypes.c_void_p, ctypes.POINTER(ctypes.c_uint64), ctypes.c_int,
                                         ctypes.c_int64, ctypes.c_int, ctypes.POINTER(ctypes.c_uint64),
                                         ctypes.POINTER(ctypes.c_int)]
    lib.gmm_fake_poll.argtypes = [ctypes.c_void_p, ctypes.c_uint64, ctypes.POINTER(Status)]
    lib.gmm_fake_drain.argtypes = [ctypes.c_void_p, ctypes.c_int64]
    lib.gmm_fake_stats.argtypes = [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int64)]
    lib.gmm_fake_destroy.argtypes = [ctypes.c_void_p]
    lib.gmm_fake_shutdown.argtypes = [ctypes.c_void_p]
    lib.gmm_arena_selftest.argtypes = [ctypes.c_uint64, ctypes.c_int, ctypes.POINTER(ctypes.c_int64),
                                       ctypes.POINTER(ctypes.c_int)]
    return lib


class Fake:
    def __init__(self, L, budget, slots, queue=1000, contexts=2, max_batch=8):
        self.L = L
        self.h = L.gmm_fake_create(budget, slots, queue, contexts, max_batch)

    def submit(self, nbytes, delay_us=0, fail=0):
        t = ctypes.c_uint64()
        rc = self.L.gmm_fake_submit(self.h, nbytes, delay_us, fail, ctypes.byref(t))
        return rc, t.value

    def submit_many(self, sizes, delay_us=0, fail=0):
        n = len(sizes)
        b = (ctypes.c_uint64 * max(n, 1))(*sizes)
        t = (ctypes.c_uint64 * max(n, 1))()
        acc = ctypes.c_int(-1)
        rc = self.L.gmm_fake_submit_many(self.h, b, n, delay_us, fail, t, ctypes.byref(acc))
        return rc, list(t)[:acc.value]

    def poll(self, t):
        s = Status()
        rc = self.L.gmm_fake_poll(self.h, t, ctypes.byref(s))
        return rc, s

    def stats(self):
        a = (ctypes.c_int64 * 6)()
        self.L.gmm_fake_stats(self.h, a)
        return dict(zip(["peak_arena", "peak_slots", "batches", "peak_ctx", "overlaps",
                         "max_batch"], list(a)))

    def drain(self, ms=-1):
        return self.L.gmm_fake_drain(self.h, ms)

    def close(self):
        if self.h:
            self.L.gmm_fake_destroy(self.h)
            self.h = None


def test_arena_first_fit_and_coalescing(L):
    rng = np.random.default_rng(0)
    for trial in range(20):
        n = 40
        sizes = rng.integers(1, 100000, n).astype(np.int64)
        size = int(sum((s + 255) // 256 * 256 for s in sizes)) + 256 * int(rng.integers(0, 10))
        order = rng.permutation(n).astype(np.int32)
        rc = L.gmm_arena_selftest(size, n, sizes.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                  order.ctypes.data_as(ctypes.POINTER(ctypes.c_int)))
        assert rc == 1, (trial, rc)


def test_lifecycle_and_unknown_ticket(L):
    f = Fake(L, budget=1 << 20, slots=4)
    try:
        rc, t = f.submit(1000, delay_us=2000)
        assert rc == OK and t > 0
        rc, s = f.poll(t)
        assert rc == OK and s.state in (QUEUED, RUNNING)
        assert f.drain(5000) == OK
        rc, s = f.poll(t)
        assert rc == OK and s.state == DONE and s.err == OK
        assert s.t_submit_ns <= s.t_admit_ns <= s.t_done_ns
        assert s.t_done_ns - s.t_admit_ns >= 2_000_000 * 0.9
        # a finished ticket is forgotten after it was reported
        assert f.poll(t)[0] == ENOTFOUND
        assert f.poll(987654)[0] == ENOTFOUND
    finally:
        f.close()


def test_budget_and_queue_limits(L):
    f = Fake(L, budget=1 << 16, slots=2, queue=3)
    try:
        assert f.submit((1 << 16) + 1)[0] == ENOMEM          # can never fit
        tickets = [f.submit(1000, delay_us=20000)[1] for _ in range(2)]  # admitted
        time.sleep(0.005)
        q = [f.submit(1000, delay_us=1000) for _ in range(3)]
        assert all(rc == OK for rc, _ in q)
        assert f.submit(1000)[0] == EAGAIN                   # queue full
        assert f.drain(10000) == OK
        for t in tickets + [t for _, t in q]:
            assert f.poll(t)[1].state == DONE
        st = f.stats()
        assert st["peak_slots"] <= 2
        assert st["overlaps"] == 0
    finally:
        f.close()


def test_admission_never_exceeds_budget_or_slots_and_batches_overlap(L):
    rng = np.random.default_rng(1)
    budget = 10_000_000
    f = Fake(L, budget=budget, slots=6, queue=10000, contexts=3, max_batch=4)
    try:
        tickets = []
        for i in range(300):
            nbytes = int(rng.integers(1000, 3_000_000))
            rc, t = f.submit(nbytes, delay_us=int(rng.integers(100, 2000)))
            assert rc == OK
            tickets.append(t)
            if i % 7 == 0:
                time.sleep(0.0005)
        assert f.drain(60000) == OK
        for t in tickets:
            rc, s = f.poll(t)
            assert rc == OK and s.state == DONE
        st = f.stats()
        assert st["peak_arena"] <= budget
        assert st["peak_slots"] <= 6
        assert st["overlaps"] == 0
        assert st["max_batch"] <= 4
        assert st["peak_ctx"] >= 2          # batches ran concurrently
        assert st["batches"] >= 300 / 4
    finally:
        f.close()


def test_fifo_admission_order(L):
    f = Fake(L, budget=1 << 20, slots=1, queue=100, contexts=1, max_batch=1)
    try:
        ts = [f.submit(1000, delay_us=500)[1] for _ in range(10)]
        assert f.drain(10000) == OK
        admits = [f.poll(t)[1].t_admit_ns for t in ts]
        assert admits == sorted(admits)
    finally:
        f.close()


def test_failed_batch_reports_failed(L):
    f = Fake(L, budget=1 << 20, slots=8, contexts=1, max_batch=8)
    try:
        rc, t1 = f.submit(1000, delay_us=200, fail=1)
        assert rc == OK
        assert f.drain(5000) == OK
        rc, s = f.poll(t1)
        assert s.state == FAILED and s.err == EHIP
        # the server keeps serving after a failed batch
        rc, t2 = f.submit(1000, delay_us=100)
        assert f.drain(5000) == OK
        assert f.poll(t2)[1].state == DONE
    finally:
        f.close()


def test_destroy_with_pending_fails_queued_and_finishes_running(L):
    f = Fake(L, budget=1 << 20, slots=1, queue=100, contexts=1, max_batch=1)
    try:
        ts = [f.submit(1000, delay_us=50000)[1] for _ in range(5)]
        time.sleep(0.01)
        L.gmm_fake_shutdown(f.h)        # returns after the running batch finished
        states = [f.poll(t)[1] for t in ts]
        assert states[0].state == DONE
        assert all(s.state == FAILED and s.err == EAGAIN for s in states[1:])
        assert f.submit(1000)[0] == EAGAIN   # a stopped server takes nothing
    finally:
        f.close()


def test_submit_many_queues_in_order_and_completes(L):
    f = Fake(L, budget=1 << 20, slots=1, queue=100, contexts=1, max_batch=1)
    try:
        rc, ts = f.submit_many([1000] * 12, delay_us=300)
        assert rc == OK and len(ts) == 12
        assert ts == sorted(ts) and len(set(ts)) == 12
        assert f.drain(10000) == OK
        st = [f.poll(t)[1] for t in ts]
        assert all(s.state == DONE for s in st)
        # one submit time for the call; admission in array order
        assert len({s.t_submit_ns for s in st}) == 1
        admits = [s.t_admit_ns for s in st]
        assert admits == sorted(admits)
        assert f.submit_many([]) == (OK, [])
    finally:
        f.close()


def test_submit_many_stops_at_the_first_request_it_cannot_queue(L):
    f = Fake(L, budget=1 << 16, slots=1, queue=4, contexts=1, max_batch=1)
    try:
        # the third can never fit the budget: the first two are queued
        rc, ts = f.submit_many([1000, 1000, (1 << 16) + 1, 1000], delay_us=100)
        assert rc == ENOMEM and len(ts) == 2
        assert f.drain(10000) == OK
        assert all(f.poll(t)[1].state == DONE for t in ts)
        # queue of four: the fifth and later are refused, the rest run
        rc, ts = f.submit_many([1000] * 7, delay_us=20000)
        assert rc == EAGAIN and len(ts) == 4
        assert f.drain(20000) == OK
        assert all(f.poll(t)[1].state == DONE for t in ts)
        assert f.stats()["overlaps"] == 0
    finally:
        f.close()


def test_admitted_jobs_are_shared_among_free_contexts(L):
    """A burst queued at once runs as concurrent batches of equal size, not
    as one large batch on one context."""
    f = Fake(L, budget=1 << 24, slots=64, queue=1000, contexts=4, max_batch=64)
    try:
        rc, ts = f.submit_many([1000] * 64, delay_us=20000)
        assert rc == OK and len(ts) == 64
        assert f.drain(20000) == OK
        st = f.stats()
        assert st["peak_ctx"] == 4
        assert st["max_batch"] == 16
        assert st["batches"] == 4
    finally:
        f.close()
