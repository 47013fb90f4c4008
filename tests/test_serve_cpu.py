"""The serving scheduler on the CPU, with a stand-in runner: requests are
admitted first in, first out; the device memory of the requests in flight
never exceeds the budget (a request larger than the budget runs alone);
results and errors reach their own futures; queued requests can be
cancelled."""
import threading
import time

import math

import pytest

from paper_1801_10187_amd import binding
from paper_1801_10187_amd.binding import FP32, FP64
from paper_1801_10187_amd.serve import Request, Server, footprint


class Recorder:
    def __init__(self):
        self.lock = threading.Lock()
        self.inflight = 0
        self.max_inflight = 0

    def __call__(self, req):
        with self.lock:
            self.inflight += 1
            self.max_inflight = max(self.max_inflight, self.inflight)
        time.sleep(0.01 * (1 + req.steps % 3))
        with self.lock:
            self.inflight -= 1
        if req.steps == 13:
            raise ValueError("request 13 fails")
        return ("result", req.steps)


def _req(i, n):
    return Request((4, 4, 4), n, i, make=None)


def test_footprint_grows_with_the_box():
    assert footprint(10**6, (100, 100, 100)) > footprint(10**5, (100, 100, 100))
    assert footprint(10**6, (100, 100, 100)) > footprint(10**6, (10, 10, 10))
    assert footprint(10**6, (50, 50, 50), precision=FP64) > footprint(10**6, (50, 50, 50))


def test_footprint_follows_the_slab_rule():
    """10^6 particles in 50^3 cells (density 8: 4 x 4 x 4 tiles, 13^3 of
    them, those at the far faces cut to 2 cells along the axis): slabs sized
    for a whole tile's mean occupancy (512) plus five standard deviations,
    +20 % (at least the mean over all tiles + 8 sigma + 64), rounded up to
    32; two slab buffers of 32 (FP32) or 52 (FP64) bytes per slot; at the
    peak the 48-byte-per-particle upload buffer beside them. The rest
    (counters and tables, a few hundred kB here) within 2 MB."""
    n, nt = 10**6, 13 ** 3
    mean = n / nt
    mx = math.ceil(512 + 5 * math.sqrt(512))
    cap = -(-max(mx + mx // 5, int(mean + 8 * math.sqrt(mean) + 64)) // 32) * 32
    for prec, rec in ((FP32, 32), (FP64, 52)):
        peak, held = binding.footprint((50, 50, 50), n, nsteps=10, precision=prec)
        slabs = 2 * rec * nt * cap
        assert slabs < held < slabs + 2e6
        assert slabs + 48 * n < peak < slabs + 48 * n + 2e6
        assert footprint(n, (50, 50, 50), prec) == peak


def test_fifo_budget_results_and_errors():
    rec = Recorder()
    sizes = [2000, 500, 30000, 100, 100, 4000, 100, 100, 100, 100, 100, 100, 100, 100, 800]
    reqs = [_req(i, n) for i, n in enumerate(sizes)]
    budget = reqs[0].bytes + reqs[1].bytes + reqs[3].bytes   # request 2 exceeds it alone
    with Server(workers=4, memory_budget=budget, runner=rec) as srv:
        futs = [srv.submit(r) for r in reqs]
    for i, f in enumerate(futs):
        if i == 13:
            with pytest.raises(ValueError):
                f.result()
        else:
            assert f.result() == ("result", i)
    assert [r.steps for r in srv.admitted] == list(range(len(reqs)))
    big = reqs[2].bytes
    assert srv.max_inflight_bytes <= max(budget, big)
    assert srv.max_inflight <= 4 and rec.max_inflight <= 4


def test_queued_requests_can_be_cancelled():
    gate = threading.Event()

    def runner(req):
        gate.wait(5)
        return req.steps

    srv = Server(workers=1, memory_budget=1 << 40, runner=runner)
    first = srv.submit(_req(1, 10))
    queued = [srv.submit(_req(2 + i, 10)) for i in range(3)]
    time.sleep(0.05)
    assert all(f.cancel() for f in queued)
    gate.set()
    srv.close()
    assert first.result() == 1
    assert all(f.cancelled() for f in queued)
