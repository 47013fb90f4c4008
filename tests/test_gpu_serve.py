"""Serving on the GPU: requests of different sizes, thermostat settings and
step counts run concurrently through the server (several in flight, each in
its own context and stream), and every result equals the same request run
alone, bit for bit; a tight memory budget serialises the largest ones and
changes nothing."""
import numpy as np
import pytest

import paper_1801_10187_amd as m
import workloads
from helpers import banner
from paper_1801_10187_amd.serve import Request, Server, run_request

pytestmark = pytest.mark.gpu


def _requests():
    rng = np.random.default_rng(90)
    out = []
    for i in range(12):
        n = int(rng.integers(5, 15))
        rho = float(rng.uniform(4.0, 10.0))
        kT = float(rng.uniform(0.5, 2.0))
        seed = 100 + i
        npart = int(round(rho * n ** 3))

        def make(n=n, rho=rho, kT=kT, seed=seed):
            return workloads.fluid((n, n, n), rho, kT=kT, seed=seed)
        prec = m.FP64 if i % 3 == 0 else m.FP32
        out.append(Request((n, n, n), npart, int(rng.integers(5, 40)), make, precision=prec,
                           kT=kT, seed=seed, thermostat=bool(i % 2)))
    return out


@pytest.mark.parametrize("budget", ["device", "tight"])
def test_results_alone_and_in_the_mix(budget):
    banner(f"serving mix, budget {budget}")
    reqs = _requests()
    alone = [run_request(r) for r in reqs]
    limit = None if budget == "device" else 2 * max(r.bytes for r in reqs)
    with Server(workers=4, memory_budget=limit) as srv:
        futs = [srv.submit(r) for r in reqs]
        got = [f.result(timeout=120) for f in futs]
    assert srv.max_inflight > 1
    if limit is not None:
        assert srv.max_inflight_bytes <= limit
    for (u0, m0), (u1, m1) in zip(alone, got):
        assert np.array_equal(m0, m1)
        assert np.array_equal(u0, u1)
