"""Serving on the GPU: requests of different sizes, thermostat settings and
step counts run concurrently through the server (several in flight, each in
its own context and stream), and every result equals the same request run
alone, bit for bit; a tight memory budget serialises the largest ones and
changes nothing."""
import numpy as np
import pytest

import paper_1801_10187_amd as m
import workloads
from helpers import PoolHighWater, banner
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
    hw = PoolHighWater()
    assert hw.current() == 0
    hw.reset()
    with Server(workers=4, memory_budget=limit) as srv:
        futs = [srv.submit(r) for r in reqs]
        got = [f.result(timeout=120) for f in futs]
    print(f"requests in flight at most {srv.max_inflight}, admitted bytes at most "
          f"{srv.max_inflight_bytes}, pool high-water {hw.high()}")
    assert srv.max_inflight > 1
    # the device memory the requests held together never exceeded what the
    # server admitted them for
    assert hw.high() <= srv.max_inflight_bytes
    if limit is not None:
        assert srv.max_inflight_bytes <= limit
    for (u0, m0), (u1, m1) in zip(alone, got):
        assert np.array_equal(m0, m1)
        assert np.array_equal(u0, u1)


@pytest.mark.parametrize("case", [((12, 12, 12), 8.0, m.FP32, False),
                                  ((50, 50, 50), 8.0, m.FP32, True),
                                  ((30, 30, 30), 10.0, m.FP64, True),
                                  ((40, 40, 40), 2.5, m.FP64, False)])
def test_footprint_bounds_the_pool(case):
    """One request run alone (create from host arrays, steps, velocity
    field, destroy): the stream-ordered pool's high-water mark stays within
    the request's footprint, and for boxes of 10^5 particles and more above
    85 % of it (the estimate is not loose)."""
    n_cells, rho, prec, thermo = case
    banner(f"footprint {n_cells} rho {rho} {'fp64' if prec == m.FP64 else 'fp32'}")
    npart = int(round(rho * np.prod(n_cells)))
    req = Request(n_cells, npart, 25, lambda: workloads.fluid(n_cells, rho, seed=7),
                  precision=prec, seed=8, thermostat=thermo)
    hw = PoolHighWater()
    assert hw.current() == 0
    hw.reset()
    run_request(req)
    used = hw.high()
    print(f"{npart} particles: pool high-water {used} B, footprint {req.bytes} B "
          f"({used / req.bytes:.3f})")
    assert hw.current() == 0
    assert used <= req.bytes
    if npart >= 100_000:
        assert used > 0.85 * req.bytes


def test_serving_stream_full_range():
    """Requests of the served stream itself, from the smallest (~9 x 10^3
    particles) to the two largest (~10^7), with their own step counts (130 to
    1226), FP32 and thermostatted as served: run in the mix they equal the
    same requests run alone, bit for bit; every field holds each particle
    once and the zero net momentum the request started with, up to the FP32
    rounding of the stored velocities (a random walk of ~2^-24 per component
    per particle and step)."""
    banner("serving stream, full size range")
    cfg = workloads.CONFIGS["srd_serve_poisson50"]
    stream = workloads.serve_requests(rate=cfg["rate"], duration=cfg["duration"], seed=cfg["seed"])
    N = np.array([int(round(r["density"] * np.prod(r["n_cells"]))) for r in stream])
    order = np.argsort(N, kind="stable")
    pick = sorted({int(order[int(f * (len(order) - 1))]) for f in (0.0, 0.2, 0.4, 0.6, 0.8, 0.95)}
                  | {int(order[-1]), int(order[-2])})
    reqs = []
    for i in pick:
        r = stream[i]

        def make(r=r, i=i):
            return workloads.fluid(r["n_cells"], r["density"], kT=cfg["kT"], seed=5000 + i)
        reqs.append(Request(r["n_cells"], int(N[i]), r["steps"], make, precision=m.FP32,
                            kT=cfg["kT"], seed=r["seed"], thermostat=cfg["thermostat"]))
    assert max(q.n_particles for q in reqs) > 9_000_000 and min(q.n_particles for q in reqs) < 10_000
    alone = [run_request(q) for q in reqs]
    with Server(workers=8) as srv:
        futs = [srv.submit(q) for q in reqs]
        got = [f.result(timeout=200) for f in futs]
    assert srv.max_inflight > 1
    for q, (u0, m0), (u1, m1) in zip(reqs, alone, got):
        assert np.array_equal(m0, m1) and np.array_equal(u0, u1)
        assert m0.sum() == q.n_particles
        P = (u0 * m0[:, None]).sum(axis=0)
        assert np.abs(P).max() < 1e-6 * np.sqrt(q.steps * q.n_particles)
