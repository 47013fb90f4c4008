"""Throughput of the SRD-MPCD step on one MI355X.

    python bench.py [--steps K] [--warmup W] [--gpus 1]

Workload (default): the 100^3-cell fluid at 10 particles per cell (10^7
particles), alpha = 130 deg, dt = 0.1, kT = 1, random grid shift,
Maxwell-Boltzmann cell thermostat, synthetic positions/velocities (seed 1).
The headline value is the FP32 cell-relative form; the plain FP64 form runs on
the same input and is reported beside it, and so does the Andersen-thermostat
collision rule (eq. 4) in both forms (without the cell thermostat, which that
rule replaces). A step is one whole pass of the hot
path: stream, grid shift, binning, cell reduction, draws and rotation. The
line also carries: the same FP32 call launched as one HIP graph
(`graph_vs_stream`); the FP32 form's error and observables against the FP64
form; the copy ceiling; the latencies of the 256-box batch below
(`batch_latency`: single-step and 500-step calls, p50/p99; --no-batch leaves
it out); and the oracle's CPU baselines.

    python bench.py --workload srd_20c_rho5_fp64

times the small parity box: 20^3 cells at 5 particles per cell (40 000),
plain FP64, no thermostat, 100 steps (its state fits in cache, so the figure
is launch- and latency-bound, not a roofline number); the oracle runs all 100
steps beside it.

    python bench.py --workload srd_400c_rho5_beads

times the largest single-GPU machine instead: 400^3 cells at 5 particles per cell
(3.2 x 10^8) plus 20 000 chains of 50 mass-5 beads, FP32, no thermostat, 200
steps.

    python bench.py --workload srd_batch256_fp32

times a batch of 256 independent boxes (sides 8..64 cells, densities 5..10,
kT 0.5..2, thermostat, FP32; 1.44 x 10^8 particles in all) stepped together:
throughput over 500 steps in one call, and the latency of single batch steps
(p50/p99 over 100 calls of mpcd_step(1), each waited for).

    python bench.py --workload srd_serve_poisson50

serves an open-loop stream of requests (Poisson, 50 per second for 60 s;
10^4..10^7 particles log-uniform, 100..2000 steps, FP32, thermostat), each
returning its n^3 x 3 cell-averaged velocity field: served vs offered
throughput and request latency p50/p99.

    python bench.py --workload srd_400c_rho5_md

couples the beads of the 400^3 box to MD: per collision 50 velocity-Verlet
steps of the bead chains on the device, the beads' state handed over and
read back on device buffers (50 collisions), beside the integrator alone and
the same context stepped without the exchange.

Prints one JSON line. `roofline` is for the dominant kernel (the collide
kernel), timed with HIP events on the library's own stream during the timed
region (the first launch and then one in every PROFILE_EVERY);
`cpu_baseline` is the FP64 numpy oracle on a bounded sample.
"""
import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
WORKLOAD = "srd_100c_rho10_mbthermo"

# Particle state per storage form (bytes): FP32 home cell 4 + offsets 12 +
# velocity 12; FP64 position 24 + velocity 24.
STATE_BYTES = {"fp32": 28, "fp64": 48}

# The timed run brackets the first launch of each kernel and then one in
# every PROFILE_EVERY with HIP events: every bracket costs a few microseconds
# of stream time, so timing all launches would slow the steps it measures.
PROFILE_EVERY = 10


def floor_bytes_per_update(form, rho):
    """Algorithmic bytes of one particle-update: the state read once and
    written once, and each cell's occupancy written and read once (8 bytes
    per cell, 8 / rho per particle). The roofline's `achieved` is this times
    the particles one step launch updates, over the launch's duration."""
    return 2 * STATE_BYTES[form] + 8.0 / rho


def layout_bytes_per_particle(form):
    """Bytes the step kernel's layout moves per particle by design: state and
    its 4-byte tag read once and written once (the one-byte local cell and
    the per-tile counters on top)."""
    return 2.0 * (STATE_BYTES[form] + 4)


def roofline(form, n_particles, n_cells, avg_us, traffic=None):
    """Roofline entry of the step kernel (HBM-bound): achieved = algorithmic
    bytes of one launch (floor_bytes_per_update per particle: 2 x state per
    particle + 8 bytes per cell) / the launch's average duration; the layout's
    own figure (state and tag in and out) beside it; `traffic` the measured
    HBM bytes per launch (or None) and its ratio to the algorithmic bytes."""
    alg = 2.0 * STATE_BYTES[form] * n_particles + 8.0 * n_cells
    lay = layout_bytes_per_particle(form) * n_particles
    sec = avg_us * 1e-6
    gbs = alg / sec / 1e9
    return {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": gbs / HBM_PEAK_GBS, "traffic": traffic,
            "kernel": "k_tile (collide + stream + bin + scatter)", "kernel_avg_us": avg_us,
            "algorithmic_bytes_per_launch": alg,
            "bytes_per_update": alg / max(n_particles, 1),
            "layout_bytes_per_particle": layout_bytes_per_particle(form),
            "layout_GBs": lay / sec / 1e9,
            "traffic_over_algorithmic": None if traffic is None else traffic / alg}


def measured_traffic(form, workload=WORKLOAD):
    """HBM bytes per launch of the step kernel from the rocprofv3 FETCH_SIZE
    / WRITE_SIZE runs recorded in profiles/traffic.json, scaled by the copy
    calibration stated there; None unless they were taken on the current
    kernel sources."""
    from paper_1801_10187_amd.build import kernel_hash
    path = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        rec = json.load(open(path))
    except (OSError, ValueError):
        return None
    if rec.get("kernel_hash") != kernel_hash():
        return None
    return rec.get("bytes_per_launch", {}).get(workload, {}).get(form)


def run_form(m, inp, cfg, precision, steps, warmup, collision=0, graph=False):
    """Time `steps` steps in one call. With graph=True the call's kernels are
    launched as one HIP graph and kernel timing stays off (it would make the
    call launch on the stream); collide_ms is then 0."""
    import torch
    pos, vel, bpos, bvel, bmass = inp
    # the AT rule thermostats by itself: it runs without the cell thermostat
    thermo = cfg["thermostat"] if collision == m.SRD else False
    sim = m.Sim(pos, vel, cfg["n_cells"], kT=cfg["kT"], seed=cfg["seed"],
                precision=precision, thermostat=thermo, collision=collision,
                emb_pos=bpos, emb_vel=bvel, emb_mass=bmass)
    try:
        sim.set_graph(graph)
        sim.step(warmup)
        sim.step(steps)       # the graph of a `steps`-step call is kept for the timed call
        sim.sync()
        if not graph:
            sim.profile(True, every=PROFILE_EVERY)
            for w in (0, 1):
                sim.profile_read(w)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sim.step(steps)
        sim.sync()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        coll_ms, coll_n = sim.profile_read(0) if not graph else (0.0, 0)
        sim.profile(False)
        P, ke, kT = sim.totals()
    finally:
        sim.close()
    return dict(seconds=t1 - t0, collide_ms=coll_ms, collide_launches=coll_n,
                net_momentum=float(np.abs(P).max()), kT=kT)


def make_input(cfg, scale=None):
    """Fluid (and beads, if the workload has them) of the workload's recipe;
    `scale` shrinks the box edge to `scale` cells for a CPU sample."""
    import workloads
    n_cells = cfg["n_cells"] if scale is None else (scale, scale, scale)
    pos, vel = workloads.fluid(n_cells, cfg["density"], kT=cfg["kT"], seed=cfg["seed"])
    bpos = bvel = bmass = None
    if cfg.get("chains"):
        frac = np.prod(n_cells) / np.prod(cfg["n_cells"])
        chains = max(1, int(round(cfg["chains"] * frac)))
        bpos, bvel, bmass = workloads.beads(n_cells, chains, cfg["chain_len"], kT=cfg["kT"],
                                            mass=cfg["bead_mass"], seed=cfg["seed"] + 1)
        # solvent and beads start with zero total momentum together (sec. 4.1)
        vel, bvel = workloads.zero_net_momentum([vel, bvel], [np.ones(len(vel)), bmass])
    return pos, vel, bpos, bvel, bmass


def copy_ceiling(m, nbytes=1 << 30, reps=20):
    """Practical HBM ceiling: read + write bytes per second of a plain copy
    between two device buffers of `nbytes`, by three copies -- the library's
    grid-stride streaming kernel (one 16-byte vector per thread and
    iteration), its unrolled variant (four vectors per thread, loads before
    stores) and the runtime's device-to-device copy (hipMemcpyAsync, through
    torch's copy_). Returns the figures and their maximum, the ceiling the
    step kernel is compared with."""
    import torch
    src = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    dst = torch.empty_like(src)
    src.fill_(1)
    stream = torch.cuda.current_stream().cuda_stream
    copies = {
        "library_kernel": lambda: m.copy_kernel(src.data_ptr(), dst.data_ptr(), nbytes, stream),
        "library_kernel_unrolled": lambda: m.copy_kernel(src.data_ptr(), dst.data_ptr(), nbytes,
                                                         stream, unrolled=True),
        "hipMemcpyAsync_d2d": lambda: dst.copy_(src),
    }
    out = {}
    for name, fn in copies.items():
        for _ in range(3):
            fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        sec = e0.elapsed_time(e1) / 1e3 / reps
        out[name] = 2.0 * nbytes / sec / 1e9
    del src, dst
    out["max"] = max(out.values())
    return out


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(inp, n_cells, cfg, nsteps, what):
    """The FP64 oracle on one core (numpy limited to one thread)."""
    from threadpoolctl import threadpool_limits
    from oracle import srd
    pos, vel, bpos, bvel, bmass = inp
    p = srd.Params(n_cells, seed=cfg["seed"], thermostat=cfg["thermostat"], kT=cfg["kT"])
    mass = np.ones(pos.shape[0])
    if bpos is not None:
        pos, vel = np.concatenate([pos, bpos]), np.concatenate([vel, bvel])
        mass = np.concatenate([mass, bmass])
    with threadpool_limits(1):
        t0 = time.perf_counter()
        srd.run(pos, vel, mass, p, 0, nsteps)
        dt = time.perf_counter() - t0
    return dict(value=pos.shape[0] * nsteps / dt, unit="particle-updates/s", cores=1,
                kind="oracle",
                sample=f"{nsteps} FP64 oracle steps of {what} ({pos.shape[0]} particles, "
                       f"{dt:.1f} s, numpy, single thread)")


def _oracle_replica(job):
    """One worker of the all-core baseline: the FP64 oracle on its own box
    (numpy limited to one thread), started together with the other workers
    (barrier); returns (updates, start, end)."""
    from threadpoolctl import threadpool_limits
    import workloads
    from oracle import srd
    (n_cells, density, kT, seed, thermostat, nsteps), barrier = job
    pos, vel = workloads.fluid(n_cells, density, kT=kT, seed=1000 + seed)
    p = srd.Params(n_cells, seed=seed, thermostat=thermostat, kT=kT)
    with threadpool_limits(1):
        barrier.wait()
        t0 = time.time()
        srd.run(pos, vel, np.ones(pos.shape[0]), p, 0, nsteps)
        t1 = time.time()
    return pos.shape[0] * nsteps, t0, t1


def cpu_baseline_all_cores(jobs, what, max_workers=16):
    """The FP64 oracle on every host core: independent boxes (`jobs`) in a
    process pool of min(cores available, 16) workers, one thread each;
    value = all updates / (last end - first start)."""
    import multiprocessing
    ctx = multiprocessing.get_context("spawn")
    cores = min(len(os.sched_getaffinity(0)), max_workers, len(jobs))
    with ctx.Manager() as mgr:
        barrier = mgr.Barrier(cores)
        with ctx.Pool(cores) as pool:
            res = pool.map(_oracle_replica, [(j, barrier) for j in jobs[:cores]], chunksize=1)
    ups = sum(r[0] for r in res)
    wall = max(r[2] for r in res) - min(r[1] for r in res)
    return dict(value=ups / wall, unit="particle-updates/s", cores=cores, kind="oracle",
                cpu_model=cpu_model(),
                sample=f"{what}: {len(jobs)} independent boxes in a pool of {cores} processes "
                       f"(one thread each), {ups} updates in {wall:.1f} s, FP64 numpy")


def fp32_accuracy(m, inp, cfg):
    """The FP32 form's error against the FP64 form, both stepped once on
    the GPU from the same input (the FP64 form agrees with the FP64 oracle
    to 1e-12): per-particle velocity and position differences, and the
    observables after the timed runs (kT and net momentum, in `forms`)."""
    pos, vel, bpos, bvel, bmass = inp
    st = {}
    for name, prec in (("fp32", m.FP32), ("fp64", m.FP64)):
        with m.Sim(pos, vel, cfg["n_cells"], kT=cfg["kT"], seed=cfg["seed"], precision=prec,
                   thermostat=cfg["thermostat"], emb_pos=bpos, emb_vel=bvel,
                   emb_mass=bmass) as s:
            s.step(1)
            st[name] = s.get_state()
    L = np.array(cfg["n_cells"], dtype=np.float64)
    dx = st["fp32"][0] - st["fp64"][0]
    dx -= L * np.round(dx / L)
    dv = st["fp32"][1] - st["fp64"][1]
    vs = np.abs(st["fp64"][1])
    return {"what": "one step from the same input, FP32 form minus FP64 form",
            "velocity_max_abs": float(np.abs(dv).max()),
            "velocity_rms": float(np.sqrt(np.mean(dv * dv))),
            "velocity_max_rel": float((np.abs(dv) / np.maximum(vs, 1.0)).max()),
            "position_max_abs": float(np.abs(dx).max())}


def fp32_observables(m, inp, cfg, steps=200):
    """Observables of the FP32 form against the FP64 form after `steps`
    steps from the same input, both on the GPU (the FP64 form agrees with
    the FP64 oracle to 1e-12; the FP32 form against the oracle itself over
    1000 steps is tests/test_gpu_observables.py): kinetic temperature,
    kurtosis of the velocity components (3 for Maxwell-Boltzmann), net
    momentum per particle (change since the start), the occupancy histogram
    of the collision cells (total variation distance between the forms)."""
    pos, vel, bpos, bvel, bmass = inp
    obs = {}
    for name, prec in (("fp32", m.FP32), ("fp64", m.FP64)):
        with m.Sim(pos, vel, cfg["n_cells"], kT=cfg["kT"], seed=cfg["seed"], precision=prec,
                   thermostat=cfg["thermostat"], emb_pos=bpos, emb_vel=bvel,
                   emb_mass=bmass) as s:
            _, v0 = s.get_state()
            P0 = v0.sum(axis=0)
            del v0
            s.step(steps)
            _, v = s.get_state()
            _, counts = s.get_cells()
        n = v.shape[0]
        P = v.sum(axis=0)
        dv = v - P / n
        m2 = (dv * dv).mean(axis=0)
        m4 = (dv ** 4).mean(axis=0)
        hist = np.bincount(counts, minlength=64)[:64] / counts.size
        obs[name] = {"T": float(m2.sum() / 3.0 * n / (n - 1)),
                     "kurtosis": float((m4 / (m2 * m2)).mean()),
                     "momentum_change_per_particle": float(np.abs(P - P0).max() / n),
                     "_hist": hist}
        del v, dv
    tvd = 0.5 * float(np.abs(obs["fp32"]["_hist"] - obs["fp64"]["_hist"]).sum())
    for o in obs.values():
        del o["_hist"]
    return {"what": f"{steps} steps from the same input, FP32 form and FP64 form on the GPU",
            "fp32": obs["fp32"], "fp64": obs["fp64"],
            "T_diff": obs["fp32"]["T"] - obs["fp64"]["T"],
            "kurtosis_diff": obs["fp32"]["kurtosis"] - obs["fp64"]["kurtosis"],
            "occupancy_tvd": tvd}


def batch_latency(m, workloads, cfg, calls=5, singles=100, warmup=20):
    """The 256-box batch's latencies for the line of the default workload
    (the metric's "p99 batch latency"): single-step calls and whole
    `cfg["steps"]`-step calls, each waited for, on the stream; every box
    completes with its call's last launch."""
    steps = cfg["steps"]
    boxes = workloads.replica_inputs(workloads.replica_boxes(cfg["n_rep"], seed=cfg["seed"]))
    N = sum(b["pos"].shape[0] for b in boxes)
    bt = m.Batch(boxes, precision=m.FP32, thermostat=cfg["thermostat"])
    del boxes
    try:
        bt.step(warmup)
        bt.sync()
        one = []
        for _ in range(singles):
            a = time.perf_counter()
            bt.step(1)
            bt.sync()
            one.append(time.perf_counter() - a)
        bt.step(steps)
        bt.sync()
        whole = []
        for _ in range(calls):
            a = time.perf_counter()
            bt.step(steps)
            bt.sync()
            whole.append(time.perf_counter() - a)
    finally:
        bt.close()
    one_ms, whole_ms = 1e3 * np.array(one), 1e3 * np.array(whole)
    return {"workload": "srd_batch256_fp32", "boxes": cfg["n_rep"], "particles": N, "form": "fp32",
            "step_call_ms": {"p50": float(np.percentile(one_ms, 50)),
                             "p99": float(np.percentile(one_ms, 99)), "calls": singles},
            f"call_{steps}_steps_ms": {"p50": float(np.percentile(whole_ms, 50)),
                                       "p99": float(np.percentile(whole_ms, 99)), "calls": calls},
            "updates_per_s": N * steps / float(np.median(whole)),
            "what": "mpcd_step calls on the whole batch, each waited for; every box "
                    "completes with its call"}


def bench_batch(m, workloads, cfg, args):
    """Throughput and single-step latency of a batch of independent boxes."""
    import torch
    steps = cfg["steps"] if args.steps == 1000 else args.steps
    boxes = workloads.replica_inputs(workloads.replica_boxes(cfg["n_rep"], seed=cfg["seed"]))
    N = sum(b["pos"].shape[0] for b in boxes)
    ncells = sum(int(np.prod(b["n_cells"])) for b in boxes)
    torch.cuda.init()
    bt = m.Batch(boxes, precision=m.FP32, thermostat=cfg["thermostat"])
    del boxes
    try:
        bt.step(args.warmup)
        bt.sync()
        bt.profile(True, every=PROFILE_EVERY)
        for w in (0, 1):
            bt.profile_read(w)
        t0 = time.perf_counter()
        bt.step(steps)
        bt.sync()
        t1 = time.perf_counter()
        coll_ms, coll_n = bt.profile_read(0)
        bt.profile(False)
        lat = []
        for _ in range(100):
            a = time.perf_counter()
            bt.step(1)
            bt.sync()
            lat.append(time.perf_counter() - a)
        # whole calls of `steps` steps, kernels launched one by one on the
        # stream and as one HIP graph (every box finishes with the call's last
        # launch, so a box's completion time is the call's)
        calls = {}
        for mode in ("stream", "graph"):
            bt.set_graph(mode == "graph")
            bt.step(steps)
            bt.sync()
            t = []
            for _ in range(args.batch_calls):
                a = time.perf_counter()
                bt.step(steps)
                bt.sync()
                t.append(time.perf_counter() - a)
            t_ms = 1e3 * np.array(t)
            calls[mode] = {"p50": float(np.percentile(t_ms, 50)), "p99": float(np.percentile(t_ms, 99)),
                           "min": float(t_ms.min()), "calls": len(t)}
            print(f"[bench] {steps}-step calls on the {mode}: p50 {calls[mode]['p50']:.1f} ms "
                  f"p99 {calls[mode]['p99']:.1f} ms", file=sys.stderr, flush=True)
        calls["graph_instantiations_updates"] = list(bt.graph_stats())
        bt.set_graph(False)
        P, ke, kT = bt.box_totals()
    finally:
        bt.close()
    ups = N * steps / (t1 - t0)
    avg_us = 1e3 * coll_ms / max(coll_n, 1)
    lat_ms = 1e3 * np.array(lat)
    out = {
        "metric": "particle-updates/s (stream+bin+SRD collide) FP32 vs FP64; p99 batch latency",
        "value": ups, "unit": "particle-updates/s", "n_gpus": 1, "steps": steps,
        "warmup": args.warmup, "ms_per_step": 1e3 * (t1 - t0) / steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "srd_batch256_fp32", "boxes": cfg["n_rep"], "particles": N,
                   "sides": [8, 64], "density": [5, 10], "kT": [0.5, 2.0],
                   "thermostat": "maxwell-boltzmann", "alpha_deg": 130, "dt": 0.1,
                   "form": "fp32"},
        "latency_ms": {"p50": float(np.percentile(lat_ms, 50)),
                       "p99": float(np.percentile(lat_ms, 99)),
                       "what": "one mpcd_step(1) call on the whole batch, waited for"},
        "call_ms": dict(calls, what=f"one mpcd_step({steps}) call on the whole batch, waited for; "
                                    "every box completes with the call"),
        "roofline": roofline("fp32", N, ncells, avg_us,
                             measured_traffic("fp32", "srd_batch256_fp32")),
        "kT_range_end": [float(kT.min()), float(kT.max())],
    }
    print(json.dumps(out), flush=True)


def bench_serve(m, workloads, cfg, args, workers=8, stop_after=75.0):
    """Open-loop serving through paper_1801_10187_amd.serve.Server: requests
    (workloads.serve_requests) are submitted at their Poisson arrival times;
    the server admits them in arrival order as a worker is free and their
    device memory fits beside the requests in flight, each in its own context
    and HIP stream, and returns its cell-averaged velocity field. Requests not
    started `stop_after` seconds after the first arrival are cancelled and
    reported as unserved. Particles of a request are a slice, at a seeded
    offset, of one pool of uniform and Gaussian numbers scaled to the
    request's box and kT (drawing 10^9 fresh numbers per second on the host
    would be the bottleneck)."""
    import threading
    import torch
    from paper_1801_10187_amd.serve import Request, Server
    reqs = workloads.serve_requests(rate=cfg["rate"], duration=cfg["duration"], seed=cfg["seed"])
    npool = int(max(r["density"] * np.prod(r["n_cells"]) for r in reqs)) + 1
    rng = np.random.default_rng(cfg["seed"])
    upool = rng.random((2 * npool, 3))
    gpool = rng.normal(size=(2 * npool, 3))
    torch.cuda.init()
    lock = threading.Lock()
    done = []

    def particles(i, r, n):
        def make():
            off = int(np.random.default_rng(5000 + i).integers(0, npool))
            L = np.array(r["n_cells"], dtype=np.float64)
            pos = upool[off:off + n] * L
            pos = np.where(pos >= L, 0.0, pos)
            vel = gpool[off:off + n] * math.sqrt(cfg["kT"])
            return pos, vel - vel.mean(axis=0)
        return make

    server = Server(workers=workers)
    futs = []
    t0 = time.perf_counter()
    try:
        for i, r in enumerate(reqs):
            now = time.perf_counter() - t0
            if now < r["t"]:
                time.sleep(r["t"] - now)
            n = int(round(r["density"] * np.prod(r["n_cells"])))
            req = Request(r["n_cells"], n, r["steps"], particles(i, r, n), precision=m.FP32,
                          kT=cfg["kT"], seed=r["seed"], thermostat=cfg["thermostat"])
            fut = server.submit(req)

            def finished(f, a=r["t"], w=n * r["steps"]):
                if f.cancelled() or f.exception() is not None:
                    return
                with lock:
                    done.append((a, time.perf_counter() - t0, w))
                    if len(done) % 250 == 0:
                        print(f"[serve] {len(done)} requests done at {done[-1][1]:.1f} s",
                              file=sys.stderr, flush=True)
            fut.add_done_callback(finished)
            futs.append(fut)
        left = stop_after - (time.perf_counter() - t0)
        if left > 0:
            time.sleep(left)
        for f in futs:
            f.cancel()              # only requests not started yet
    finally:
        server.close()
    wall = time.perf_counter() - t0
    errors = [f.exception() for f in futs if not f.cancelled() and f.exception() is not None]
    if errors:
        raise errors[0]
    lat = np.array([e - a for a, e, _ in done])
    served = sum(w for _, _, w in done)
    offered = sum(r["density"] * np.prod(r["n_cells"]) * r["steps"] for r in reqs) / cfg["duration"]
    out = {
        "metric": "particle-updates/s (stream+bin+SRD collide) FP32 vs FP64; p99 batch latency",
        "value": served / wall, "unit": "particle-updates/s", "n_gpus": 1,
        "steps": int(sum(r["steps"] for r in reqs[:len(done)])), "warmup": 0,
        "ms_per_step": None, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": "srd_serve_poisson50", "rate_per_s": cfg["rate"],
                   "duration_s": cfg["duration"], "requests": len(reqs),
                   "particles": "log-uniform 1e4..1e7", "steps": "uniform 100..2000",
                   "density": [5, 10], "kT": cfg["kT"], "thermostat": "maxwell-boltzmann",
                   "form": "fp32", "workers": workers, "stop_after_s": stop_after,
                   "admission": "FIFO by worker slot and device-memory budget"},
        "served_requests": len(done), "unserved_requests": len(reqs) - len(done),
        "offered_updates_per_s": offered, "served_updates_per_s": served / wall,
        "wall_s": wall, "max_requests_in_flight": server.max_inflight,
        "max_bytes_in_flight": server.max_inflight_bytes, "memory_budget": server.budget,
        "latency_ms": {"p50": float(np.percentile(lat, 50) * 1e3) if len(lat) else None,
                       "p99": float(np.percentile(lat, 99) * 1e3) if len(lat) else None,
                       "what": "request completion minus arrival, completed requests"},
    }
    print(json.dumps(out), flush=True)


def bench_md(m, workloads, cfg, args):
    """Solutes coupled through MD (sec. 3.6, sec. 4.3): per collision the
    beads move by 50 velocity-Verlet steps of 0.002 (harmonic bonds along
    each chain, the library's mpcd_md_verlet_chains, on the device), their
    state is handed over (mpcd_set_embedded), one MPCD step runs and the
    collided bead velocities come back (mpcd_get_embedded) -- all on device
    buffers and one stream. Reported beside it: the integrator alone and the
    same context stepping without the exchange."""
    import torch
    steps = cfg["steps"] if args.steps == 1000 else args.steps
    pos, vel, bpos, bvel, bmass = make_input(cfg)
    N = pos.shape[0] + bpos.shape[0]
    clen, nchains = cfg["chain_len"], cfg["chains"]
    torch.cuda.init()
    # one stream for the integrator and the context (the handle of torch's
    # default stream is 0, for which the context would make its own stream)
    md_stream = torch.cuda.Stream()
    stream = md_stream.cuda_stream
    sim = m.Sim(pos, vel, cfg["n_cells"], kT=cfg["kT"], seed=cfg["seed"], precision=m.FP32,
                thermostat=False, emb_pos=bpos, emb_vel=bvel, emb_mass=bmass,
                flags=m.binding.FLAG_MD_SOLUTE, hip_stream=stream)
    del pos, vel
    dpos = torch.from_numpy(bpos).cuda()
    dvel = torch.from_numpy(bvel).cuda()
    dmass = torch.from_numpy(bmass).cuda()
    L = [float(x) for x in cfg["n_cells"]]
    md_steps, md_dt = 50, 0.002
    torch.cuda.synchronize()

    def integrate():
        m.binding.md_verlet_chains(dpos.data_ptr(), dvel.data_ptr(), dmass.data_ptr(), nchains,
                                   clen, L, md_dt, md_steps, hip_stream=stream)

    def cycle():
        integrate()
        sim.set_embedded_device(dpos.data_ptr(), dvel.data_ptr())
        sim.step(1)
        sim.get_embedded_device(dpos.data_ptr(), dvel.data_ptr())

    try:
        for _ in range(args.warmup):
            cycle()
        sim.sync()
        sim.profile(True, every=PROFILE_EVERY)
        for w in (0, 1):
            sim.profile_read(w)
        t0 = time.perf_counter()
        for _ in range(steps):
            cycle()
        sim.sync()
        t1 = time.perf_counter()
        coll_ms, coll_n = sim.profile_read(0)
        bin_ms, bin_n = sim.profile_read(1)
        sim.profile(False)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(md_stream)
        for _ in range(10):
            integrate()
        e1.record(md_stream)
        torch.cuda.synchronize()
        md_ms = e0.elapsed_time(e1) / 10
        t2 = time.perf_counter()
        sim.step(steps)
        sim.sync()
        t3 = time.perf_counter()
        handovers = sim.handover_stats()
    finally:
        sim.close()
    cyc = (t1 - t0) / steps
    plain = (t3 - t2) / steps
    avg_us = 1e3 * coll_ms / max(coll_n, 1)
    out = {
        "metric": "particle-updates/s (stream+bin+SRD collide) FP32 vs FP64; p99 batch latency",
        "value": N / cyc, "unit": "particle-updates/s", "n_gpus": 1, "steps": steps,
        "warmup": args.warmup, "ms_per_step": 1e3 * cyc, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "srd_400c_rho5_md", "n_cells": list(cfg["n_cells"]),
                   "particles": N, "density": cfg["density"], "embedded_beads": int(bpos.shape[0]),
                   "coupling": f"{md_steps} velocity-Verlet steps of {md_dt} per collision on the "
                               "device (harmonic bonds), state exchanged on device every collision",
                   "thermostat": "none", "form": "fp32"},
        "roofline": roofline("fp32", N, int(np.prod(cfg["n_cells"])), avg_us),
        "bin_kernel_avg_us": 1e3 * bin_ms / max(bin_n, 1),
        "md_integrator_ms": md_ms,
        "ms_per_step_without_exchange": 1e3 * plain,
        "exchange_overhead_ms": 1e3 * (cyc - plain) - md_ms,
        "handovers_kept_given_up": list(handovers),
    }
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--cpu-steps", type=int, default=4)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--forms", default=None,
                    help="storage forms to time, a suffix _at for the Andersen-thermostat "
                         "rule (default fp32,fp64,fp32_at,fp64_at; fp32 for the large box)")
    ap.add_argument("--workload", default=WORKLOAD,
                    choices=["srd_100c_rho10_mbthermo", "srd_20c_rho5_fp64", "srd_400c_rho5_beads",
                             "srd_batch256_fp32", "srd_serve_poisson50", "srd_400c_rho5_md"])
    ap.add_argument("--serve-workers", type=int, default=8,
                    help="host threads serving requests (srd_serve_poisson50)")
    ap.add_argument("--no-batch", action="store_true",
                    help="leave the 256-box batch latencies out of the default workload's line")
    ap.add_argument("--batch-calls", type=int, default=12,
                    help="timed whole calls per launch mode (srd_batch256_fp32)")
    ap.add_argument("--copy-only", action="store_true",
                    help="only run the streaming copy kernel (1 GiB, 20 times)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {args.gpus} is not supported "
              "(this measurement covers one GPU's share)", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_1801_10187_amd as m
    import workloads

    if args.copy_only:
        torch.cuda.init()
        print(json.dumps({"copy_GBs": copy_ceiling(m)}), flush=True)
        return
    wl = args.workload
    cfg = workloads.CONFIGS[wl]
    if wl == "srd_batch256_fp32":
        return bench_batch(m, workloads, cfg, args)
    if wl == "srd_serve_poisson50":
        return bench_serve(m, workloads, cfg, args, workers=args.serve_workers)
    if wl == "srd_400c_rho5_md":
        return bench_md(m, workloads, cfg, args)
    big = wl != WORKLOAD
    small = wl == "srd_20c_rho5_fp64"   # the 40 000-particle parity box, plain FP64
    if big and args.steps == 1000:
        args.steps = cfg["steps"]
    inp = make_input(cfg)
    N = inp[0].shape[0] + (0 if inp[2] is None else inp[2].shape[0])
    rho = cfg["density"]
    ncells = int(np.prod(cfg["n_cells"]))
    torch.cuda.init()
    default_forms = "fp64" if small else ("fp32" if big else "fp32,fp64,fp32_at,fp64_at")
    forms = [f.strip() for f in (args.forms or default_forms).split(",") if f.strip()]
    res = {}
    for form in forms:
        base = form.split("_")[0]
        if base not in STATE_BYTES or form not in (base, base + "_at"):
            sys.exit(f"unknown form {form}")
        prec = m.FP32 if base == "fp32" else m.FP64
        rule = m.AT if form.endswith("_at") else m.SRD
        r = run_form(m, inp, cfg, prec, args.steps, args.warmup, rule)
        r["updates_per_s"] = N * args.steps / r["seconds"]
        r["ms_per_step"] = 1e3 * r["seconds"] / args.steps
        avg_us = 1e3 * r["collide_ms"] / max(r["collide_launches"], 1)
        r["collide_avg_us"] = avg_us
        r["collide_GBs"] = roofline(base, N, ncells, avg_us)["achieved"]
        r["step_floor_frac"] = r["updates_per_s"] * floor_bytes_per_update(base, rho) / (HBM_PEAK_GBS * 1e9)
        r["rule"] = "at" if rule == m.AT else "srd"
        r["thermostat"] = "maxwell-boltzmann" if (cfg["thermostat"] and rule == m.SRD) else "none"
        res[form] = r
        print(f"[bench] {form}: {r['updates_per_s']:.4g} updates/s, "
              f"{r['ms_per_step']:.4f} ms/step, collide {avg_us:.1f} us "
              f"({r['collide_GBs']:.0f} GB/s)",
              file=sys.stderr, flush=True)

    head = res.get("fp32") or res[forms[0]]
    head_form = "fp32" if "fp32" in res else forms[0]
    # the same call with its kernels launched as one HIP graph
    base = head_form.split("_")[0]
    g = run_form(m, inp, cfg, m.FP32 if base == "fp32" else m.FP64, args.steps, args.warmup,
                 m.AT if head_form.endswith("_at") else m.SRD, graph=True)
    graph_cmp = {"form": head_form, "stream_ms_per_step": head["ms_per_step"],
                 "graph_ms_per_step": 1e3 * g["seconds"] / args.steps,
                 "what": f"one {args.steps}-step call, kernels launched one by one on the "
                         "stream against one HIP graph (kept and updated between calls)"}
    print(f"[bench] graph: {graph_cmp['graph_ms_per_step']:.4f} ms/step "
          f"(stream {head['ms_per_step']:.4f})", file=sys.stderr, flush=True)
    out = {
        "metric": "particle-updates/s (stream+bin+SRD collide) FP32 vs FP64; p99 batch latency",
        "value": head["updates_per_s"],
        "unit": "particle-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if head_form.startswith("fp32") else "f64",
        "data": "synthetic",
        "config": {"workload": wl, "n_cells": list(cfg["n_cells"]),
                   "particles": N, "density": rho, "alpha_deg": 130, "dt": 0.1,
                   "kT": cfg["kT"],
                   "thermostat": "maxwell-boltzmann" if cfg["thermostat"] else "none",
                   "embedded_beads": 0 if inp[2] is None else int(inp[2].shape[0]),
                   "grid_shift": True, "form": head_form},
        "roofline": roofline(head_form.split("_")[0], N, ncells, head["collide_avg_us"],
                             measured_traffic(head_form, wl) if head_form in STATE_BYTES else None),
        "step_floor_frac": head["step_floor_frac"],
        "graph_vs_stream": graph_cmp,
        "forms": {f: {"updates_per_s": r["updates_per_s"], "ms_per_step": r["ms_per_step"],
                      "collide_avg_us": r["collide_avg_us"], "collide_GBs": r["collide_GBs"],
                      "rule": r["rule"], "thermostat": r["thermostat"],
                      "step_floor_frac": r["step_floor_frac"], "kT_end": r["kT"],
                      "net_momentum_end": r["net_momentum"]} for f, r in res.items()},
    }
    if wl == WORKLOAD and not args.no_batch:
        out["batch_latency"] = batch_latency(m, workloads, workloads.CONFIGS["srd_batch256_fp32"])
        b = out["batch_latency"]
        print(f"[bench] batch: step call p99 {b['step_call_ms']['p99']:.3f} ms, "
              f"{b['updates_per_s']:.4g} updates/s", file=sys.stderr, flush=True)
    copies = copy_ceiling(m)
    out["copy_ceiling_GBs"] = copies["max"]
    out["copies_GBs"] = copies
    out["roofline"]["frac_of_copy_ceiling"] = head["collide_GBs"] / copies["max"]
    if "fp32" in res and "fp64" in res:
        out["fp32_over_fp64"] = res["fp32"]["updates_per_s"] / res["fp64"]["updates_per_s"]
        out["fp32_accuracy"] = fp32_accuracy(m, inp, cfg)
        out["fp32_observables"] = fp32_observables(m, inp, cfg)
    for base in ("fp32", "fp64"):  # the AT rule against the thermostatted SRD step
        if base in res and base + "_at" in res:
            out[base + "_at_over_srd"] = res[base + "_at"]["updates_per_s"] / res[base]["updates_per_s"]
    if not args.no_cpu_baseline:
        if big and not small:
            single = cpu_baseline(make_input(cfg, scale=60), (60, 60, 60), cfg, args.cpu_steps,
                                  "a 60^3-cell sample box of the same recipe")
        else:
            single = cpu_baseline(inp, cfg["n_cells"], cfg,
                                  cfg["steps"] if small else args.cpu_steps, "the full workload")
        if small:
            single["cpu_model"] = cpu_model()
            out["cpu_baseline"] = single
        else:
            # every core: independent 60^3-cell boxes of the workload's recipe
            # (density, kT, thermostat), one per worker, seeds 1, 2, ...
            jobs = [((60, 60, 60), rho, cfg["kT"], 1 + i, cfg["thermostat"], args.cpu_steps)
                    for i in range(min(len(os.sched_getaffinity(0)), 16))]
            allc = cpu_baseline_all_cores(jobs, f"{args.cpu_steps} oracle steps per box")
            allc["single_core"] = single
            out["cpu_baseline"] = allc
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
