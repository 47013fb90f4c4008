"""The Andersen-thermostat collision rule (eq. 4, sec. 3.7) on the GPU
against the oracle: cells bit-exact, FP64 velocities within 1e-12, FP32 one
step within one ulp plus the single-precision rounding of the kicks (the FP32
form draws them in single precision, sec. 4.1), beads, batches and the
re-read path of crowded tiles."""
import numpy as np
import pytest

import paper_1801_10187_amd as m
import workloads
from helpers import (FP64_REL, at32_close, at32_kick_units, banner, periodic_dist,
                     vel_err_fp64)
from oracle import fp32form, srd

pytestmark = pytest.mark.gpu


def _sim(pos, vel, p, precision=m.FP64, **kw):
    return m.Sim(pos, vel, p.n_cells, a=p.a, alpha=p.alpha, dt=p.dt, kT=p.kT, seed=p.seed,
                 solvent_mass=p.solvent_mass, precision=precision, thermostat=False,
                 grid_shift=p.grid_shift, collision=m.AT, **kw)


def test_at_fp64_three_steps():
    banner("AT fp64 3 steps")
    p = srd.Params((14, 9, 11), seed=41, kT=1.4, rule="at")
    pos, vel = workloads.fluid(p.n_cells, 7, seed=42, kT=0.8)
    mass = np.ones(pos.shape[0])
    with _sim(pos, vel, p) as s:
        s.step(3)
        gpos, gvel = s.get_state()
        gcells, _ = s.get_cells()
        with pytest.raises(m.MpcdError):
            s.stream()
            s.bin()
            s.get_cell_draws()
    opos, ovel, info = srd.run(pos, vel, mass, p, 0, 3)
    assert np.array_equal(gcells, info["cell"])
    assert vel_err_fp64(gvel, ovel) < FP64_REL
    assert periodic_dist(gpos, opos, p.L).max() < 1e-12


def test_at_fp64_with_beads():
    banner("AT fp64 beads")
    p = srd.Params((12, 12, 12), seed=43, kT=1.0, rule="at")
    pos, vel = workloads.fluid(p.n_cells, 5, seed=44)
    bpos, bvel, bmass = workloads.beads(p.n_cells, 10, 20, seed=45)
    with _sim(pos, vel, p, emb_pos=bpos, emb_vel=bvel, emb_mass=bmass) as s:
        s.step(2)
        gpos, gvel = s.get_state()
    mass = np.concatenate([np.ones(pos.shape[0]), bmass])
    opos, ovel, _ = srd.run(np.concatenate([pos, bpos]), np.concatenate([vel, bvel]), mass, p, 0, 2)
    assert vel_err_fp64(gvel, ovel) < FP64_REL
    assert periodic_dist(gpos, opos, p.L).max() < 1e-12


def test_at_fp32_one_step():
    banner("AT fp32 one step")
    p = srd.Params((16, 12, 10), seed=46, kT=1.0, rule="at")
    pos, vel = workloads.fluid(p.n_cells, 8, seed=47)
    mass = np.ones(pos.shape[0])
    h, o, v = fp32form.from_double(pos, vel, p)
    with _sim(pos, vel, p, precision=m.FP32) as s:
        s.step(1)
        gpos, gvel = s.get_state()
        gcells, _ = s.get_cells()
    h1, o1, v1, info = fp32form.step32(h, o, v, mass, p, 0)
    assert np.array_equal(gcells, info["cell"])
    assert np.array_equal(gpos, fp32form.to_double(h1, o1, p))
    assert np.all(at32_close(gvel, v1, info))
    print(f"[gpu-test] AT fp32: largest difference beyond one ulp: "
          f"{at32_kick_units(gvel, v1, info):.3g} kick ulps")


def test_at_batch_matches_each_box():
    banner("AT batch")
    specs = [dict(n_cells=(8, 6, 5), density=9.0, kT=0.9, seed=51),
             dict(n_cells=(10, 10, 10), density=5.0, kT=1.5, seed=52)]
    boxes = []
    for i, b in enumerate(specs):
        pos, vel = workloads.fluid(b["n_cells"], b["density"], kT=b["kT"], seed=60 + i)
        boxes.append(dict(b, pos=pos, vel=vel))
    with m.Batch(boxes, precision=m.FP64, collision=m.AT) as bt:
        bt.step(2)
        gpos, gvel = bt.get_state()
        info = [bt.box(b) for b in range(len(boxes))]
    for b, bx in enumerate(boxes):
        t0, n, _, _, _ = info[b]
        p = srd.Params(bx["n_cells"], seed=bx["seed"], kT=bx["kT"], rule="at")
        opos, ovel, _ = srd.run(bx["pos"], bx["vel"], np.ones(n), p, 0, 2)
        assert vel_err_fp64(gvel[t0:t0 + n], ovel) < FP64_REL


def test_at_crowded_cell():
    """More particles in one tile than the kernel holds in registers: the
    random velocities are drawn again on the re-read path and must agree."""
    banner("AT crowded cell")
    p = srd.Params((4, 4, 4), seed=53, grid_shift=False, dt=0.01, rule="at")
    rng = np.random.default_rng(54)
    pos = np.concatenate([1.2 + 0.6 * rng.random((3000, 3)), rng.random((500, 3)) * 4.0])
    vel = rng.normal(size=pos.shape) * 0.5
    with _sim(pos, vel, p) as s:
        s.step(2)
        gpos, gvel = s.get_state()
    opos, ovel, _ = srd.run(pos, vel, np.ones(pos.shape[0]), p, 0, 2)
    assert vel_err_fp64(gvel, ovel) < FP64_REL


@pytest.mark.parametrize("form", ["fp64", "fp32"])
def test_at_full_size_benchmark_fluid(form):
    """The 10^7-particle fluid of the benchmark under the AT rule, in the
    launch configuration the benchmark times: one step against the oracle
    element by element (FP32: its emulation; cells and positions exact,
    velocities within one ulp plus the single-precision rounding of the
    kicks, at32_close)."""
    cfg = workloads.CONFIGS["srd_100c_rho10_mbthermo"]
    banner(f"AT full size {form}")
    p = srd.Params(cfg["n_cells"], seed=cfg["seed"], kT=cfg["kT"], rule="at")
    pos, vel = workloads.fluid(cfg["n_cells"], cfg["density"], seed=cfg["seed"])
    mass = np.ones(pos.shape[0])
    prec = m.FP64 if form == "fp64" else m.FP32
    with _sim(pos, vel, p, precision=prec) as s:
        s.step(1)
        gpos, gvel = s.get_state()
        gcells, gcounts = s.get_cells()
    assert gcounts.sum() == pos.shape[0]
    if form == "fp64":
        opos, ovel, info = srd.run(pos, vel, mass, p, 0, 1)
        assert np.array_equal(gcells, info["cell"])
        assert vel_err_fp64(gvel, ovel) < FP64_REL
        assert periodic_dist(gpos, opos, p.L).max() < 1e-12
    else:
        h, o, v = fp32form.from_double(pos, vel, p)
        h1, o1, v1, info = fp32form.step32(h, o, v, mass, p, 0)
        assert np.array_equal(gcells, info["cell"])
        assert np.array_equal(gpos, fp32form.to_double(h1, o1, p))
        assert np.all(at32_close(gvel, v1, info))
        print(f"[gpu-test] AT fp32 full size: largest difference beyond one ulp: "
              f"{at32_kick_units(gvel, v1, info):.3g} kick ulps")
