"""How a run is split into mpcd_step calls must not change it: a call leaves
the collided state readable and the next step's binning prepared, and the
next call starts from that binning. Every split below is compared bit for
bit with one long call (or with the oracle where the split itself is what
is tested)."""
import numpy as np
import pytest

import paper_1801_10187_amd as m
import workloads
from helpers import FP64_REL, banner, periodic_dist, vel_err_fp64
from oracle import srd

pytestmark = pytest.mark.gpu


def _sim(pos, vel, p, precision=m.FP64, collision=None, **kw):
    extra = {} if collision is None else {"collision": collision}
    return m.Sim(pos, vel, p.n_cells, a=p.a, alpha=p.alpha, dt=p.dt, kT=p.kT, seed=p.seed,
                 solvent_mass=p.solvent_mass, precision=precision, thermostat=p.thermostat,
                 grid_shift=p.grid_shift, **extra, **kw)


def _same(a, b):
    # a stale count left in the scatter's counters would show as particles
    # placed twice, which the slabs have no room for
    assert a.layout()[3] == 0 and b.layout()[3] == 0
    pa, va = a.get_state()
    pb, vb = b.get_state()
    ca, na = a.get_cells()
    cb, nb = b.get_cells()
    assert np.array_equal(pa, pb) and np.array_equal(va, vb)
    assert np.array_equal(ca, cb) and np.array_equal(na, nb)


@pytest.mark.parametrize("form,thermo,rule", [("fp64", True, "srd"), ("fp64", False, "srd"),
                                              ("fp32", True, "srd"), ("fp64", False, "at"),
                                              ("fp32", False, "at")])
def test_single_step_calls_equal_one_call(form, thermo, rule):
    banner(f"step(1) x 6 == step(6) {form} thermo={thermo} {rule}")
    p = srd.Params((13, 9, 10), seed=51, thermostat=thermo)
    pos, vel = workloads.fluid(p.n_cells, 7, seed=52)
    prec = m.FP64 if form == "fp64" else m.FP32
    coll = m.AT if rule == "at" else None
    with _sim(pos, vel, p, prec, coll) as a, _sim(pos, vel, p, prec, coll) as b:
        a.step(6)
        for _ in range(6):
            b.step(1)
        assert b.step_count == 6
        _same(a, b)


def test_reads_between_calls_leave_the_run_unchanged():
    """State, cells, totals and the velocity field read between calls see the
    collided state; the run goes on as if they had not been read."""
    banner("reads between calls")
    p = srd.Params((11, 12, 9), seed=53, thermostat=True)
    pos, vel = workloads.fluid(p.n_cells, 6, seed=54)
    mass = np.ones(pos.shape[0])
    with _sim(pos, vel, p) as a, _sim(pos, vel, p) as b:
        a.step(5)
        b.step(2)
        gpos, gvel = b.get_state()
        gcells, _ = b.get_cells()
        u, M = b.velocity_field()
        P, ke, _ = b.totals()
        b.step(3)
        _same(a, b)
    opos, ovel, info = srd.run(pos, vel, mass, p, 0, 2)
    assert np.array_equal(gcells, info["cell"])
    assert vel_err_fp64(gvel, ovel) < FP64_REL
    assert periodic_dist(gpos, opos, p.L).max() < 1e-12
    ou, oM = srd.velocity_field(gpos, gvel, mass, p)
    assert np.array_equal(M, oM)
    assert np.max(np.abs(u - ou)) < 1e-14 * max(1.0, np.abs(ou).max())
    oP, oke, _ = srd.totals(ovel, mass)
    assert np.allclose(P, oP, atol=1e-10) and abs(ke - oke) < 1e-9 * oke


def test_separate_calls_between_fused_calls():
    banner("step, stream/bin/collide, step")
    p = srd.Params((10, 9, 8), seed=55, thermostat=True)
    pos, vel = workloads.fluid(p.n_cells, 5, seed=56)
    with _sim(pos, vel, p) as a, _sim(pos, vel, p) as b:
        a.step(6)
        b.step(2)
        b.stream()
        b.bin()
        b.get_cell_props()
        b.collide()
        b.step(1)
        b.step(2)
        _same(a, b)


def test_step_counter_change_between_calls():
    """Moving the step counter drops the prepared binning (it used the old
    step's grid shift): the result equals a fresh context at the new step."""
    banner("set_step between calls")
    p = srd.Params((9, 10, 11), seed=57, thermostat=True)
    pos, vel = workloads.fluid(p.n_cells, 6, seed=58)
    with _sim(pos, vel, p) as a:
        a.step(3)
        p3, v3 = a.get_state()
        a.step_count = 40
        a.step(2)
        pa, va = a.get_state()
        a.step_count = 42          # unchanged: the prepared binning stays valid
        a.step(1)
        pa1, va1 = a.get_state()
        assert a.layout()[3] == 0
    with _sim(p3, v3, p) as c:
        c.step_count = 40
        c.step(2)
        pc, vc = c.get_state()
    with _sim(pc, vc, p) as d:
        d.step_count = 42
        d.step(1)
        pd, vd = d.get_state()
    assert np.array_equal(pa, pc) and np.array_equal(va, vc)
    assert np.array_equal(pa1, pd) and np.array_equal(va1, vd)


def test_overflow_in_the_last_launch_of_a_call():
    """Single-step calls on a converging flow with slabs sized to the initial
    maximum: scatters into the prepared binning overflow, the slabs grow and
    the launch is replayed; the run still matches the oracle."""
    banner("overflow at the end of a call")
    p = srd.Params((12, 12, 12), seed=59, thermostat=True)
    pos, vel = workloads.fluid(p.n_cells, 9, seed=60)
    vel = vel - (pos - p.L / 2)
    mass = np.ones(pos.shape[0])
    with _sim(pos, vel, p, flags=m.binding.FLAG_TIGHT_SLABS) as b:
        _, _, cap0, _ = b.layout()
        for _ in range(6):
            b.step(1)
        gpos, gvel = b.get_state()
        gcells, _ = b.get_cells()
        _, _, cap1, regrows = b.layout()
    assert regrows >= 1 and cap1 > cap0
    opos, ovel, info = srd.run(pos, vel, mass, p, 0, 6)
    assert np.array_equal(gcells, info["cell"])
    assert vel_err_fp64(gvel, ovel) < FP64_REL
    assert periodic_dist(gpos, opos, p.L).max() < 1e-12


@pytest.mark.parametrize("form", ["fp64", "fp32"])
def test_batch_single_step_calls(form):
    banner(f"batch step(1) x 4 == step(4) {form}")
    boxes = []
    for i, (n, rho) in enumerate([((9, 7, 5), 8.0), ((3, 10, 12), 5.5), ((16, 16, 16), 6.5)]):
        pos, vel = workloads.fluid(n, rho, seed=200 + i)
        boxes.append(dict(n_cells=n, density=rho, seed=70 + i, kT=1.0 + 0.2 * i, pos=pos, vel=vel))
    prec = m.FP64 if form == "fp64" else m.FP32
    with m.Batch(boxes, precision=prec, thermostat=True) as a, \
            m.Batch(boxes, precision=prec, thermostat=True) as b:
        a.step(4)
        for _ in range(4):
            b.step(1)
        _same(a, b)


def test_embedded_state_set_between_calls():
    """Handing the embedded particles their own state back between calls
    drops the prepared binning and changes nothing."""
    banner("set_embedded between calls")
    p = srd.Params((10, 10, 10), seed=61, thermostat=True)
    pos, vel = workloads.fluid(p.n_cells, 6, seed=62)
    bpos, bvel, bmass = workloads.beads(p.n_cells, 4, 10, seed=63)
    kw = dict(emb_pos=bpos, emb_vel=bvel, emb_mass=bmass)
    with _sim(pos, vel, p, **kw) as a, _sim(pos, vel, p, **kw) as b:
        a.step(4)
        b.step(2)
        ep, ev = b.get_embedded()
        b.set_embedded(ep, ev)
        b.step(1)
        b.set_embedded(*b.get_embedded())
        b.step(1)
        _same(a, b)


def test_embedded_index_survives_regrow():
    """The library finds embedded particles through a slot index kept by
    every kernel that moves them; after slab regrows and single-step calls
    the exchange still returns exactly the embedded rows of the state, and
    the run still matches the oracle."""
    banner("embedded index after regrow")
    p = srd.Params((12, 12, 12), seed=64, thermostat=True)
    pos, vel = workloads.fluid(p.n_cells, 9, seed=65)
    vel = vel - (pos - p.L / 2)
    bpos, bvel, bmass = workloads.beads(p.n_cells, 10, 10, seed=66)
    ns = pos.shape[0]
    with _sim(pos, vel, p, flags=m.binding.FLAG_TIGHT_SLABS, emb_pos=bpos, emb_vel=bvel,
              emb_mass=bmass) as b:
        for _ in range(4):
            b.step(1)
        ep, ev = b.get_embedded()
        gpos, gvel = b.get_state()
        assert np.array_equal(ep, gpos[ns:]) and np.array_equal(ev, gvel[ns:])
        b.set_embedded(ep, ev)
        b.step(2)
        gpos, gvel = b.get_state()
        ep, ev = b.get_embedded()
        regrows = b.layout()[3]
    assert regrows >= 1
    assert np.array_equal(ep, gpos[ns:]) and np.array_equal(ev, gvel[ns:])
    apos = np.concatenate([pos, bpos])
    avel = np.concatenate([vel, bvel])
    amass = np.concatenate([np.ones(ns), bmass])
    opos, ovel, _ = srd.run(apos, avel, amass, p, 0, 6)
    assert vel_err_fp64(gvel, ovel, m=1.0) < FP64_REL
    assert periodic_dist(gpos, opos, p.L).max() < 1e-12


def test_sampled_kernel_timing():
    """mpcd_profile_enable(P) brackets the first launch of each kind and one
    in every P after it; P = 0 turns timing off, P < 0 is refused."""
    banner("sampled kernel timing")
    p = srd.Params((8, 8, 8), seed=67, thermostat=True)
    pos, vel = workloads.fluid(p.n_cells, 6, seed=68)
    with _sim(pos, vel, p) as s:
        s.step(1)
        s.profile(True, every=3)
        s.step(10)
        ms, n = s.profile_read(0)
        assert n == 4 and ms > 0.0   # launches 0, 3, 6, 9
        # the thermostat's draws run inside the collision kernel: no third kind
        with pytest.raises(m.MpcdError):
            s.profile_read(2)
        s.profile(True, every=1)
        s.step(5)
        assert s.profile_read(0)[1] == 5
        s.profile(False)
        s.step(2)
        assert s.profile_read(0)[1] == 0
        with pytest.raises(m.MpcdError):
            s.profile(True, every=-1)


@pytest.mark.parametrize("form", ["fp32", "fp64"])
def test_split_state_reads(form):
    """Between calls the collided velocities live in the prepared binning and
    the positions in the current buffer; state, embedded rows and totals read
    there equal those of a context that stepped with separate calls (state
    whole in one buffer), and the run goes on unchanged."""
    banner(f"split-state reads {form}")
    p = srd.Params((10, 11, 9), seed=69, thermostat=True)
    pos, vel = workloads.fluid(p.n_cells, 6, seed=70)
    bpos, bvel, bmass = workloads.beads(p.n_cells, 3, 10, seed=71)
    prec = m.FP64 if form == "fp64" else m.FP32
    kw = dict(emb_pos=bpos, emb_vel=bvel, emb_mass=bmass)
    with _sim(pos, vel, p, prec, **kw) as a, _sim(pos, vel, p, prec, **kw) as b, \
            _sim(pos, vel, p, prec, **kw) as c:
        a.step(5)
        b.step(2)
        sb, eb, tb = b.get_state(), b.get_embedded(), b.totals()
        b.step(3)
        for _ in range(2):
            c.stream()
            c.bin()
            c.collide()
        sc, ec, tc = c.get_state(), c.get_embedded(), c.totals()
        for x, y in zip(sb + eb, sc + ec):
            assert np.array_equal(x, y)
        assert np.array_equal(tb[0], tc[0]) and tb[1] == tc[1] and tb[2] == tc[2]
        _same(a, b)
