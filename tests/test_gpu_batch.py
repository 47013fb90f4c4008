"""Batches of independent boxes (mpcd_create_batch): every box of a batch
must evolve exactly as the same box alone, i.e. as the oracle run on that
box with its own parameters and seed."""
import numpy as np
import pytest

import paper_1801_10187_amd as m
import workloads
from helpers import FP64_REL, banner, periodic_dist, ulp_diff_f32, vel_err_fp64
from oracle import fp32form, srd

pytestmark = pytest.mark.gpu

# sizes that exercise every tile shape: a box smaller than a tile along an
# axis, densities on both sides of the 64-/128-cell tile threshold (3.5),
# partial tiles at the far faces
BOXES = [
    dict(n_cells=(9, 7, 5), density=8.0, kT=1.0, seed=11),
    dict(n_cells=(3, 10, 12), density=2.5, kT=0.7, seed=12),
    dict(n_cells=(16, 16, 16), density=6.5, kT=1.6, seed=13),
    dict(n_cells=(5, 5, 5), density=9.0, kT=1.2, seed=14, a=0.8),
]


def _inputs(boxes):
    out = []
    for i, b in enumerate(boxes):
        pos, vel = workloads.fluid(b["n_cells"], b["density"], kT=b["kT"], seed=100 + i,
                                   a=b.get("a", 1.0))
        out.append(dict(b, pos=pos, vel=vel))
    return out


def _params(b, thermo):
    return srd.Params(b["n_cells"], a=b.get("a", 1.0), seed=b["seed"], thermostat=thermo,
                      kT=b["kT"])


@pytest.mark.parametrize("thermo", [True, False])
def test_batch_fp64_matches_each_box_alone(thermo):
    banner(f"batch fp64 thermo={thermo}")
    boxes = _inputs(BOXES)
    with m.Batch(boxes, precision=m.FP64, thermostat=thermo) as bt:
        assert bt.n_boxes == len(boxes)
        bt.step(3)
        gpos, gvel = bt.get_state()
        gcells, gcounts = bt.get_cells()
        P, ke, kT = bt.box_totals()
        info = [bt.box(b, step=2) for b in range(len(boxes))]
    for b, bx in enumerate(boxes):
        t0, n, c0, nc, s2 = info[b]
        p = _params(bx, thermo)
        assert n == bx["pos"].shape[0] and nc == p.ncells
        assert np.array_equal(s2, srd.grid_shift(p, 2))
        mass = np.ones(n)
        opos, ovel, oinfo = srd.run(bx["pos"], bx["vel"], mass, p, 0, 3)
        sl = slice(t0, t0 + n)
        assert np.array_equal(gcells[sl], oinfo["cell"])
        assert np.array_equal(gcounts[c0:c0 + nc], oinfo["count"])
        assert vel_err_fp64(gvel[sl], ovel) < FP64_REL
        assert periodic_dist(gpos[sl], opos, p.L).max() < 1e-12
        oP, oke, _ = srd.totals(ovel, mass)
        assert np.allclose(P[b], oP, atol=1e-9) and abs(ke[b] - oke) < 1e-9 * oke


def test_batch_fp32_one_step_each_box():
    banner("batch fp32 one step")
    boxes = _inputs(BOXES)
    with m.Batch(boxes, precision=m.FP32, thermostat=True) as bt:
        bt.step(1)
        gpos, gvel = bt.get_state()
        gcells, _ = bt.get_cells()
        info = [bt.box(b) for b in range(len(boxes))]
    for b, bx in enumerate(boxes):
        t0, n, _, _, _ = info[b]
        p = _params(bx, True)
        h, o, v = fp32form.from_double(bx["pos"], bx["vel"], p)
        h1, o1, v1, oinfo = fp32form.step32(h, o, v, np.ones(n), p, 0)
        sl = slice(t0, t0 + n)
        assert np.array_equal(gcells[sl], oinfo["cell"])
        assert np.array_equal(gpos[sl], fp32form.to_double(h1, o1, p))
        assert ulp_diff_f32(gvel[sl].astype(np.float32), v1).max() <= 1


def test_batch_cell_props_and_draws():
    banner("batch cell props and draws")
    boxes = _inputs(BOXES)
    with m.Batch(boxes, precision=m.FP64, thermostat=True) as bt:
        bt.stream()
        bt.bin()
        gm, gP, gek = bt.get_cell_props()
        gax, gxi = bt.get_cell_draws()
        info = [bt.box(b) for b in range(len(boxes))]
    for b, bx in enumerate(boxes):
        _, n, c0, nc, _ = info[b]
        p = _params(bx, True)
        opos = srd.stream(bx["pos"], bx["vel"], p)
        cell = srd.bin_cells(opos, srd.grid_shift(p, 0), p)
        count, M, P, u, ek = srd.cell_sums(cell, bx["vel"], np.ones(n), p.ncells)
        cs = slice(c0, c0 + nc)
        assert np.array_equal(gm[cs], M)
        assert np.max(np.abs(gP[cs] - P)) < 1e-13
        assert np.allclose(gek[cs], ek, rtol=1e-12, atol=1e-14)
        occ = count > 0
        ax = srd.cell_axes(np.arange(p.ncells), 0, p)
        assert np.max(np.abs(gax[cs][occ] - ax[occ])) < 1e-15
        xi = srd.thermostat_xi(count, ek, np.arange(p.ncells, dtype=np.uint64), 0, p)
        assert np.allclose(gxi[cs], xi, rtol=1e-12, atol=0)


def test_batch_of_one_equals_single_box():
    banner("batch of one == single box")
    bx = _inputs(BOXES[2:3])[0]
    with m.Batch([bx], precision=m.FP64, thermostat=True) as bt:
        bt.step(4)
        bpos, bvel = bt.get_state()
    with m.Sim(bx["pos"], bx["vel"], bx["n_cells"], seed=bx["seed"], kT=bx["kT"],
               precision=m.FP64, thermostat=True) as s:
        s.step(4)
        spos, svel = s.get_state()
    assert np.array_equal(bpos, spos) and np.array_equal(bvel, svel)


@pytest.mark.parametrize("form", ["fp64", "fp32"])
def test_batch_velocity_field(form):
    """Cell-averaged velocity field (unshifted grid) of every box after two
    steps, against the oracle's field of the same state."""
    banner(f"batch velocity field {form}")
    boxes = _inputs(BOXES)
    prec = m.FP64 if form == "fp64" else m.FP32
    with m.Batch(boxes, precision=prec, thermostat=True) as bt:
        bt.step(2)
        gpos, gvel = bt.get_state()
        gu, gM = bt.velocity_field()
        info = [bt.box(b) for b in range(len(boxes))]
    for b, bx in enumerate(boxes):
        t0, n, c0, nc, _ = info[b]
        p = _params(bx, True)
        sl, cs = slice(t0, t0 + n), slice(c0, c0 + nc)
        # the oracle's field of the GPU's own state: exact sums, so only the
        # final division rounds
        u, M = srd.velocity_field(gpos[sl], gvel[sl], np.ones(n), p)
        assert np.array_equal(gM[cs], M)
        assert np.max(np.abs(gu[cs] - u)) < 1e-14 * max(1.0, np.abs(u).max())


def test_velocity_field_with_beads():
    banner("velocity field with beads")
    p = srd.Params((10, 9, 8), seed=31, thermostat=False)
    pos, vel = workloads.fluid(p.n_cells, 5, seed=32)
    bpos, bvel, bmass = workloads.beads(p.n_cells, 4, 10, seed=33)
    with m.Sim(pos, vel, p.n_cells, seed=p.seed, emb_pos=bpos, emb_vel=bvel, emb_mass=bmass) as s:
        s.step(1)
        gpos, gvel = s.get_state()
        gu, gM = s.velocity_field()
    mass = np.concatenate([np.ones(pos.shape[0]), bmass])
    u, M = srd.velocity_field(gpos, gvel, mass, p)
    assert np.array_equal(gM, M)
    assert np.max(np.abs(gu - u)) < 1e-14 * max(1.0, np.abs(u).max())
