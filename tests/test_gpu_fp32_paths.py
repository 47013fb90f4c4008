"""The FP32 storage form on the kernels' less common paths, through the C
ABI: tiles holding more particles than a block keeps in registers (768 in a
64-cell tile, 1024 in a 128-cell one; the rest are read again from the slab),
under the SRD rule with the thermostat and under the AT rule (eq. 4); and the
enlarge-and-replay path after a slab overflow. Every step is checked element
by element against the emulation of that step from the GPU's state before it
(cells and positions bit-exact, velocities within one ulp; the AT rule's
kick sums allow 2^-40 absolute for results within ~1e-6 of zero, sec. 3.7).
"""
import numpy as np
import pytest

import paper_1801_10187_amd as m
import workloads
from helpers import (FP64_REL, at32_close, banner, fp32_step_matches, ulp_diff_f32,
                     vel_err_fp64)
from oracle import fp32form, srd

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _lib():
    m.load()


# box, particles in one crowded cell, particles spread over the box, the
# tile shape (set through the flags: the AT rule's density rule never picks
# 8x4x4) and the register-resident part per tile
CROWD = {"cpt64": ((4, 4, 4), 3000, 500, (4, 4, 2), 768),
         "cpt128": ((8, 8, 8), 1100, 900, (8, 4, 4), 1024)}


def _crowd(layout, seed):
    n_cells, n_crowd, n_rest, _, _ = CROWD[layout]
    rng = np.random.default_rng(seed)
    crowd = 2.2 + 0.6 * rng.random((n_crowd, 3))
    rest = rng.random((n_rest, 3)) * np.array(n_cells, dtype=np.float64)
    pos = np.concatenate([crowd, rest])
    vel = rng.normal(size=pos.shape) * 0.5
    return pos, vel - vel.mean(axis=0)


def _sim(pos, vel, p, prec, **kw):
    return m.Sim(pos, vel, p.n_cells, seed=p.seed, kT=p.kT, dt=p.dt, precision=prec,
                 thermostat=p.thermostat, grid_shift=p.grid_shift,
                 collision=m.AT if p.rule == "at" else m.SRD, **kw)


def _step_matches_at(gpos0, gvel0, gpos1, gvel1, gcells1, mass, p, step):
    """fp32_step_matches with the AT rule's bar (at32_close: one ulp plus the
    single-precision rounding of the kicks)."""
    h, o, v = fp32form.from_double(gpos0, gvel0, p)
    assert np.array_equal(fp32form.to_double(h, o, p), gpos0)
    h1, o1, v1, info = fp32form.step32(h, o, v, mass, p, step)
    assert np.array_equal(gcells1, info["cell"])
    assert np.array_equal(gpos1, fp32form.to_double(h1, o1, p))
    assert np.all(at32_close(gvel1, v1, info))


@pytest.mark.parametrize("layout", sorted(CROWD))
@pytest.mark.parametrize("rule", ["srd_thermo", "at"])
def test_fp32_crowded_tile(rule, layout):
    """Two single-step calls of a box with one crowded cell, each checked
    against the emulation from the GPU's state before it."""
    n_cells, _, _, tile, treg = CROWD[layout]
    banner(f"fp32 crowded tile {rule} {layout}")
    p = srd.Params(n_cells, seed=91, thermostat=rule == "srd_thermo", grid_shift=False,
                   dt=0.01, rule="at" if rule == "at" else "srd")
    pos, vel = _crowd(layout, 92)
    mass = np.ones(pos.shape[0])
    check = fp32_step_matches if rule == "srd_thermo" else (
        lambda *a: _step_matches_at(*a[:-1]))
    with _sim(pos, vel, p, m.FP32, tile="x".join(map(str, tile))) as s:
        assert s.layout()[0] == tile
        gpos, gvel = s.get_state()
        for k in range(2):
            s.step(1)
            gpos1, gvel1 = s.get_state()
            gcells1, counts = s.get_cells()
            # the occupancy of the crowded cell's tile exceeds what the block
            # holds in registers
            assert counts.max() > treg
            check(gpos, gvel, gpos1, gvel1, gcells1, mass, p, k, fp32form)
            gpos, gvel = gpos1, gvel1


@pytest.mark.parametrize("rule", ["srd_thermo", "at"])
def test_fp64_crowded_128_cell_tile(rule):
    """The FP64 form on the same 128-cell-tile box: two fused steps within
    1e-12 of the oracle."""
    n_cells, _, _, tile, treg = CROWD["cpt128"]
    banner(f"fp64 crowded 128-cell tile {rule}")
    p = srd.Params(n_cells, seed=93, thermostat=rule == "srd_thermo", grid_shift=False,
                   dt=0.01, rule="at" if rule == "at" else "srd")
    pos, vel = _crowd("cpt128", 94)
    with _sim(pos, vel, p, m.FP64, tile="x".join(map(str, tile))) as s:
        assert s.layout()[0] == tile
        s.step(2)
        _, gvel = s.get_state()
        _, counts = s.get_cells()
    assert counts.max() > treg
    _, ovel, _ = srd.run(pos, vel, np.ones(pos.shape[0]), p, 0, 2)
    assert vel_err_fp64(gvel, ovel) < FP64_REL


def _converging(seed):
    p = srd.Params((12, 12, 12), seed=seed, thermostat=True)
    pos, vel = workloads.fluid(p.n_cells, 9, seed=seed + 1)
    vel = vel - (pos - p.L / 2)          # up to 0.6 cells per step inwards
    return p, pos, vel


def test_fp32_slab_regrow_each_step():
    """A converging flow overflows slabs sized to the initial maximum
    occupancy; the library enlarges them and replays the launch. Four
    single-step calls, each checked against the emulation from the GPU's
    state before it."""
    banner("fp32 slab regrow, each step")
    p, pos, vel = _converging(95)
    mass = np.ones(pos.shape[0])
    with _sim(pos, vel, p, m.FP32, flags=m.binding.FLAG_TIGHT_SLABS) as s:
        cap0 = s.layout()[2]
        gpos, gvel = s.get_state()
        for k in range(4):
            s.step(1)
            gpos1, gvel1 = s.get_state()
            gcells1, _ = s.get_cells()
            fp32_step_matches(gpos, gvel, gpos1, gvel1, gcells1, mass, p, k, fp32form)
            gpos, gvel = gpos1, gvel1
        _, _, cap1, regrows = s.layout()
    assert regrows >= 1 and cap1 > cap0


def test_fp32_slab_regrow_fused_equals_single_steps():
    """The same overflow inside one four-step call (the replay starts from
    the failing launch of the call) gives the single-step calls' result bit
    for bit."""
    banner("fp32 slab regrow, fused call")
    p, pos, vel = _converging(95)
    with _sim(pos, vel, p, m.FP32, flags=m.binding.FLAG_TIGHT_SLABS) as s:
        s.step(4)
        fpos, fvel = s.get_state()
        regrows = s.layout()[3]
    with _sim(pos, vel, p, m.FP32, flags=m.binding.FLAG_TIGHT_SLABS) as s:
        for _ in range(4):
            s.step(1)
        spos, svel = s.get_state()
    assert regrows >= 1
    assert np.array_equal(fpos, spos)
    assert ulp_diff_f32(fvel.astype(np.float32), svel.astype(np.float32)).max() == 0
