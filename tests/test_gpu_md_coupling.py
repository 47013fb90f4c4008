"""Solutes moved by an external MD integrator between collisions and coupled
to the solvent only in the collision (sec. 3.6; MPCD_FLAG_MD_SOLUTE with
mpcd_set_embedded / mpcd_get_embedded), against the oracle doing the same
sequence: MD for one collision time, stream the solvent only, collide all."""
import numpy as np
import pytest

import paper_1801_10187_amd as m
import workloads
from helpers import FP64_REL, banner, periodic_dist, vel_err_fp64
from md_chain import verlet
from oracle import srd

pytestmark = pytest.mark.gpu


def test_md_coupled_chains_match_the_oracle():
    banner("md-coupled chains")
    p = srd.Params((10, 10, 10), seed=71, thermostat=True, kT=1.0)
    chains, clen = 6, 12
    pos, vel = workloads.fluid(p.n_cells, 6, seed=72)
    bpos, bvel, bmass = workloads.beads(p.n_cells, chains, clen, seed=73)
    ns = pos.shape[0]
    mass = np.concatenate([np.ones(ns), bmass])
    moving = np.concatenate([np.ones(ns, bool), np.zeros(bpos.shape[0], bool)])
    nsub, cycles = 10, 4
    # GPU: MD on the host, collisions on the device
    gb_pos, gb_vel = bpos.copy(), bvel.copy()
    with m.Sim(pos, vel, p.n_cells, seed=p.seed, kT=p.kT, thermostat=True, emb_pos=bpos,
               emb_vel=bvel, emb_mass=bmass, flags=m.binding.FLAG_MD_SOLUTE) as s:
        for c in range(cycles):
            gb_pos, gb_vel = verlet(gb_pos, gb_vel, bmass, clen, p.L, p.dt / nsub, nsub)
            s.set_embedded(gb_pos, gb_vel)
            s.step(1)
            gb_pos, gb_vel = s.get_embedded()
        gpos, gvel = s.get_state()
    # oracle: the same sequence
    opos, ovel = np.concatenate([pos, bpos]), np.concatenate([vel, bvel])
    for c in range(cycles):
        ob_pos, ob_vel = verlet(opos[ns:], ovel[ns:], bmass, clen, p.L, p.dt / nsub, nsub)
        opos = np.concatenate([opos[:ns], ob_pos])
        ovel = np.concatenate([ovel[:ns], ob_vel])
        opos, ovel, _ = srd.srd_step(opos, ovel, mass, p, c, moving=moving)
    assert vel_err_fp64(gvel[:ns], ovel[:ns]) < FP64_REL
    assert periodic_dist(gpos[:ns], opos[:ns], p.L).max() < 1e-12
    # beads: the MD amplifies the 1e-16 differences of the collision a little
    assert np.abs(gb_vel - ovel[ns:]).max() < 1e-10
    assert periodic_dist(gb_pos, opos[ns:], p.L).max() < 1e-10
    assert np.array_equal(gpos[ns:], gb_pos)


def test_md_solutes_are_not_streamed():
    banner("md solutes not streamed")
    p = srd.Params((6, 6, 6), seed=74)
    pos, vel = workloads.fluid(p.n_cells, 5, seed=75)
    bpos, bvel, bmass = workloads.beads(p.n_cells, 2, 5, seed=76)
    with m.Sim(pos, vel, p.n_cells, seed=p.seed, emb_pos=bpos, emb_vel=bvel, emb_mass=bmass,
               flags=m.binding.FLAG_MD_SOLUTE) as s:
        s.step(3)
        ep, ev = s.get_embedded()
        assert np.array_equal(ep, bpos)          # positions untouched by MPCD
        assert not np.array_equal(ev, bvel)      # velocities changed by collisions
        s.stream()
        with pytest.raises(m.MpcdError):
            s.set_embedded(ep, ev)                # only between steps
        s.bin()
        s.collide()
        bad = ep.copy()
        bad[0, 0] = -1.0
        with pytest.raises(m.MpcdError):
            s.set_embedded(bad, ev)
