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


def test_md_exchange_on_device_buffers():
    """The exchange through device buffers gives the host-array exchange's
    results bit for bit (pointers_on_device = 1)."""
    import torch
    banner("md exchange on device buffers")
    p = srd.Params((8, 8, 8), seed=77, thermostat=True)
    pos, vel = workloads.fluid(p.n_cells, 6, seed=78)
    bpos, bvel, bmass = workloads.beads(p.n_cells, 3, 8, seed=79)
    kw = dict(seed=p.seed, thermostat=True, emb_pos=bpos, emb_vel=bvel, emb_mass=bmass,
              flags=m.binding.FLAG_MD_SOLUTE)
    with m.Sim(pos, vel, p.n_cells, **kw) as a, m.Sim(pos, vel, p.n_cells, **kw) as b:
        dpos = torch.empty((bpos.shape[0], 3), dtype=torch.float64, device="cuda")
        dvel = torch.empty_like(dpos)
        hp, hv = bpos.copy(), bvel.copy()
        for _ in range(3):
            hp = (hp + 0.05) % p.L            # stands in for the integrator's move
            dpos.copy_(torch.from_numpy(hp))
            dvel.copy_(torch.from_numpy(hv))
            torch.cuda.synchronize()
            a.set_embedded(hp, hv)
            a.step(1)
            hp, hv = a.get_embedded()
            b.set_embedded_device(dpos.data_ptr(), dvel.data_ptr())
            b.step(1)
            b.get_embedded_device(dpos.data_ptr(), dvel.data_ptr())
            assert np.array_equal(dpos.cpu().numpy(), hp)
            assert np.array_equal(dvel.cpu().numpy(), hv)
        pa, va = a.get_state()
        pb, vb = b.get_state()
    assert np.array_equal(pa, pb) and np.array_equal(va, vb)
