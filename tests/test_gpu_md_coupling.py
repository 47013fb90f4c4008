"""Solutes moved by an external MD integrator between collisions and coupled
to the solvent only in the collision (sec. 3.6; MPCD_FLAG_MD_SOLUTE with
mpcd_set_embedded / mpcd_get_embedded), against the oracle doing the same
sequence: MD for one collision time, stream the solvent only, collide all.
A handover after mpcd_step moves the solutes into the prepared binning of
the next step (O(solutes)); it must give what binning everything afresh
gives, bit for bit, also when solutes jump across the box, crowd into one
tile, or overflow a slab (the prepared binning is then given up)."""
import numpy as np
import pytest

import paper_1801_10187_amd as m
import workloads
from helpers import FP64_REL, banner, f32_close, periodic_dist, vel_err_fp64
from md_chain import verlet
from oracle import fp32form, srd

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
        # every handover after the first step went into the prepared binning
        assert s.handover_stats() == (cycles - 1, 0)
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


def _jumping_run(prec, n_cells, rho, nb, seed, cycles, fresh, crowd_at=None, thermo=True,
                 collision=m.SRD):
    """MD-flagged context whose solutes jump to new random places before each
    collision (crowd_at: the cycle from which all of them sit in one cell).
    fresh: before each handover the prepared binning is given up (a step
    counter changed and restored), so the next step bins everything."""
    rng = np.random.default_rng(seed)
    L = np.array(n_cells, dtype=np.float64)
    pos, vel = workloads.fluid(n_cells, rho, seed=seed + 1)
    bpos = rng.random((nb, 3)) * L
    bvel = rng.normal(size=(nb, 3)) * 0.4
    bmass = np.full(nb, 3.0)
    with m.Sim(pos, vel, n_cells, seed=seed + 2, thermostat=thermo and collision == m.SRD,
               precision=prec, collision=collision, emb_pos=bpos, emb_vel=bvel, emb_mass=bmass,
               flags=m.binding.FLAG_MD_SOLUTE) as s:
        for c in range(cycles):
            if crowd_at is not None and c >= crowd_at:
                hp = 2.0 + 0.999 * rng.random((nb, 3))
            else:
                hp = rng.random((nb, 3)) * L
            hv = rng.normal(size=(nb, 3)) * 0.4
            if fresh:
                s.step_count = s.step_count + 1
                s.step_count = s.step_count - 1
            s.set_embedded(hp, hv)
            s.step(1)
            ep, _ = s.get_embedded()
            if prec == m.FP64:
                assert np.array_equal(ep, hp)      # solutes are not streamed
        st = s.get_state()
        cells = s.get_cells()
        return st, cells, s.handover_stats(), s.layout()[3]


@pytest.mark.parametrize("prec,collision", [(m.FP64, m.SRD), (m.FP32, m.SRD), (m.FP32, m.AT)])
def test_handover_jumping_solutes_equal_fresh_binning(prec, collision):
    """300 solutes jumping anywhere in a 10^3 box every cycle (most change
    tile, several leave or enter one tile at once): six cycles with the
    handover give the state of the same cycles binned afresh, bit for bit
    (both forms; the AT rule too)."""
    banner(f"handover, jumping solutes, prec {prec} rule {collision}")
    a = _jumping_run(prec, (10, 10, 10), 6.0, 300, 81, 6, fresh=False, collision=collision)
    b = _jumping_run(prec, (10, 10, 10), 6.0, 300, 81, 6, fresh=True, collision=collision)
    for x, y in zip(a[0] + a[1], b[0] + b[1]):
        assert np.array_equal(x, y)
    assert a[2] == (5, 0) and b[2] == (0, 0)


def test_handover_full_slab_gives_the_binning_up():
    """From the third cycle all 600 solutes are put into one cell, more than
    its tile's slab holds beside the solvent: that handover gives the
    prepared binning up (the next step enlarges the slabs), the later ones
    fit again; results equal the fresh binning's bit for bit."""
    banner("handover, full slab")
    a = _jumping_run(m.FP64, (8, 8, 8), 5.0, 600, 85, 5, fresh=False, crowd_at=2)
    b = _jumping_run(m.FP64, (8, 8, 8), 5.0, 600, 85, 5, fresh=True, crowd_at=2)
    for x, y in zip(a[0] + a[1], b[0] + b[1]):
        assert np.array_equal(x, y)
    kept, given_up = a[2]
    assert given_up == 1 and kept == 3
    assert a[3] >= 1     # the slabs were enlarged


def test_md_coupled_chains_fp32_each_cycle():
    """The FP32 form with MD-coupled chains: every cycle (handover into the
    prepared binning, one step) checked element by element against the FP32
    emulation of that step from the GPU's state after the handover (solvent
    streamed, solutes not): cells and positions bit-exact, velocities within
    one ulp or 2^-40."""
    banner("md-coupled chains, fp32, each cycle")
    p = srd.Params((10, 10, 10), seed=86, thermostat=True, kT=1.0)
    chains, clen = 6, 12
    pos, vel = workloads.fluid(p.n_cells, 6, seed=87)
    bpos, bvel, bmass = workloads.beads(p.n_cells, chains, clen, seed=88)
    ns = pos.shape[0]
    mass = np.concatenate([np.ones(ns), bmass])
    gb_pos, gb_vel = bpos.copy(), bvel.copy()
    with m.Sim(pos, vel, p.n_cells, seed=p.seed, kT=p.kT, thermostat=True, precision=m.FP32,
               emb_pos=bpos, emb_vel=bvel, emb_mass=bmass,
               flags=m.binding.FLAG_MD_SOLUTE) as s:
        for c in range(5):
            gb_pos, gb_vel = verlet(gb_pos, gb_vel, bmass, clen, p.L, p.dt / 10, 10)
            s.set_embedded(gb_pos, gb_vel)
            gpos0, gvel0 = s.get_state()
            s.step(1)
            gpos1, gvel1 = s.get_state()
            gcells1, _ = s.get_cells()
            h, o, v = fp32form.from_double(gpos0, gvel0, p)
            assert np.array_equal(fp32form.to_double(h, o, p), gpos0)
            hs, os_ = fp32form.stream32(h[:ns], o[:ns], v[:ns], p)
            h1 = np.concatenate([hs, h[ns:]])
            o1 = np.concatenate([os_, o[ns:]])
            v1, info = fp32form.collide32(h1, o1, v, mass, p, c)
            assert np.array_equal(gcells1, info["cell"])
            assert np.array_equal(gpos1, fp32form.to_double(h1, o1, p))
            assert np.all(f32_close(gvel1, v1))
            gb_pos, gb_vel = s.get_embedded()
        assert s.handover_stats() == (4, 0)


def _device_chains(bpos, bvel, bmass):
    import torch
    return (torch.from_numpy(bpos.copy()).cuda(), torch.from_numpy(bvel.copy()).cuda(),
            torch.from_numpy(bmass.copy()).cuda())


@pytest.mark.parametrize("clen,chains", [(12, 6), (50, 40), (64, 3), (100, 2)])
def test_device_verlet_equals_host_integrator(clen, chains):
    """mpcd_md_verlet_chains (sec. 3.6 / 4.3: 50 velocity-Verlet steps of
    0.002 per collision) against the host integrator of the tests, bit for
    bit: both do the same IEEE operations in the same order."""
    import torch
    banner(f"device verlet, {chains} chains of {clen}")
    L = np.array([9.0, 11.0, 10.0])
    bpos, bvel, bmass = workloads.beads((9, 11, 10), chains, clen, seed=90 + clen)
    hp, hv = verlet(bpos, bvel, bmass, clen, L, 0.002, 50)
    dp, dv, dm = _device_chains(bpos, bvel, bmass)
    m.binding.md_verlet_chains(dp.data_ptr(), dv.data_ptr(), dm.data_ptr(), chains, clen, L,
                               0.002, 50, hip_stream=torch.cuda.current_stream().cuda_stream)
    gp, gv = dp.cpu().numpy(), dv.cpu().numpy()
    print(f"max |dpos| {np.abs(gp - hp).max():.3g}, max |dvel| {np.abs(gv - hv).max():.3g}")
    assert np.array_equal(gp, hp) and np.array_equal(gv, hv)


def test_coupled_cycle_on_device_equals_host_cycle():
    """The whole coupled cycle on the device (integrator, handover, step,
    read back, all on one stream) equals the cycle with the host integrator
    and host arrays, bit for bit."""
    import torch
    banner("coupled cycle on device")
    p = srd.Params((10, 10, 10), seed=97, thermostat=True)
    clen, chains = 12, 6
    pos, vel = workloads.fluid(p.n_cells, 6, seed=98)
    bpos, bvel, bmass = workloads.beads(p.n_cells, chains, clen, seed=99)
    kw = dict(seed=p.seed, thermostat=True, emb_pos=bpos, emb_vel=bvel, emb_mass=bmass,
              flags=m.binding.FLAG_MD_SOLUTE)
    with m.Sim(pos, vel, p.n_cells, **kw) as s:
        hp, hv = bpos.copy(), bvel.copy()
        for _ in range(4):
            hp, hv = verlet(hp, hv, bmass, clen, p.L, 0.002, 50)
            s.set_embedded(hp, hv)
            s.step(1)
            hp, hv = s.get_embedded()
        want = s.get_state()
    # one stream for the integrator and the context (torch's default stream
    # has handle 0, for which the context would create a stream of its own)
    ts = torch.cuda.Stream()
    stream = ts.cuda_stream
    dp, dv, dm = _device_chains(bpos, bvel, bmass)
    torch.cuda.synchronize()
    with m.Sim(pos, vel, p.n_cells, hip_stream=stream, **kw) as s:
        for _ in range(4):
            m.binding.md_verlet_chains(dp.data_ptr(), dv.data_ptr(), dm.data_ptr(), chains, clen,
                                       p.L, 0.002, 50, hip_stream=stream)
            s.set_embedded_device(dp.data_ptr(), dv.data_ptr())
            s.step(1)
            s.get_embedded_device(dp.data_ptr(), dv.data_ptr())
        got = s.get_state()
        assert s.handover_stats() == (3, 0)
    assert np.array_equal(want[0], got[0]) and np.array_equal(want[1], got[1])


def test_device_verlet_rejects_bad_arguments():
    with pytest.raises(m.MpcdError):
        m.binding.md_verlet_chains(0, 0, 0, 1, 0, (5, 5, 5), 0.002, 1)
    with pytest.raises(m.MpcdError):
        m.binding.md_verlet_chains(0, 0, 0, 1, 2000, (5, 5, 5), 0.002, 1)
    with pytest.raises(m.MpcdError):
        m.binding.md_verlet_chains(0, 0, 0, 1, 10, (5, 0, 5), 0.002, 1)
    m.binding.md_verlet_chains(0, 0, 0, 0, 10, (5, 5, 5), 0.002, 1)   # nothing to do
