"""Full-size check of the largest single-GPU workload: the 400^3-cell fluid
at 5 particles per cell (3.2 x 10^8 solvent particles) with 20 000 chains of
50 mass-5 beads, FP32 form, no thermostat. The oracle cannot step 3.2 x 10^8
particles, so one GPU step is checked on sampled regions, each against the
oracle's FP32 emulation of the particles that can reach it, and the whole
system through properties that hold at any size."""
import numpy as np
import pytest

import paper_1801_10187_amd as m
import workloads
from helpers import banner, ulp_diff_f32
from oracle import fp32form, srd

pytestmark = pytest.mark.gpu

MARGIN = 2   # cells around a sampled block from which particles can enter it
BLOCK = 4    # sampled block edge, in cells


def _region_mask(home, lo, edge, n):
    """Particles whose home cell lies in the periodic block [lo, lo + edge)^3."""
    mask = np.ones(home.shape[0], dtype=bool)
    for d in range(3):
        mask &= ((home[:, d] - lo[d]) % n[d]) < edge
    return mask


def test_large_box_with_beads_one_step_sampled():
    cfg = workloads.CONFIGS["srd_400c_rho5_beads"]
    banner("large box 400^3 rho=5 + beads, fp32, one step")
    n = np.array(cfg["n_cells"])
    p = srd.Params(cfg["n_cells"], seed=cfg["seed"], thermostat=False, kT=cfg["kT"])
    pos, vel = workloads.fluid(cfg["n_cells"], cfg["density"], kT=cfg["kT"], seed=cfg["seed"])
    bpos, bvel, bmass = workloads.beads(cfg["n_cells"], cfg["chains"], cfg["chain_len"],
                                        kT=cfg["kT"], mass=cfg["bead_mass"],
                                        seed=cfg["seed"] + 1)
    ns = pos.shape[0]
    N = ns + bpos.shape[0]
    allpos = np.concatenate([pos, bpos])
    allvel = np.concatenate([vel, bvel])
    del pos, vel
    mass = np.concatenate([np.full(ns, 1.0), bmass])
    # no particle moves a cell or more in one step, so a margin of two
    # cells around a block holds everything that can land in it
    assert np.abs(allvel).max() * p.dt < 1.0

    with m.Sim(allpos[:ns], allvel[:ns], cfg["n_cells"], seed=cfg["seed"], kT=cfg["kT"],
               precision=m.FP32, thermostat=False, emb_pos=bpos, emb_vel=bvel,
               emb_mass=bmass) as s:
        P0, _, _ = s.totals()
        s.step(1)
        P1, _, _ = s.totals()
        gpos, gvel = s.get_state()
        gcells, gcounts = s.get_cells()

    # whole system: every particle binned once; the collision conserves
    # momentum up to the final rounding of each velocity to FP32 (random
    # errors of 2^-24 |v| per component: about sqrt(N) 2^-24 = 1e-3 in total)
    assert gcounts.sum() == N
    assert np.abs(P1 - P0).max() < 0.05
    assert np.all(np.isfinite(gvel))

    # sampled blocks, one of them across the periodic corner of the box
    rng = np.random.default_rng(7)
    starts = [np.array([n[0] - 2, n[1] - 2, n[2] - 2])] + \
             [rng.integers(0, n) for _ in range(3)]
    home = np.floor(allpos * p.inv_a).astype(np.int32)
    shift = srd.grid_shift(p, 0)
    checked = 0
    for lo in starts:
        cand = np.flatnonzero(_region_mask(home, (lo - MARGIN) % n, BLOCK + 2 * MARGIN, n))
        h, o, v = fp32form.from_double(allpos[cand], allvel[cand], p)
        h, o = fp32form.stream32(h, o, v, p)
        cell = fp32form.bin32(h, o, shift, p)
        c3 = np.stack([cell % n[0], (cell // n[0]) % n[1], cell // (n[0] * n[1])], axis=1)
        inside = np.ones(cand.size, dtype=bool)
        for d in range(3):
            inside &= ((c3[:, d] - lo[d]) % n[d]) < BLOCK
        sel = cand[inside]
        assert sel.size > 0.5 * cfg["density"] * BLOCK ** 3
        # the block's cells hold exactly these particles on the GPU too
        assert np.array_equal(gcells[sel], cell[inside])
        cells_u, local = np.unique(cell[inside], return_inverse=True)
        assert gcounts[cells_u].sum() == sel.size
        # oracle collision of the block's cells (FP64 on the FP32 values)
        v64 = v[inside].astype(np.float64)
        count, M, P, u, ek = srd.cell_sums(local, v64, mass[sel], cells_u.size)
        axis = srd.cell_axes(cells_u.astype(np.uint64), 0, p)
        vnew = srd.rotate(v64, local, u, axis, np.ones(cells_u.size), p).astype(np.float32)
        assert ulp_diff_f32(gvel[sel].astype(np.float32), vnew).max() <= 1
        assert np.array_equal(gpos[sel], fp32form.to_double(h[inside], o[inside], p))
        checked += sel.size
    assert checked > 1000
