"""Galilean invariance of the HIP path (sec. 2), FP64 form, through the C ABI.

Two runs of the same fluid, one flowing at -V0/2 and one at +V0/2 with
V0 = L / dt per axis (every displacement stays below one box length per
step): the particles of the two runs are one box apart after every step, so
the periodic positions, the cells and the per-cell random numbers are the
same, and the velocities stay V0 apart to the rounding of the boosted sums.
Each run also matches the oracle at the FP64 bar (|V0 / 2| ~ 1e2 is inside
the FP64 form's fixed-point range of 2^30 per term).
"""
import numpy as np
import pytest

import paper_1801_10187_amd as m
import workloads
from helpers import banner, periodic_dist, vel_err_fp64, FP64_REL
from oracle import srd

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("thermo", [False, True])
def test_boost_by_box_per_step_gpu_fp64(thermo):
    n_cells, steps = (20, 20, 20), 20
    banner(f"galilean boost fp64 thermo={thermo} {n_cells} {steps} steps")
    p = srd.Params(n_cells, seed=31, thermostat=thermo)
    V0 = p.L / p.dt
    assert np.array_equal(V0 * p.dt, p.L)
    pos, vel = workloads.fluid(n_cells, 5, seed=32)
    mass = np.ones(pos.shape[0])
    out = {}
    for name, v in (("minus", vel - 0.5 * V0), ("plus", vel + 0.5 * V0)):
        with m.Sim(pos, v, n_cells, seed=p.seed, thermostat=thermo, precision=m.FP64) as s:
            s.step(steps)
            gpos, gvel = s.get_state()
            gcells, gcounts = s.get_cells()
        opos, ovel, info = srd.run(pos, v, mass, p, 0, steps)
        assert np.array_equal(gcells, info["cell"])
        assert vel_err_fp64(gvel, ovel) < FP64_REL
        assert periodic_dist(gpos, opos, p.L).max() < 1e-12
        out[name] = (gpos, gvel, gcells, gcounts)
    (pa, va, ca, na), (pb, vb, cb, nb) = out["minus"], out["plus"]
    assert np.array_equal(ca, cb) and np.array_equal(na, nb)
    assert periodic_dist(pa, pb, p.L).max() < 1e-12
    assert np.abs(vb - va - V0).max() < 1e-12
