"""Galilean invariance of the oracle's SRD step, and what the random grid
shift is for (sec. 2: without the shift the rule is not Galilean invariant
when the mean free path is small against the cell size; shifting the grid by
a random vector every step restores it).

* Exact: two runs whose velocities differ by V0 = L / dt per axis move every
  particle by exactly one box length apart per step, so after the periodic
  wrap the positions, the cells and every random number are the same, and
  the velocities stay V0 apart, to the rounding of the boosted sums (|V0| ~
  1e2 times the FP64 epsilon per step). The two runs are a fluid flowing at
  -V0/2 and the same fluid at +V0/2, so that every displacement stays below
  one box length per step, as streaming requires. This holds over many
  streamed and collided steps, with and without the thermostat (its scale
  factor depends only on velocities relative to the cell mean).
* Statistical: a transverse shear wave u_x = A sin(k z) decays at a rate
  nu k^2. With the shift, a uniform flow V0 along z only advects the wave, so
  the decay rate is the same with and without the flow. Without the shift,
  at mean free path lambda = dt sqrt(kT/m) = 0.1 a, particles keep meeting
  the same cell-mates; a flow along z carries them across cell faces and
  changes the rate by far more than its statistical error.
"""
import math

import numpy as np
import pytest

import workloads
from oracle import srd


def _boost_runs(n_cells, dt, thermo, steps, seed):
    p = srd.Params(n_cells, dt=dt, seed=seed, thermostat=thermo)
    V0 = p.L / p.dt
    assert np.array_equal(V0 * p.dt, p.L), "V0 dt must equal L exactly"
    pos, vel = workloads.fluid(n_cells, 5, seed=seed + 1)
    mass = np.ones(pos.shape[0])
    pa, va, pb, vb = pos, vel - 0.5 * V0, pos, vel + 0.5 * V0
    for s in range(steps):
        pa, va, ia = srd.srd_step(pa, va, mass, p, s)
        pb, vb, ib = srd.srd_step(pb, vb, mass, p, s)
        yield p, V0, (pa, va, ia), (pb, vb, ib)


@pytest.mark.parametrize("n_cells,dt,thermo", [((20, 20, 20), 0.1, False),
                                               ((6, 9, 7), 0.1, True),
                                               ((8, 5, 12), 0.125, True)])
def test_boost_by_box_per_step_reproduces_the_trajectory(n_cells, dt, thermo):
    worst_v = worst_x = 0.0
    for p, V0, (pa, va, ia), (pb, vb, ib) in _boost_runs(n_cells, dt, thermo, 20, 7):
        # the same cells (no particle comes within rounding of a face here)
        assert np.array_equal(ia["cell"], ib["cell"])
        assert np.array_equal(ia["count"], ib["count"])
        d = np.abs(pa - pb)
        worst_x = max(worst_x, np.minimum(d, p.L - d).max())
        worst_v = max(worst_v, np.abs(vb - V0 - va).max())
    # each step rounds the boosted velocity at |V0| ~ 200: ulp 2.8e-14
    assert worst_x < 1e-12
    assert worst_v < 1e-12


def test_boost_changes_the_trajectory_unless_it_is_a_whole_box():
    """Control: a boost by half of L / dt is a different trajectory (the
    exact match above is not trivially true)."""
    p = srd.Params((10, 10, 10), seed=3)
    pos, vel = workloads.fluid(p.n_cells, 5, seed=4)
    mass = np.ones(pos.shape[0])
    _, _, ia = srd.srd_step(pos, vel, mass, p, 0)
    _, _, ib = srd.srd_step(pos, vel + 0.5 * p.L / p.dt, mass, p, 0)
    assert not np.array_equal(ia["cell"], ib["cell"])


def _mode(pos, vel, k):
    """Complex amplitude of u_x(z): 2 <v_x exp(-i k z)>. Its modulus does
    not change when a uniform flow along z advects the wave."""
    return 2.0 * np.mean(vel[:, 0] * np.exp(-1j * k * pos[:, 2]))


def _decay_rate(shift, V0, seed, n=(6, 6, 16), rho=10, A=0.3, steps=60, every=5):
    p = srd.Params(n, seed=100 + seed, grid_shift=shift)
    k = 2.0 * math.pi / (n[2] * p.a)
    pos, vel = workloads.fluid(n, rho, seed=seed)
    vel[:, 0] += A * np.sin(k * pos[:, 2])
    vel -= vel.mean(axis=0)
    vel[:, 2] += V0
    mass = np.ones(pos.shape[0])
    t, amp = [0.0], [abs(_mode(pos, vel, k))]
    for s in range(steps):
        pos, vel, _ = srd.srd_step(pos, vel, mass, p, s)
        if (s + 1) % every == 0:
            t.append((s + 1) * p.dt)
            amp.append(abs(_mode(pos, vel, k)))
    return -np.polyfit(np.array(t), np.log(np.array(amp)), 1)[0]


def test_shift_makes_shear_wave_decay_independent_of_a_uniform_flow():
    """Paired seeds (same particles, same random numbers), 16 of them, with
    and without a flow of 2.5 sqrt(kT/m) along z. Shift on: the rate changes
    by less than 3 standard errors; shift off: by more than 8 (measured
    0.010 +- 0.010 against 0.080 +- 0.005). With the shift the rate also
    matches the paper's viscosity for this fluid (8.7, sec. 4):
    nu = eta / rho = 0.87, rate nu k^2 = 0.134 for k = 2 pi / 16."""
    k = 2.0 * math.pi / 16
    seeds = range(16)
    res = {}
    for shift in (True, False):
        still = np.array([_decay_rate(shift, 0.0, s) for s in seeds])
        moving = np.array([_decay_rate(shift, 2.5, s) for s in seeds])
        d = moving - still
        res[shift] = (still.mean(), d.mean(), d.std(ddof=1) / math.sqrt(len(d)))
    (r_on, d_on, e_on), (r_off, d_off, e_off) = res[True], res[False]
    print(f"shift on: rate {r_on:.4f}, flow changes it by {d_on:+.4f} +- {e_on:.4f}; "
          f"shift off: rate {r_off:.4f}, by {d_off:+.4f} +- {e_off:.4f}")
    assert abs(d_on) < 3.0 * e_on
    assert d_off > 8.0 * e_off
    assert abs(r_on / (k * k) - 0.87) < 0.1
    # without the shift the fluid at this mean free path is far from it
    assert r_off < 0.6 * r_on
