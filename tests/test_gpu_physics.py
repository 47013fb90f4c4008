"""Physics checks of the GPU engine at the paper's benchmark parameters
(density 10 per cell, alpha = 130 deg, dt = 0.1, kT = 1, random shift):

* shear viscosity: the paper states 8.7 (units of energy x time / length^3)
  for this fluid (sec. 4); measured here from the decay of a transverse shear
  wave, whose amplitude falls as exp(-nu k^2 t) with kinematic viscosity
  nu = eta / (rho m);
* FP32 form: the centre-of-mass velocity stays small and shows no drift
  (sec. 4.1, mixed-precision model), while the FP64 form keeps it at
  rounding level.
"""
import math

import numpy as np
import pytest

import paper_1801_10187_amd as m
import workloads
from helpers import banner

pytestmark = pytest.mark.gpu

PAPER_VISCOSITY = 8.7  # stated for rho = 10, alpha = 130 deg, dt = 0.1 (sec. 4)


def _shear_wave_amplitude(u, M, n):
    """Amplitude A of u_x(z) = A sin(k z) from the cell-averaged field
    (cell centres; the cell average of sin multiplies A by a constant)."""
    iz = np.arange(n[0] * n[1] * n[2]) // (n[0] * n[1])
    s = np.sin(2.0 * math.pi * (iz + 0.5) / n[2])
    return 2.0 * np.sum(M * u[:, 0] * s) / np.sum(M)


@pytest.mark.parametrize("form", ["fp64", "fp32"])
def test_shear_viscosity_matches_the_paper(form):
    banner(f"shear viscosity {form}")
    n = (64, 64, 64)
    k = 2.0 * math.pi / n[2]
    amp0 = 0.1
    every, chunks = 40, 60          # readouts every 4 time units, 240 in total
    rates = []
    for seed in (1, 2, 3, 4, 5, 6):
        pos, vel = workloads.fluid(n, 10, seed=seed)
        vel[:, 0] += amp0 * np.sin(k * pos[:, 2])
        vel -= vel.mean(axis=0)
        prec = m.FP64 if form == "fp64" else m.FP32
        t, amp = [], []
        with m.Sim(pos, vel, n, seed=100 + seed, precision=prec, thermostat=False) as s:
            for c in range(chunks + 1):
                if c:
                    s.step(every)
                u, M = s.velocity_field()
                t.append(c * every * 0.1)
                amp.append(_shear_wave_amplitude(u, M, n))
        t, amp = np.array(t), np.array(amp)
        use = amp > 0.3 * amp0   # well above the thermal noise (~1e-3)
        rates.append(-np.polyfit(t[use], np.log(amp[use]), 1)[0])
    nu = np.mean(rates) / (k * k)
    eta = 10.0 * nu
    print(f"measured viscosity {eta:.3f} (paper {PAPER_VISCOSITY}), per-run rates {rates}")
    assert abs(eta - PAPER_VISCOSITY) < 0.05 * PAPER_VISCOSITY


def test_fp32_centre_of_mass_velocity_stays_small():
    """50^3 cells at density 10 (1.25 x 10^6 particles, the paper's smaller
    precision benchmark box), 20 000 steps: the FP64 form keeps the net
    momentum at rounding level; in the FP32 form each step rounds every
    velocity to FP32, so the centre-of-mass velocity wanders like a random
    walk of size ~ sqrt(steps / N) 2^-24 -- small, bounded, and without drift."""
    banner("fp32 centre-of-mass velocity")
    n = (50, 50, 50)
    pos, vel = workloads.fluid(n, 10, seed=7)
    N = pos.shape[0]
    with m.Sim(pos, vel, n, seed=7, precision=m.FP64, thermostat=True) as s:
        s.step(2000)
        P, _, _ = s.totals()
    assert np.abs(P).max() / N < 1e-15
    vc = []
    with m.Sim(pos, vel, n, seed=7, precision=m.FP32, thermostat=True) as s:
        for _ in range(20):
            s.step(1000)
            P, _, kT = s.totals()
            vc.append(P / N)
    vc = np.array(vc)
    walk = math.sqrt(20000 / N) * 2.0 ** -24
    print(f"|v_c| max {np.abs(vc).max():.3e}, random-walk scale {walk:.3e}")
    assert np.abs(vc).max() < 50 * walk
    assert abs(kT - 1.0) < 0.01
