"""Pins of the oracle's Maxwell-Boltzmann thermostat and of the velocity
distribution the collision produces (CPU only)."""
import math

import numpy as np
import pytest
from scipy import stats

import workloads
from oracle import srd


@pytest.mark.parametrize("k", [1.5, 3.0, 13.5])
def test_gamma_sampler_matches_scipy_gamma(k):
    """Marsaglia-Tsang draws follow Gamma(k, theta) (KS against the library
    distribution, 2e5 draws, false alarm 1e-4)."""
    p = srd.Params((1, 1, 1), seed=99)
    n = 200000
    draws, attempts = srd.gamma_marsaglia_tsang(np.full(n, k), np.arange(n), 7, p, 2.0)
    assert not np.any(np.isnan(draws))
    assert stats.kstest(draws, stats.gamma(k, scale=2.0).cdf).pvalue > 1e-4
    # the method's acceptance rate is above 0.95 for shape >= 1
    assert attempts.mean() < 1.06


def test_thermostat_sets_cell_energy_to_the_draw():
    """After the scale xi = sqrt(E_hat / E_k) the relative kinetic energy of
    a cell equals E_hat, to rounding (sec. 2, eq. 3)."""
    p = srd.Params((5, 5, 5), seed=3, thermostat=True, kT=1.7)
    pos, vel = workloads.fluid(p.n_cells, 6, seed=8, kT=0.6)
    mass = np.ones(pos.shape[0])
    vnew, info = srd.collide(pos, vel, mass, p, 4)
    cnt1, _, _, u1, ek1 = srd.cell_sums(info["cell"], vnew, mass, p.ncells)
    act = info["count"] >= 2
    assert np.allclose(u1[act], info["u"][act], atol=1e-14)
    assert np.allclose(ek1[act], info["ek"][act] * info["xi"][act] ** 2, rtol=1e-12)
    assert np.all(info["xi"][~act] == 1.0)


def test_cell_energy_distribution_is_gamma():
    """Post-thermostat cell energies of N_c-particle cells follow
    Gamma(3(N_c-1)/2, kT) (Maxwell-Boltzmann consistent with N_c)."""
    p = srd.Params((30, 30, 30), seed=5, thermostat=True, kT=1.0)
    pos, vel = workloads.fluid(p.n_cells, 5, seed=6, kT=3.0)
    mass = np.ones(pos.shape[0])
    vnew, info = srd.collide(pos, vel, mass, p, 0)
    _, _, _, _, ek1 = srd.cell_sums(info["cell"], vnew, mass, p.ncells)
    for nc in (3, 5, 7):
        sel = info["count"] == nc
        assert sel.sum() > 1000
        assert stats.kstest(ek1[sel], stats.gamma(1.5 * (nc - 1), scale=1.0).cdf).pvalue > 1e-4


def test_thermostat_relaxes_temperature():
    p = srd.Params((10, 10, 10), seed=2, thermostat=True, kT=1.0)
    pos, vel = workloads.fluid(p.n_cells, 10, seed=3, kT=2.0)
    mass = np.ones(pos.shape[0])
    _, _, t0 = srd.totals(vel, mass)
    assert abs(t0 - 2.0) < 0.05
    pos, vel, _ = srd.run(pos, vel, mass, p, 0, 20)
    _, _, t1 = srd.totals(vel, mass)
    # every cell is rescaled to kT each step; the residual reflects the
    # centre-of-mass motion of the cells and sampling noise
    assert abs(t1 - 1.0) < 0.05


def test_maxwell_boltzmann_relaxation_from_equal_speeds():
    """SRD gives the Maxwell-Boltzmann velocity distribution (sec. 2). From
    a start with every speed sqrt(3 kT/m), after 60 energy-conserving steps
    one velocity component is Gaussian with variance kT/m."""
    p = srd.Params((16, 16, 16), seed=8)
    pos, vel = workloads.non_gaussian_fluid(p.n_cells, 5, seed=4)
    mass = np.ones(pos.shape[0])
    assert stats.kurtosis(vel[:, 0], fisher=False) < 2.0     # far from 3
    pos, vel, _ = srd.run(pos, vel, mass, p, 0, 60)
    vx = vel[:, 0]
    assert stats.kstest(vx, stats.norm(scale=1.0).cdf).pvalue > 1e-4
    assert abs(stats.kurtosis(vx, fisher=False) - 3.0) < 0.1


@pytest.mark.parametrize("k", [1.5, 3.0, 13.5, 60.0])
def test_squeeze_is_inside_the_acceptance_region(k):
    """Marsaglia and Tsang's squeeze U < 1 - 0.0331 g^4 only accepts points
    the full test log U < g^2/2 + d - dV + d log V accepts too, so using it
    changes no decision (checked in FP64 on 10^6 random points)."""
    rng = np.random.default_rng(int(k * 10))
    d = k - 1.0 / 3.0
    c = 1.0 / math.sqrt(9.0 * d)
    g = rng.normal(size=1_000_000)
    u = rng.random(1_000_000)
    t = 1.0 + c * g
    ok = t > 0
    g, u, t = g[ok], u[ok], t[ok]
    V = t * t * t
    sq = g * g
    squeeze = u < 1.0 - 0.0331 * (sq * sq)
    full = np.log(u) < 0.5 * g * g + d - d * V + d * np.log(V)
    assert squeeze.mean() > 0.9
    assert not np.any(squeeze & ~full)
