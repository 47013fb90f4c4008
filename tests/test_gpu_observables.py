"""Observables of the FP32 storage form against the FP64 oracle over a long
run (sec. 4.1: the mixed-precision model is judged by what it does to the
physics, e.g. the net momentum).

A thermostatted fluid of 16^3 cells at ten particles per cell starts from one
state in both runs: the FP32 form on the GPU and the FP64 oracle on the host,
1000 steps each. Sampled after each of the first ten steps and then every ten
steps, the two runs give: the kinetic temperature T, the kurtosis
<v_x^4>/<v_x^2>^2 (3 for Maxwell-Boltzmann velocities), the net momentum per
particle (its change since the start), the occupancy histogram of the cells (Poisson at equilibrium, sec.
3.4), the distribution of the per-cell temperature and the velocity
autocorrelation C(t) = sum v(0).v(t) / sum v(0).v(0). The trajectories stay
within rounding of each other for the first steps and then part (the
dynamics is chaotic), so early values are compared directly and late ones as
time averages within their statistical errors. Each observable's FP32 value
and its difference from the oracle's are printed as a table.
"""
import numpy as np
import pytest

import paper_1801_10187_amd as m
import workloads
from helpers import banner
from oracle import srd

pytestmark = pytest.mark.gpu

N_CELLS = (16, 16, 16)
RHO = 10
STEPS = 1000
SAMPLES = list(range(1, 11)) + list(range(20, STEPS + 1, 10))


def _observables(pos, vel, v0, p):
    n = vel.shape[0]
    P = vel.sum(axis=0)
    dv = vel - P / n
    T = (dv * dv).sum() / (3.0 * (n - 1))
    kurt = float(np.mean([np.mean(dv[:, d] ** 4) / np.mean(dv[:, d] ** 2) ** 2 for d in range(3)]))
    cell = np.floor(pos).astype(np.int64)
    cell = cell[:, 0] + p.n_cells[0] * (cell[:, 1] + p.n_cells[1] * cell[:, 2])
    count, M, Pc, u, ek = srd.cell_sums(cell, vel, np.ones(n), p.ncells)
    ok = count >= 2
    Tc = 2.0 * ek[ok] / (3.0 * (count[ok] - 1))
    P0 = v0.sum(axis=0)
    return dict(T=T, kurtosis=kurt, momentum_per_particle=float(np.abs(P - P0).max() / n),
                occupancy=np.bincount(count, minlength=40)[:40],
                cellT_mean=float(Tc.mean()), cellT_std=float(Tc.std()),
                vacf=float((v0 * vel).sum() / (v0 * v0).sum()))


def _gpu_run(pos, vel, p):
    out = {}
    with m.Sim(pos, vel, p.n_cells, seed=p.seed, kT=p.kT, precision=m.FP32, thermostat=True) as s:
        _, v0 = s.get_state()
        done = 0
        for k in SAMPLES:
            s.step(k - done)
            done = k
            gpos, gvel = s.get_state()
            out[k] = _observables(gpos, gvel, v0, p)
    return out


def _oracle_run(pos, vel, p):
    out = {}
    mass = np.ones(pos.shape[0])
    v0 = vel
    done = 0
    for k in SAMPLES:
        pos, vel, _ = srd.run(pos, vel, mass, p, done, k - done)
        done = k
        out[k] = _observables(pos, vel, v0, p)
    return out


def _mean_se(series):
    a = np.asarray(series, dtype=np.float64)
    return a.mean(), a.std(ddof=1) / np.sqrt(a.size)


def test_fp32_observables_against_fp64_oracle():
    banner("fp32 observables over 1000 steps vs FP64 oracle")
    p = srd.Params(N_CELLS, seed=7, thermostat=True)
    pos, vel = workloads.fluid(N_CELLS, RHO, seed=8)
    g = _gpu_run(pos, vel, p)
    # the oracle starts from the FP32 form's initial state (velocities
    # rounded to FP32, as the GPU stores them), so the early steps compare
    # the arithmetic alone
    with m.Sim(pos, vel, p.n_cells, seed=p.seed, kT=p.kT, precision=m.FP32, thermostat=True) as s:
        pos32, vel32 = s.get_state()
    o = _oracle_run(pos32, vel32, p)

    rows = []
    # early steps: the same trajectory up to FP32 rounding
    for k in range(1, 6):
        d = abs(g[k]["vacf"] - o[k]["vacf"])
        rows.append((f"C(t) after step {k}", g[k]["vacf"], d))
        assert d < 1e-5
        assert abs(g[k]["T"] - o[k]["T"]) < 1e-5
    late = [k for k in SAMPLES if k >= 100]
    for key in ("T", "kurtosis", "cellT_mean", "cellT_std"):
        gm, gse = _mean_se([g[k][key] for k in late])
        om, ose = _mean_se([o[k][key] for k in late])
        bound = 5.0 * np.hypot(gse, ose) + 1e-9
        rows.append((f"<{key}> steps 100-1000", gm, gm - om))
        assert abs(gm - om) < bound, (key, gm, om, bound)
    # temperature held at kT by the thermostat, velocities Maxwellian
    assert abs(_mean_se([g[k]["T"] for k in late])[0] - p.kT) < 0.01
    assert abs(_mean_se([g[k]["kurtosis"] for k in late])[0] - 3.0) < 0.05
    # change of the net momentum since the start: exact conservation in
    # FP64 (rounding only), an FP32 rounding random walk of about
    # sqrt(steps / N) 2^-24 per particle
    gP = max(g[k]["momentum_per_particle"] for k in SAMPLES)
    oP = max(o[k]["momentum_per_particle"] for k in SAMPLES)
    rows.append(("max |P(t) - P(0)| / N over the run", gP, gP - oP))
    assert oP < 1e-13
    assert gP < 1e-7
    # occupancy histograms: the two runs agree, and both are Poisson(rho)
    gh = sum(g[k]["occupancy"] for k in late).astype(np.float64)
    oh = sum(o[k]["occupancy"] for k in late).astype(np.float64)
    gh /= gh.sum()
    oh /= oh.sum()
    from scipy.stats import poisson
    pois = poisson.pmf(np.arange(40), RHO)
    tvd = 0.5 * np.abs(gh - oh).sum()
    rows.append(("occupancy histogram: distance to the oracle's", 0.5 * np.abs(gh - pois).sum(), tvd))
    assert tvd < 0.01
    assert 0.5 * np.abs(gh - pois).sum() < 0.01
    print("\nobservable | FP32 value | FP32 - FP64 oracle")
    for name, val, diff in rows:
        print(f"{name} | {val:.6g} | {diff:+.3g}")
