"""Pins of the oracle's Andersen-thermostat collision rule (eq. 4, sec. 3.7)."""
import math

import numpy as np
from scipy import stats

import workloads
from oracle import brute, fp32form, srd


def _params(**kw):
    return srd.Params((6, 5, 4), seed=17, rule="at", **kw)


def test_kicks_are_independent_gaussians_at_kT_over_m():
    """The per-particle random velocities are N(0, kT/m) per component,
    uncorrelated between components (KS and correlation on 10^5 draws)."""
    p = _params(kT=1.7)
    n = 100000
    mass = np.where(np.arange(n) % 4 == 0, 5.0, 1.0)
    dv = srd.at_kicks(np.arange(n), 3, mass, p)
    g = dv / np.sqrt(p.kT / mass)[:, None]
    for d in range(3):
        assert stats.kstest(g[:, d], "norm").pvalue > 1e-4
    c = np.corrcoef(g.T)
    assert np.abs(c - np.eye(3)).max() < 0.02
    # a different step or seed gives different numbers
    assert not np.array_equal(srd.at_kicks(np.arange(10), 4, mass[:10], p), dv[:10])


def test_at_conserves_cell_momentum_and_keeps_lone_particles():
    p = _params()
    pos, vel = workloads.fluid(p.n_cells, 2, seed=3)
    rng = np.random.default_rng(4)
    mass = rng.choice([1.0, 5.0], size=pos.shape[0])
    pos1 = srd.stream(pos, vel, p)
    vnew, info = srd.collide(pos1, vel, mass, p, 0)
    cell = info["cell"]
    for d in range(3):
        before = np.bincount(cell, weights=mass * vel[:, d], minlength=p.ncells)
        after = np.bincount(cell, weights=mass * vnew[:, d], minlength=p.ncells)
        assert np.allclose(before, after, atol=1e-12)
    lone = info["count"][cell] == 1
    assert lone.any()
    assert np.allclose(vnew[lone], vel[lone], rtol=0, atol=1e-14)


def test_at_relative_velocities_have_the_reduced_variance():
    """In a cell of N_c equal masses the new velocity relative to u is
    dv_i - mean(dv): Gaussian with variance (1 - 1/N_c) kT / m."""
    p = srd.Params((30, 30, 30), seed=5, rule="at", kT=2.0)
    pos, vel = workloads.fluid(p.n_cells, 5, seed=6, kT=0.3)
    mass = np.ones(pos.shape[0])
    vnew, info = srd.collide(pos, vel, mass, p, 0)
    rel = vnew - info["u"][info["cell"]]
    for nc in (2, 5, 8):
        sel = info["count"][info["cell"]] == nc
        x = rel[sel, 0] / math.sqrt((1.0 - 1.0 / nc) * p.kT)
        assert stats.kstest(x, "norm").pvalue > 1e-4


def test_at_thermalises_to_kT():
    p = srd.Params((10, 10, 10), seed=2, rule="at", kT=1.0)
    pos, vel = workloads.fluid(p.n_cells, 10, seed=3, kT=3.0)
    mass = np.ones(pos.shape[0])
    pos, vel, _ = srd.run(pos, vel, mass, p, 0, 10)
    _, _, kT = srd.totals(vel, mass)
    assert abs(kT - 1.0) < 0.03


def test_at_oracle_matches_brute_force():
    """Vectorised AT step against the particle-by-particle pure-Python one
    (scalar Philox, rational cell sums) on a few-cell box with beads."""
    p = srd.Params((3, 2, 2), seed=9, rule="at", kT=1.2)
    pos, vel = workloads.fluid(p.n_cells, 4, seed=10)
    rng = np.random.default_rng(11)
    mass = rng.choice([1.0, 5.0], size=pos.shape[0])
    opos, ovel, info = srd.srd_step(pos, vel, mass, p, 7)
    bpos, bvel, bcells = brute.brute_at_step(pos.tolist(), vel.tolist(), mass.tolist(), p, 7)
    assert np.array_equal(np.array(bcells), info["cell"])
    assert np.array_equal(np.array(bpos), opos)
    assert np.allclose(np.array(bvel), ovel, rtol=0, atol=1e-13)


def test_fp32_emulation_of_at_rounds_the_fp64_result():
    p = _params()
    pos, vel = workloads.fluid(p.n_cells, 3, seed=12)
    mass = np.ones(pos.shape[0])
    h, o, v = fp32form.from_double(pos, vel, p)
    h1, o1, v1, info = fp32form.step32(h, o, v, mass, p, 0)
    v64, _ = srd.collide_at(info["cell"], v.astype(np.float64), mass, p, 0,
                            kicks=fp32form.at_kicks32)
    assert np.array_equal(v1, v64.astype(np.float32))


def test_fp32_uniforms_are_exact_single_precision_values_inside_0_1():
    w = np.array([0, 511, 512, 2**31, 2**32 - 1], dtype=np.uint64)
    u = fp32form.uniform23(w)
    assert u[0] == 2.0 ** -24 and u[1] == 2.0 ** -24
    assert u[2] == 1.5 * 2.0 ** -23
    assert u[3] == 0.5 + 2.0 ** -24
    assert u[4] == 1.0 - 2.0 ** -24
    rng = np.random.default_rng(3)
    w = rng.integers(0, 2**32, size=100000, dtype=np.uint64)
    u = fp32form.uniform23(w)
    assert np.array_equal(u, u.astype(np.float32).astype(np.float64))
    assert u.min() > 0.0 and u.max() < 1.0
    # 2^23 equally spaced levels: the spacing of the values is 2^-23
    assert np.all(np.mod(u * 2.0 ** 23 - 0.5, 1.0) == 0.0)


def _words(tags, step, p):
    from oracle.philox import TAG_AT, philox4x32_10, seed_key
    n = tags.size
    ctr = np.stack([tags, np.full(n, step), np.full(n, TAG_AT), np.zeros(n)], axis=1).astype(np.uint32)
    return philox4x32_10(ctr, seed_key(p.seed))


def test_fp32_kicks_are_box_muller_of_their_uniforms():
    """The FP32 form's kicks (sec. 3.7, sec. 4.1): for each particle the
    first two components lie on the circle of radius sqrt(-2 ln u0) at angle
    2 pi u1, the third is sqrt(-2 ln u2) cos(2 pi u3); the scale is
    sqrt(kT / m) rounded to FP32; the components are N(0, 1) after it."""
    p = _params(kT=1.3)
    n = 100000
    tags = np.arange(n, dtype=np.uint64)
    mass = np.where(np.arange(n) % 3 == 0, 5.0, 1.0)
    dv = fp32form.at_kicks32(tags, 5, mass, p)
    scale = np.sqrt(p.kT / mass)
    s32 = scale.astype(np.float32).astype(np.float64)
    assert np.all(np.abs(s32 - scale) <= 2.0 ** -24 * scale)
    g = dv / s32[:, None]
    u = fp32form.uniform23(_words(tags, 5, p))
    r0sq = -2.0 * np.log(u[:, 0])
    assert np.allclose(g[:, 0] ** 2 + g[:, 1] ** 2, r0sq, rtol=1e-12, atol=0)
    ang = np.mod(np.arctan2(g[:, 1], g[:, 0]), 2.0 * math.pi)
    d = np.abs(ang - 2.0 * math.pi * u[:, 1])
    assert np.minimum(d, 2.0 * math.pi - d).max() < 1e-9
    c3 = g[:, 2] / np.sqrt(-2.0 * np.log(u[:, 2]))
    assert np.allclose(c3, np.cos(2.0 * math.pi * u[:, 3]), rtol=0, atol=1e-12)
    for k in range(3):
        assert stats.kstest(g[:, k], "norm").pvalue > 1e-4


def test_fp32_kicks_follow_the_fp64_form_from_the_same_words():
    """Both forms draw from the same words with the same pairing; the FP32
    form's uniforms drop the low 9 bits, so away from u0 -> 0 the two kicks
    agree to about 2^-23 relative of the uniforms' effect."""
    p = _params(kT=1.0)
    n = 20000
    tags = np.arange(n, dtype=np.uint64)
    mass = np.ones(n)
    a = fp32form.at_kicks32(tags, 2, mass, p)
    b = srd.at_kicks(tags, 2, mass, p)
    u = fp32form.uniform23(_words(tags, 2, p))
    ok = (u[:, 0] > 1e-3) & (u[:, 2] > 1e-3)
    assert ok.mean() > 0.99
    assert np.abs(a[ok] - b[ok]).max() < 1e-4
