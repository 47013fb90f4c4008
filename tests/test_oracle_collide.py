"""Pins of the oracle's cell sums, axis draw, rotation and whole collision
(CPU only)."""
import math
from fractions import Fraction

import numpy as np
import pytest
from scipy import stats
from scipy.spatial.transform import Rotation

import workloads
from oracle import brute, srd

EPS = 2.0 ** -53


def _state(n_cells=(6, 5, 4), rho=6, seed=3, kT=1.0):
    pos, vel = workloads.fluid(n_cells, rho, kT=kT, seed=seed)
    return pos, vel, np.ones(pos.shape[0])


# ----------------------------------------------------------------- rotation
def test_rotation_matches_scipy_rotvec():
    """Rodrigues' rotation by +alpha about n equals the library rotation
    from the rotation vector alpha*n (eq. 2)."""
    rng = np.random.default_rng(1)
    for alpha in (130.0 * math.pi / 180, 0.3, 2.9):
        p = srd.Params((3, 3, 3), alpha=alpha)
        n = rng.normal(size=(27, 3))
        n /= np.linalg.norm(n, axis=1, keepdims=True)
        u = rng.normal(size=(27, 3))
        cell = rng.integers(0, 27, size=500)
        v = rng.normal(size=(500, 3))
        out = srd.rotate(v, cell, u, n, np.ones(27), p)
        ref = u[cell] + Rotation.from_rotvec(alpha * n[cell]).apply(v - u[cell])
        assert np.max(np.abs(out - ref)) < 1e-14


def test_rotation_invariants_and_special_angles():
    rng = np.random.default_rng(2)
    n = rng.normal(size=(1, 3))
    n /= np.linalg.norm(n)
    d = rng.normal(size=(300, 3))
    cell = np.zeros(300, dtype=np.int64)
    zero_u = np.zeros((1, 3))
    alpha = 130.0 * math.pi / 180
    out = srd.rotate(d, cell, zero_u, n, np.ones(1), srd.Params((1, 1, 1), alpha=alpha))
    # component along the axis and length are preserved
    assert np.allclose(out @ n[0], d @ n[0], atol=1e-14)
    assert np.allclose(np.linalg.norm(out, axis=1), np.linalg.norm(d, axis=1), rtol=1e-14)
    # perpendicular parts turn by alpha, right-handed about n
    dp = d - np.outer(d @ n[0], n[0])
    op = out - np.outer(out @ n[0], n[0])
    cosang = (dp * op).sum(1) / (np.linalg.norm(dp, axis=1) * np.linalg.norm(op, axis=1))
    assert np.allclose(cosang, math.cos(alpha), atol=1e-12)
    sinang = (np.cross(dp, op) @ n[0]) / (np.linalg.norm(dp, axis=1) * np.linalg.norm(op, axis=1))
    assert np.allclose(sinang, math.sin(alpha), atol=1e-12)
    # alpha = 0 is the identity; alpha = pi reflects through the axis
    out0 = srd.rotate(d, cell, zero_u, n, np.ones(1), srd.Params((1, 1, 1), alpha=0.0))
    assert np.array_equal(out0, d)
    outpi = srd.rotate(d, cell, zero_u, n, np.ones(1), srd.Params((1, 1, 1), alpha=math.pi))
    assert np.allclose(outpi, 2 * np.outer(d @ n[0], n[0]) - d, atol=1e-14)


# ---------------------------------------------------------------- cell sums
def test_cell_sums_exact_rational_bound():
    """FP64 sums agree with the exact rational sums within
    N_c * eps * sum |m v| (plus the rounding of the mean)."""
    pos, vel, _ = _state((2, 2, 2), rho=9, seed=4)
    rng = np.random.default_rng(0)
    mass = rng.choice([1.0, 5.0], size=pos.shape[0])
    p = srd.Params((2, 2, 2))
    cell = srd.bin_cells(pos, np.zeros(3), p)
    count, M, P, u, ek = srd.cell_sums(cell, vel, mass, p.ncells)
    for c in range(p.ncells):
        idx = np.nonzero(cell == c)[0]
        Mx = sum(Fraction(float(mass[i])) for i in idx)
        assert M[c] == float(Mx)
        for d in range(3):
            Px = sum(Fraction(float(mass[i])) * Fraction(float(vel[i, d])) for i in idx)
            bound = 2 * len(idx) * EPS * float(sum(abs(mass[i] * vel[i, d]) for i in idx))
            assert abs(P[c, d] - float(Px)) <= bound
            assert abs(u[c, d] - float(Px / Mx)) <= bound / float(Mx) + EPS * abs(u[c, d])
        assert count[c] == idx.size
        ekx = 0.5 * math.fsum(mass[i] * ((vel[i] - u[c]) ** 2).sum() for i in idx)
        assert abs(ek[c] - ekx) <= 8 * len(idx) * EPS * ekx


def test_hand_computed_mass_weighted_mean():
    """One cell, a solvent particle (m = 1) and a bead (m = 5): the centre
    of mass velocity is (1*v1 + 5*v2) / 6 (sec. 2, embedded particles)."""
    vel = np.array([[1.0, -2.0, 0.5], [-1.0, 4.0, 3.5]])
    mass = np.array([1.0, 5.0])
    count, M, P, u, ek = srd.cell_sums(np.array([0, 0]), vel, mass, 1)
    assert count[0] == 2 and M[0] == 6.0
    assert np.allclose(u[0], [(1 - 5) / 6, (-2 + 20) / 6, (0.5 + 17.5) / 6], rtol=0, atol=1e-15)
    # E_k relative to u: 1/2 [1*|v1-u|^2 + 5*|v2-u|^2]; u = (-2/3, 3, 3)
    e = 0.5 * (1 * ((1 + 2 / 3) ** 2 + 25 + 6.25) + 5 * ((-1 + 2 / 3) ** 2 + 1 + 0.25))
    assert abs(ek[0] - e) < 1e-13


# ------------------------------------------------------------------- axes
def test_axes_unit_and_isotropic():
    p = srd.Params((1, 1, 1), seed=13)
    n = srd.cell_axes(np.arange(200000), 3, p)
    assert np.max(np.abs(np.linalg.norm(n, axis=1) - 1.0)) < 4e-16
    assert np.all(np.abs(n.mean(axis=0)) < 0.01)
    assert np.allclose(n.T @ n / n.shape[0], np.eye(3) / 3, atol=0.006)
    # Archimedes: z is uniform on (-1, 1); so is each other component
    for d in range(3):
        assert stats.kstest(n[:, d], stats.uniform(loc=-1, scale=2).cdf).pvalue > 1e-4


# ------------------------------------------------------------ conservation
def test_collision_conserves_cell_momentum_and_energy():
    pos, vel, mass = _state((5, 5, 5), rho=8, seed=6)
    rng = np.random.default_rng(5)
    mass = rng.choice([1.0, 5.0], p=[0.9, 0.1], size=pos.shape[0])
    p = srd.Params((5, 5, 5))
    vnew, info = srd.collide(pos, vel, mass, p, 12)
    cell = info["cell"]
    for d in range(3):
        P0 = np.bincount(cell, weights=mass * vel[:, d], minlength=p.ncells)
        P1 = np.bincount(cell, weights=mass * vnew[:, d], minlength=p.ncells)
        scale = np.bincount(cell, weights=np.abs(mass * vel[:, d]), minlength=p.ncells)
        assert np.all(np.abs(P1 - P0) <= 8 * info["count"] * EPS * scale + 1e-300)
    K0 = np.bincount(cell, weights=mass * (vel ** 2).sum(1), minlength=p.ncells)
    K1 = np.bincount(cell, weights=mass * (vnew ** 2).sum(1), minlength=p.ncells)
    assert np.all(np.abs(K1 - K0) <= 16 * info["count"] * EPS * K0 + 1e-300)


def test_lonely_particle_keeps_its_velocity():
    p = srd.Params((4, 4, 4), grid_shift=False)
    pos = np.array([[0.5, 0.5, 0.5], [2.5, 2.5, 2.5], [2.7, 2.1, 2.2]])
    vel = np.array([[0.3, -1.2, 2.2], [1.0, 0.0, 0.0], [-1.0, 0.5, 0.0]])
    vnew, info = srd.collide(pos, vel, np.ones(3), p, 0)
    assert np.array_equal(vnew[0], vel[0])
    assert not np.allclose(vnew[1], vel[1])


def test_exact_rational_conservation_with_quarter_turn():
    """alpha = 90 deg about the z axis maps (x, y, z) -> (-y, x, z): with
    dyadic velocities every step is exact, and the cell momentum is
    conserved exactly in rational arithmetic."""
    p = srd.Params((1, 1, 1), alpha=math.pi / 2)
    vel = np.array([[0.5, 0.25, 1.0], [-0.75, 1.5, 0.0], [0.25, -1.75, -1.0],
                    [0.0, 0.0, 0.5]])
    mass = np.ones(4)
    cell = np.zeros(4, dtype=np.int64)
    _, _, _, u, _ = srd.cell_sums(cell, vel, mass, 1)
    p_exact = srd.Params((1, 1, 1), alpha=math.pi / 2)
    p_exact.cos_a, p_exact.sin_a = 0.0, 1.0
    out = srd.rotate(vel, cell, u, np.array([[0.0, 0.0, 1.0]]), np.ones(1), p_exact)
    dv = vel - u[0]
    assert np.array_equal(out - u[0], np.stack([-dv[:, 1], dv[:, 0], dv[:, 2]], 1))
    Pin = [sum(Fraction(x) for x in vel[:, d]) for d in range(3)]
    Pout = [sum(Fraction(x) for x in out[:, d]) for d in range(3)]
    assert Pin == Pout


# ------------------------------------------------------------ brute force
@pytest.mark.parametrize("n_cells,thermo", [((1, 1, 1), False), ((2, 2, 2), False),
                                            ((2, 2, 2), True), ((2, 1, 3), True)])
def test_full_step_matches_brute_force(n_cells, thermo):
    p = srd.Params(n_cells, seed=77, thermostat=thermo, kT=1.3)
    pos, vel = workloads.fluid(n_cells, 5, seed=31)
    rng = np.random.default_rng(2)
    mass = rng.choice([1.0, 5.0], p=[0.8, 0.2], size=pos.shape[0])
    for step in range(4):
        bpos, bvel, bcells, _, props = brute.brute_step(pos.tolist(), vel.tolist(),
                                                        mass.tolist(), p, step)
        pos1, vel1, info = srd.srd_step(pos, vel, mass, p, step)
        assert np.array_equal(np.array(bpos), pos1)
        assert info["cell"].tolist() == bcells
        for c, pr in props.items():
            assert info["count"][c] == pr["count"]
            assert np.allclose(info["u"][c], pr["u"], rtol=1e-14, atol=1e-15)
            assert np.allclose(info["axis"][c], pr["axis"], rtol=0, atol=1e-15)
            assert abs(info["xi"][c] - pr["xi"]) < 1e-13
        assert np.max(np.abs(np.array(bvel) - vel1)) < 1e-13
        pos, vel = pos1, vel1


# ------------------------------------------------------- global properties
def test_net_momentum_stays_at_rounding_level():
    """Double precision keeps the net momentum per particle at the
    rounding level after the initial correction (sec. 4.1 reports
    |v_cx| below 1e-16 for the FP64 model)."""
    p = srd.Params((12, 12, 12), seed=1)
    pos, vel = workloads.fluid(p.n_cells, 5, seed=1)
    mass = np.ones(pos.shape[0])
    P0, _, _ = srd.totals(vel, mass)
    assert np.all(np.abs(P0) / pos.shape[0] < 1e-16)
    pos, vel, _ = srd.run(pos, vel, mass, p, 0, 60)
    P, _, _ = srd.totals(vel, mass)
    assert np.all(np.abs(P) / pos.shape[0] < 1e-16)


def test_energy_conserved_without_thermostat():
    p = srd.Params((8, 8, 8), seed=2)
    pos, vel = workloads.fluid(p.n_cells, 5, seed=2)
    mass = np.ones(pos.shape[0])
    _, ke0, _ = srd.totals(vel, mass)
    pos, vel, _ = srd.run(pos, vel, mass, p, 0, 30)
    _, ke1, _ = srd.totals(vel, mass)
    assert abs(ke1 - ke0) < 1e-11 * ke0


def test_collision_commutes_with_a_boost():
    """Galilean invariance of the collision (eq. 2): boosting every velocity
    by V0 boosts u by V0 and leaves v - u unchanged, so the result is the
    unboosted one plus V0, to rounding of order |V0| * eps."""
    p = srd.Params((6, 6, 6), seed=4, thermostat=True)
    pos, vel = workloads.fluid(p.n_cells, 5, seed=5)
    mass = np.ones(pos.shape[0])
    V0 = np.array([200.0, -37.5, 3.0])
    va, ia = srd.collide(pos, vel, mass, p, 3)
    vb, ib = srd.collide(pos, vel + V0, mass, p, 3)
    assert np.array_equal(ia["cell"], ib["cell"])
    assert np.max(np.abs(vb - V0 - va)) < 64 * 200.0 * EPS
    assert np.allclose(ia["xi"], ib["xi"], rtol=1e-10)


def test_velocity_field_pins():
    """Cell-averaged field: a uniform flow gives that flow in every occupied
    cell and zero elsewhere; cell masses add up to the total mass; the field
    weighted by the cell masses gives the total momentum; one hand-placed
    pair of particles gives their mass-weighted mean in their cell."""
    p = srd.Params((5, 4, 3), seed=1)
    rng = np.random.default_rng(3)
    pos = rng.random((200, 3)) * p.L
    mass = rng.choice([1.0, 5.0], size=200)
    flow = np.array([0.3, -1.2, 0.05])
    u, M = srd.velocity_field(pos, np.tile(flow, (200, 1)), mass, p)
    occ = M > 0
    assert np.allclose(u[occ], flow, rtol=0, atol=1e-15) and np.all(u[~occ] == 0.0)
    assert abs(M.sum() - mass.sum()) < 1e-12
    vel = rng.normal(size=(200, 3))
    u, M = srd.velocity_field(pos, vel, mass, p)
    assert np.allclose((M[:, None] * u).sum(axis=0), (mass[:, None] * vel).sum(axis=0), atol=1e-12)
    # two particles in cell (1, 2, 0): index 1 + 5 * 2 = 11
    two = np.array([[1.2, 2.5, 0.1], [1.9, 2.0, 0.9]])
    u, M = srd.velocity_field(two, np.array([[1.0, 0, 0], [4.0, 0, 0]]), np.array([1.0, 3.0]), p)
    assert M[11] == 4.0 and u[11, 0] == (1.0 + 12.0) / 4.0 and np.count_nonzero(M) == 1
