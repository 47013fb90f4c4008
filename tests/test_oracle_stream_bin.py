"""Pins of the oracle's streaming, grid shift and binning (CPU only)."""
import math

import numpy as np
import pytest
from scipy import stats

import workloads
from oracle import brute, srd


def test_stream_dt_zero_is_identity():
    p = srd.Params((4, 3, 5), dt=0.0)
    pos, vel = workloads.fluid(p.n_cells, 3, seed=4)
    assert np.array_equal(srd.stream(pos, vel, p), pos)


def test_stream_returns_after_whole_box_periods():
    """Closed form (eq. 1): with v = L / (k dt) a particle is back where it
    started after k steps. Binary-exact numbers make every step exact."""
    p = srd.Params((8, 8, 8), a=1.0, dt=0.25)
    pos = np.array([[0.5, 3.25, 7.875], [0.0, 0.0, 0.0], [7.5, 1.0, 2.0]])
    vel = np.array([[8.0, -8.0, 4.0], [-16.0, 2.0, 8.0], [4.0, 16.0, -2.0]])
    # per-axis periods: k = L / (v dt) steps
    x = pos.copy()
    for _ in range(16):
        x = srd.stream(x, vel, p)
    assert np.array_equal(x, pos)
    # one step moves exactly v*dt modulo L
    x1 = srd.stream(pos, vel, p)
    assert np.array_equal(x1, np.mod(pos + vel * 0.25, 8.0))


def test_wrap_rules_at_the_box_edge():
    L = np.array([10.0, 10.0, 10.0])
    w = np.array([10.0, 10.0 + 2**-40, -1e-300, -2.0, 19.999, 0.0])
    out = srd.wrap(w, 10.0)
    assert out[0] == 0.0                    # exactly L -> 0
    assert out[1] == 2**-40                 # exact (Sterbenz)
    assert out[2] == 0.0                    # tiny negative rounds to L -> 0
    assert out[3] == 8.0
    assert out[4] == 19.999 - 10.0
    assert out[5] == 0.0
    assert np.all((out >= 0) & (out < 10.0))


def test_stream_rejects_whole_box_moves():
    p = srd.Params((2, 2, 2), dt=1.0)
    with pytest.raises(ValueError):
        srd.stream(np.zeros((1, 3)), np.array([[2.0, 0, 0]]), p)


def test_bin_hand_computed_cells():
    """Cells typed in by hand: box 4x3x2, a = 1, shift (0.25, -0.5, 0.5).
    (3.9, 0.2, 1.7) + s = (4.15, -0.3, 2.2) -> wrapped (0.15, 2.7, 0.2)
    -> (0, 2, 0) -> 0 + 4*(2 + 3*0) = 8.
    (1.0, 2.5, 0.0) + s = (1.25, 2.0, 0.5) -> (1, 2, 0) -> 9.
    (0.74, 0.49, 1.49) + s = (0.99, -0.01, 1.99) -> (0.99, 2.99, 1.99)
    -> (0, 2, 1) -> 0 + 4*(2 + 3*1) = 20."""
    p = srd.Params((4, 3, 2))
    pos = np.array([[3.9, 0.2, 1.7], [1.0, 2.5, 0.0], [0.74, 0.49, 1.49]])
    cells = srd.bin_cells(pos, np.array([0.25, -0.5, 0.5]), p)
    assert cells.tolist() == [8, 9, 20]


def test_bin_clamps_top_edge():
    """w just below L can give floor(w / a) == n after the multiply by a
    rounded 1/a; the index is clamped to n - 1."""
    p = srd.Params((3, 3, 3), a=0.1)
    w = np.nextafter(p.L[0], 0.0)
    cells = srd.bin_cells(np.array([[w, w, w]]), np.zeros(3), p)
    assert cells[0] == 2 + 3 * (2 + 3 * 2)


def test_shift_uniform_and_bounded():
    p = srd.Params((2, 2, 2), a=2.0, seed=11)
    s = np.array([srd.grid_shift(p, n) for n in range(4000)])
    assert np.all(np.abs(s) < 1.0)
    for d in range(3):
        assert stats.kstest(s[:, d], stats.uniform(loc=-1.0, scale=2.0).cdf).pvalue > 1e-4
    # components of one step and consecutive steps are uncorrelated
    c = np.corrcoef(s.T)
    assert np.all(np.abs(c[np.triu_indices(3, 1)]) < 0.08)


def test_shift_off_is_zero():
    p = srd.Params((2, 2, 2), grid_shift=False)
    assert np.array_equal(srd.grid_shift(p, 5), np.zeros(3))


def test_occupancy_sums_to_n_and_is_poisson():
    """Cell occupancy of a uniform fluid is Poisson(rho) (sec. 3.4)."""
    n_cells, rho = (30, 30, 30), 5
    p = srd.Params(n_cells)
    pos, _ = workloads.fluid(n_cells, rho, seed=21)
    cells = srd.bin_cells(pos, srd.grid_shift(p, 0), p)
    count = np.bincount(cells, minlength=p.ncells)
    assert count.sum() == pos.shape[0]
    # the mean is fixed at rho; compare the shape with Poisson(rho)
    kmax = 14
    obs = np.bincount(np.minimum(count, kmax), minlength=kmax + 1)
    pmf = stats.poisson.pmf(np.arange(kmax), rho)
    exp = np.append(pmf, 1 - pmf.sum()) * p.ncells
    chi2 = ((obs - exp) ** 2 / exp).sum()
    assert chi2 < stats.chi2.ppf(1 - 1e-4, kmax)


@pytest.mark.parametrize("n_cells", [(1, 1, 1), (2, 1, 1), (2, 2, 2), (1, 3, 2)])
def test_bin_matches_brute_force(n_cells):
    p = srd.Params(n_cells, seed=5)
    pos, vel = workloads.fluid(n_cells, 4, seed=9)
    mass = np.ones(pos.shape[0])
    for step in range(5):
        bpos, bvel, bcells, bs, _ = brute.brute_step(pos.tolist(), vel.tolist(),
                                                     mass.tolist(), p, step)
        pos1 = srd.stream(pos, vel, p)
        s = srd.grid_shift(p, step)
        cells = srd.bin_cells(pos1, s, p)
        assert np.array_equal(np.array(bpos), pos1)
        assert np.array_equal(np.array(bs), s)
        assert cells.tolist() == bcells
        pos, vel = pos1, np.array(bvel)


def test_binning_with_shift_equals_translated_positions():
    """Binning positions r with shift s gives the cells of r + s binned
    without a shift (the shift moves the grid, not the particles)."""
    p = srd.Params((5, 4, 3), a=0.5)
    pos, _ = workloads.fluid(p.n_cells, 3, seed=8, a=0.5)
    s = np.array([0.2, -0.11, 0.049])
    moved = srd.wrap(pos + s, p.L)
    assert np.array_equal(srd.bin_cells(pos, s, p),
                          srd.bin_cells(moved, np.zeros(3), p))
