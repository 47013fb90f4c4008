"""GPU parity of the HIP path against the FP64 oracle, through the C ABI.

Bar: bit-exact positions after a stream, bit-exact cell indices and
occupancy; velocities within 1e-12 relative (with a thermal floor) in the
FP64 form; in the FP32 form, cells bit-exact and velocities within one FP32
ulp after one step from a shared FP32 state.
"""
import math

import numpy as np
import pytest

import paper_1801_10187_amd as m
import workloads
from helpers import banner, fp32_step_matches, periodic_dist, ulp_diff_f32, vel_err_fp64, FP64_REL
from oracle import fp32form, philox, srd

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _lib():
    m.load()


def _sim(pos, vel, p, precision=m.FP64, **kw):
    return m.Sim(pos, vel, p.n_cells, a=p.a, alpha=p.alpha, dt=p.dt, kT=p.kT,
                 seed=p.seed, solvent_mass=p.solvent_mass, precision=precision,
                 thermostat=p.thermostat, grid_shift=p.grid_shift, **kw)


# ------------------------------------------------------------------ Philox
def test_philox_bitexact():
    banner("philox")
    rng = np.random.default_rng(0)
    ctr = rng.integers(0, 2**32, size=(4097, 4), dtype=np.uint64).astype(np.uint32)
    key = 0x0123456789ABCDEF
    out = m.philox(ctr, key)
    ref = philox.philox4x32_10(ctr.astype(np.uint64),
                               np.array(philox.seed_key(key), dtype=np.uint64))
    assert np.array_equal(out, ref)


def test_philox_matches_rocrand():
    """An independent Philox4x32-10: rocRAND's generator (seed -> key,
    counter (i, 0, 0, 0) for the i-th block of four words)."""
    banner("philox vs rocRAND")
    import ctypes
    lib = ctypes.CDLL("/opt/rocm/lib/librocrand.so")
    gen = ctypes.c_void_p()
    assert lib.rocrand_create_generator_host_blocking(ctypes.byref(gen), 404) == 0
    try:
        seed = 0x00000005DEADBEEF
        assert lib.rocrand_set_seed(gen, ctypes.c_ulonglong(seed)) == 0
        n = 4 * 64
        out = np.zeros(n, dtype=np.uint32)
        st = lib.rocrand_generate(gen, out.ctypes.data_as(ctypes.c_void_p), ctypes.c_size_t(n))
        assert st == 0
    finally:
        lib.rocrand_destroy_generator(gen)
    ctr = np.zeros((64, 4), dtype=np.uint64)
    ctr[:, 0] = np.arange(64)
    ref = philox.philox4x32_10(ctr, np.array(philox.seed_key(seed), dtype=np.uint64))
    assert np.array_equal(out.reshape(64, 4), ref)


# ----------------------------------------------------- stream, shift, bin
def test_shift_bitexact():
    banner("shift")
    p = srd.Params((5, 6, 7), a=0.75, seed=123456789012)
    pos, vel = workloads.fluid(p.n_cells, 2, seed=1, a=0.75)
    with _sim(pos, vel, p) as s:
        for n in (0, 1, 2, 99, 2**31 + 5):
            assert np.array_equal(s.shift(n), srd.grid_shift(p, n))


@pytest.mark.parametrize("n_cells,rho,a", [((20, 20, 20), 5, 1.0), ((7, 3, 11), 3.3, 0.5),
                                           ((1, 1, 1), 9, 2.0)])
def test_stream_and_bin_bitexact(n_cells, rho, a):
    banner(f"stream+bin {n_cells} rho={rho} a={a}")
    p = srd.Params(n_cells, a=a, seed=3)
    pos, vel = workloads.fluid(n_cells, rho, seed=4, a=a)
    with _sim(pos, vel, p) as s:
        s.stream()
        gpos, gvel = s.get_state()
        opos = srd.stream(pos, vel, p)
        assert np.array_equal(gpos, opos)
        assert np.array_equal(gvel, vel)
        s.bin()
        cells, counts = s.get_cells()
        ocells = srd.bin_cells(opos, srd.grid_shift(p, 0), p)
        assert np.array_equal(cells, ocells)
        assert np.array_equal(counts, np.bincount(ocells, minlength=p.ncells))


@pytest.mark.parametrize("form,n_cells,rho", [
    ("fp64", (9, 8, 7), 7), ("fp64", (3, 9, 10), 7), ("fp64", (5, 6, 9), 4),
    ("fp32", (9, 8, 7), 7), ("fp32", (3, 9, 10), 4)])
def test_cell_props_and_draws(form, n_cells, rho):
    """Per-cell mass, momentum, relative kinetic energy, axis and thermostat
    factor after stream + bin. Boxes with an axis shorter than a tile and
    partial tiles at the far faces included. FP64 form: exact sums, so the
    mass is bit-exact; FP32 form: each term of the momentum and energy sums
    is rounded to 2^-40 (one-limb fixed point), so the cell sums are within
    N_c 2^-41 of the exact ones."""
    banner(f"cell props and draws {form} {n_cells} rho={rho}")
    p = srd.Params(n_cells, seed=11, thermostat=True, kT=1.3)
    pos, vel = workloads.fluid(p.n_cells, rho, seed=5, kT=0.7)
    mass = np.ones(pos.shape[0])
    prec = m.FP64 if form == "fp64" else m.FP32
    with _sim(pos, vel, p, precision=prec) as s:
        s.stream()
        s.bin()
        gm, gP, gek = s.get_cell_props()
        gax, gxi = s.get_cell_draws()
    if form == "fp64":
        opos = srd.stream(pos, vel, p)
        cell = srd.bin_cells(opos, srd.grid_shift(p, 0), p)
        v64 = vel
        ptol = 1e-13
    else:
        h, o, v = fp32form.from_double(pos, vel, p)
        h, o = fp32form.stream32(h, o, v, p)
        cell = fp32form.bin32(h, o, srd.grid_shift(p, 0), p)
        v64 = v.astype(np.float64)
    count, M, P, u, ek = srd.cell_sums(cell, v64, mass, p.ncells)
    assert np.array_equal(gm, M)
    if form == "fp32":
        ptol = count.max() * 2.0 ** -41 + 1e-13
    assert np.max(np.abs(gP - P)) < ptol
    assert np.allclose(gek, ek, rtol=1e-12 if form == "fp64" else 1e-9, atol=1e-14)
    occ = count > 0
    ax = srd.cell_axes(np.arange(p.ncells), 0, p)
    assert np.max(np.abs(gax[occ] - ax[occ])) < 1e-15
    assert np.all(gax[~occ] == 0.0)
    xi = srd.thermostat_xi(count, ek, np.arange(p.ncells, dtype=np.uint64), 0, p)
    assert np.allclose(gxi, xi, rtol=1e-12 if form == "fp64" else 1e-9, atol=0)


# ------------------------------------------------------------ collisions
@pytest.mark.parametrize("thermo", [False, True])
def test_one_step_fp64(thermo):
    banner(f"one step fp64 thermo={thermo}")
    p = srd.Params((12, 10, 8), seed=21, thermostat=thermo)
    pos, vel = workloads.fluid(p.n_cells, 6.5, seed=6)
    mass = np.ones(pos.shape[0])
    with _sim(pos, vel, p) as s:
        s.stream()
        s.bin()
        s.collide()
        gpos, gvel = s.get_state()
        assert s.step_count == 1
    opos, ovel, _ = srd.srd_step(pos, vel, mass, p, 0)
    assert np.array_equal(gpos, opos)
    assert vel_err_fp64(gvel, ovel) < FP64_REL


def test_config1_100_steps():
    """The 20^3-cell, 40 000-particle FP64 fluid (no thermostat), 100 steps
    of the fused step path against the oracle."""
    cfg = workloads.CONFIGS["srd_20c_rho5_fp64"]
    banner("config srd_20c_rho5_fp64, 100 steps")
    p = srd.Params(cfg["n_cells"], seed=cfg["seed"], thermostat=cfg["thermostat"])
    pos, vel = workloads.fluid(cfg["n_cells"], cfg["density"], seed=cfg["seed"])
    mass = np.ones(pos.shape[0])
    with _sim(pos, vel, p) as s:
        s.step(cfg["steps"])
        gpos, gvel = s.get_state()
        gcells, gcounts = s.get_cells()
        assert s.step_count == cfg["steps"]
    opos, ovel, info = srd.run(pos, vel, mass, p, 0, cfg["steps"])
    assert np.array_equal(gcells, info["cell"])
    assert np.array_equal(gcounts, info["count"])
    assert vel_err_fp64(gvel, ovel) < FP64_REL
    assert periodic_dist(gpos, opos, p.L).max() < 1e-12


def test_separate_calls_equal_fused_steps():
    banner("separate calls == fused steps")
    p = srd.Params((10, 9, 8), seed=8, thermostat=True)
    pos, vel = workloads.fluid(p.n_cells, 5, seed=9)
    with _sim(pos, vel, p) as a, _sim(pos, vel, p) as b:
        a.step(7)
        for _ in range(7):
            b.stream()
            b.bin()
            b.collide()
        pa, va = a.get_state()
        pb, vb = b.get_state()
    assert np.array_equal(pa, pb) and np.array_equal(va, vb)


def test_deterministic_and_resumable():
    banner("determinism and resume")
    p = srd.Params((11, 11, 11), seed=10, thermostat=True)
    pos, vel = workloads.fluid(p.n_cells, 8, seed=11)
    with _sim(pos, vel, p) as a, _sim(pos, vel, p) as b:
        a.step(20)
        b.step(20)
        pa, va = a.get_state()
        pb, vb = b.get_state()
        assert np.array_equal(pa, pb) and np.array_equal(va, vb)
    with _sim(pos, vel, p) as c:
        c.step(8)
        pc, vc = c.get_state()
    with _sim(pc, vc, p) as d:
        d.step_count = 8
        d.step(12)
        pd, vd = d.get_state()
    assert np.array_equal(pd, pa) and np.array_equal(vd, va)


# ------------------------------------------------------------ edge cases
def test_empty_system():
    banner("empty system")
    p = srd.Params((3, 3, 3))
    with _sim(np.zeros((0, 3)), np.zeros((0, 3)), p) as s:
        s.step(3)
        s.stream()
        s.bin()
        _, counts = s.get_cells()
        assert counts.sum() == 0
        s.collide()
        assert s.step_count == 4


@pytest.mark.parametrize("n", [1, 2, 1001])
def test_ragged_sizes(n):
    banner(f"ragged n={n}")
    p = srd.Params((4, 5, 6), seed=12, thermostat=True)
    rng = np.random.default_rng(n)
    pos = rng.random((n, 3)) * p.L
    vel = rng.normal(size=(n, 3))
    mass = np.ones(n)
    with _sim(pos, vel, p) as s:
        s.step(3)
        gpos, gvel = s.get_state()
    opos, ovel, _ = srd.run(pos, vel, mass, p, 0, 3)
    assert vel_err_fp64(gvel, ovel) < FP64_REL
    assert periodic_dist(gpos, opos, p.L).max() < 1e-12


def test_crowded_cell_overflows_register_staging():
    """3000 particles in one cell: more than a tile block holds in registers
    (1024), so the kernels' global-memory path runs."""
    banner("crowded cell")
    p = srd.Params((4, 4, 4), seed=13, thermostat=True, grid_shift=False, dt=0.01)
    rng = np.random.default_rng(2)
    crowd = 1.2 + 0.6 * rng.random((3000, 3))
    rest = rng.random((500, 3)) * 4.0
    pos = np.concatenate([crowd, rest])
    vel = rng.normal(size=pos.shape) * 0.5
    mass = np.ones(pos.shape[0])
    with _sim(pos, vel, p) as s:
        s.step(2)
        gpos, gvel = s.get_state()
        _, counts = s.get_cells()
    opos, ovel, info = srd.run(pos, vel, mass, p, 0, 2)
    assert counts.max() > 1024
    assert np.array_equal(counts, info["count"])
    assert vel_err_fp64(gvel, ovel) < FP64_REL


def test_embedded_beads_fp64():
    banner("embedded beads")
    p = srd.Params((10, 10, 10), seed=14, thermostat=True)
    pos, vel = workloads.fluid(p.n_cells, 5, seed=15)
    bpos, bvel, bmass = workloads.beads(p.n_cells, 20, 50, seed=16)
    vel, bvel = workloads.zero_net_momentum([vel, bvel], [np.ones(len(vel)), bmass])
    with _sim(pos, vel, p, emb_pos=bpos, emb_vel=bvel, emb_mass=bmass) as s:
        s.step(4)
        gpos, gvel = s.get_state()
        P, ke, _ = s.totals()
    apos = np.concatenate([pos, bpos])
    avel = np.concatenate([vel, bvel])
    amass = np.concatenate([np.ones(len(pos)), bmass])
    opos, ovel, _ = srd.run(apos, avel, amass, p, 0, 4)
    assert vel_err_fp64(gvel, ovel, m=1.0) < FP64_REL
    assert periodic_dist(gpos, opos, p.L).max() < 1e-12
    oP, oke, _ = srd.totals(ovel, amass)
    assert np.allclose(P, oP, atol=1e-10)
    assert abs(ke - oke) < 1e-9 * oke


def test_slab_overflow_regrow_replay():
    """A converging flow piles particles into the central tiles, beyond the
    slab capacity fixed at create (sized to the initial maximum here); the
    library enlarges the slabs and replays the step, and the result still
    matches the oracle."""
    banner("slab regrow")
    p = srd.Params((12, 12, 12), seed=22)
    pos, vel = workloads.fluid(p.n_cells, 9, seed=23)
    vel = vel - (pos - p.L / 2)          # up to 0.6 cells per step inwards
    mass = np.ones(pos.shape[0])
    with _sim(pos, vel, p, flags=m.binding.FLAG_TIGHT_SLABS) as b:
        _, _, cap0, _ = b.layout()
        b.step(6)
        gpos, gvel = b.get_state()
        gcells, _ = b.get_cells()
        _, _, cap1, regrows = b.layout()
    assert regrows >= 1 and cap1 > cap0
    opos, ovel, info = srd.run(pos, vel, mass, p, 0, 6)
    assert np.array_equal(gcells, info["cell"])
    assert vel_err_fp64(gvel, ovel) < FP64_REL
    assert periodic_dist(gpos, opos, p.L).max() < 1e-12


def test_range_errors_and_call_order():
    banner("errors")
    p = srd.Params((4, 4, 4), dt=0.1)
    pos = np.full((3, 3), 1.5)
    vel = np.zeros((3, 3))
    vel[1, 0] = 100.0        # |v dt| = 10 > L = 4
    with _sim(pos, vel, p) as s:
        with pytest.raises(m.MpcdError) as e:
            s.bin()
        assert e.value.status == 5
        s.stream()
        with pytest.raises(m.MpcdError) as e:
            s.sync()
        assert e.value.status == 4
    with pytest.raises(m.MpcdError) as e:
        _sim(np.array([[4.0, 0.0, 0.0]]), np.zeros((1, 3)), p)
    assert e.value.status == 1


# ---------------------------------------------------------------- FP32 form
def test_fp32_one_step_from_shared_state():
    banner("fp32 one step")
    p = srd.Params((16, 12, 10), seed=17, thermostat=True)
    pos, vel = workloads.fluid(p.n_cells, 8, seed=18)
    mass = np.ones(pos.shape[0])
    h, o, v = fp32form.from_double(pos, vel, p)
    with _sim(pos, vel, p, precision=m.FP32) as s:
        gpos0, gvel0 = s.get_state()
        assert np.array_equal(gpos0, fp32form.to_double(h, o, p))
        assert np.array_equal(gvel0, v.astype(np.float64))
        s.step(1)
        gpos, gvel = s.get_state()
        gcells, _ = s.get_cells()
    h1, o1, v1, info = fp32form.step32(h, o, v, mass, p, 0)
    assert np.array_equal(gcells, info["cell"])
    assert np.array_equal(gpos, fp32form.to_double(h1, o1, p))
    assert ulp_diff_f32(gvel.astype(np.float32), v1).max() <= 1


def test_fp32_twenty_steps_each_from_gpu_state():
    """Twenty single-step calls of the thermostatted FP32 form, each checked
    element by element against the emulation of that step from the GPU's
    state before it (cells and positions exact, velocities within one ulp)."""
    banner("fp32 20 steps")
    p = srd.Params((20, 20, 20), seed=19, thermostat=True)
    pos, vel = workloads.fluid(p.n_cells, 5, seed=20)
    mass = np.ones(pos.shape[0])
    with _sim(pos, vel, p, precision=m.FP32) as s:
        gpos, gvel = s.get_state()
        for k in range(20):
            s.step(1)
            gpos1, gvel1 = s.get_state()
            gcells1, _ = s.get_cells()
            fp32_step_matches(gpos, gvel, gpos1, gvel1, gcells1, mass, p, k, fp32form)
            gpos, gvel = gpos1, gvel1


# --------------------------------------------------- full benchmark size
@pytest.mark.parametrize("form", ["fp64"])
def test_full_size_benchmark_fluid_two_steps(form):
    """The 100^3-cell, 10^7-particle thermostatted fluid that the benchmark
    times, in the same launch configuration: two fused steps checked
    element by element against the oracle."""
    cfg = workloads.CONFIGS["srd_100c_rho10_mbthermo"]
    banner(f"full size {form}")
    p = srd.Params(cfg["n_cells"], seed=cfg["seed"], thermostat=True, kT=cfg["kT"])
    pos, vel = workloads.fluid(cfg["n_cells"], cfg["density"], seed=cfg["seed"])
    mass = np.ones(pos.shape[0])
    prec = m.FP64 if form == "fp64" else m.FP32
    with _sim(pos, vel, p, precision=prec) as s:
        s.step(2)
        gpos, gvel = s.get_state()
        gcells, gcounts = s.get_cells()
    if form == "fp64":
        opos, ovel, info = srd.run(pos, vel, mass, p, 0, 2)
        assert np.array_equal(gcells, info["cell"])
        assert vel_err_fp64(gvel, ovel) < FP64_REL
        assert periodic_dist(gpos, opos, p.L).max() < 1e-12
    assert gcounts.sum() == pos.shape[0]


def test_full_size_benchmark_fluid_fp32_each_step():
    """The benchmark's 10^7-particle thermostatted fluid in the FP32 form, in
    the launch configuration the benchmark times: two single-step calls, each
    checked element by element against the emulation of that step from the
    GPU's state before it -- every cell index and position bit-exact, every
    velocity component within one ulp."""
    cfg = workloads.CONFIGS["srd_100c_rho10_mbthermo"]
    banner("full size fp32, each step")
    p = srd.Params(cfg["n_cells"], seed=cfg["seed"], thermostat=True, kT=cfg["kT"])
    pos, vel = workloads.fluid(cfg["n_cells"], cfg["density"], seed=cfg["seed"])
    mass = np.ones(pos.shape[0])
    with _sim(pos, vel, p, precision=m.FP32) as s:
        gpos, gvel = s.get_state()
        for k in range(2):
            s.step(1)
            gpos1, gvel1 = s.get_state()
            gcells1, gcounts = s.get_cells()
            assert gcounts.sum() == pos.shape[0]
            fp32_step_matches(gpos, gvel, gpos1, gvel1, gcells1, mass, p, k, fp32form)
            gpos, gvel = gpos1, gvel1


TILE_SHAPES = {1.2: (8, 8, 4), 5.0: (8, 4, 4), 12.5: (4, 4, 2)}


@pytest.mark.parametrize("rho,n_cells", [(1.2, (19, 11, 10)), (5.0, (17, 9, 10)), (12.5, (9, 10, 7))])
def test_extreme_tile_shapes(rho, n_cells):
    """The tile shapes a box alone takes under the SRD rule at sparse
    densities (8x8x4 cells, 256-cell kernels, below density 3.75; 8x4x4,
    128-cell kernels, below 7.5) and the densest (4x4x2, density 12 and up),
    each with partial tiles on every axis: three thermostatted
    FP64 steps against the oracle, and one FP32 step from a shared state
    against its emulation."""
    banner(f"tile shapes rho={rho} {n_cells}")
    p = srd.Params(n_cells, seed=81, thermostat=True)
    pos, vel = workloads.fluid(n_cells, rho, seed=82)
    mass = np.ones(pos.shape[0])
    with _sim(pos, vel, p) as s:
        tile = s.layout()[0]
        s.step(3)
        gpos, gvel = s.get_state()
        gcells, gcounts = s.get_cells()
    assert tile == TILE_SHAPES[rho]
    opos, ovel, info = srd.run(pos, vel, mass, p, 0, 3)
    assert np.array_equal(gcells, info["cell"])
    assert np.array_equal(gcounts, info["count"])
    assert vel_err_fp64(gvel, ovel) < FP64_REL
    assert periodic_dist(gpos, opos, p.L).max() < 1e-12
    h, o, v = fp32form.from_double(pos, vel, p)
    with _sim(pos, vel, p, precision=m.FP32) as s:
        s.step(1)
        gpos, gvel = s.get_state()
        gcells, _ = s.get_cells()
    h1, o1, v1, info = fp32form.step32(h, o, v, mass, p, 0)
    assert np.array_equal(gcells, info["cell"])
    assert np.array_equal(gpos, fp32form.to_double(h1, o1, p))
    assert ulp_diff_f32(gvel.astype(np.float32), v1).max() <= 1
