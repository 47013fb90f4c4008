"""Pins of the FP32 cell-relative emulation (CPU only)."""
import numpy as np

import workloads
from oracle import fp32form, srd


def test_float32_ops_equal_rounded_double_ops():
    """numpy float32 + - * equal the FP64 result rounded once to FP32:
    double rounding through binary64 is innocuous for binary32 operands
    because 53 >= 2*24 + 2 (Figueroa, 1995)."""
    rng = np.random.default_rng(0)
    a = (rng.normal(size=200000) * 10.0 ** rng.integers(-3, 3, 200000)).astype(np.float32)
    b = (rng.normal(size=200000) * 10.0 ** rng.integers(-3, 3, 200000)).astype(np.float32)
    A, B = a.astype(np.float64), b.astype(np.float64)
    assert np.array_equal(a + b, (A + B).astype(np.float32))
    assert np.array_equal(a - b, (A - B).astype(np.float32))
    assert np.array_equal(a * b, (A * B).astype(np.float32))


def test_from_double_roundtrip():
    p = srd.Params((7, 5, 9), a=1.0)
    pos, vel = workloads.fluid(p.n_cells, 6, seed=3)
    h, o, v = fp32form.from_double(pos, vel, p)
    assert np.all((o >= 0) & (o < np.float32(p.a)))
    assert np.all((h >= 0) & (h < np.array(p.n_cells)))
    back = fp32form.to_double(h, o, p)
    d = np.abs(back - pos)
    d = np.minimum(d, p.L - d)          # periodic distance
    assert d.max() <= 2.0 ** -24


def test_stream_and_bin_track_fp64():
    """One FP32 stream + bin from the FP32 state agrees with the FP64 form
    started from the same (exactly representable) state, except for
    particles within FP32 rounding of a cell face."""
    p = srd.Params((10, 10, 10), seed=4)
    pos, vel = workloads.fluid(p.n_cells, 5, seed=5)
    h, o, v = fp32form.from_double(pos, vel, p)
    x = fp32form.to_double(h, o, p)
    v64 = v.astype(np.float64)
    h1, o1 = fp32form.stream32(h, o, v, p)
    x1 = srd.stream(x, v64, p)
    d = np.abs(fp32form.to_double(h1, o1, p) - x1)
    d = np.minimum(d, p.L - d)
    assert d.max() < 1e-6
    s = srd.grid_shift(p, 0)
    c32 = fp32form.bin32(h1, o1, s, p)
    c64 = srd.bin_cells(x1, s, p)
    bad = np.nonzero(c32 != c64)[0]
    assert bad.size < 5
    w = srd.wrap(x1[bad] + s, p.L)
    frac = np.abs(w - np.round(w))
    assert np.all(frac.min(axis=1) < 1e-5)


def test_collide32_close_to_fp64():
    p = srd.Params((8, 8, 8), seed=6, thermostat=True)
    pos, vel = workloads.fluid(p.n_cells, 7, seed=6)
    h, o, v = fp32form.from_double(pos, vel, p)
    mass = np.ones(pos.shape[0])
    v1, info = fp32form.collide32(h, o, v, mass, p, 2)
    vref, _ = srd.collide(fp32form.to_double(h, o, p), v.astype(np.float64), mass, p, 2)
    # the FP32 form differs only by the final rounding (when cells agree)
    same = info["cell"] == srd.bin_cells(fp32form.to_double(h, o, p), srd.grid_shift(p, 2), p)
    assert same.mean() > 0.999
    ulp = np.spacing(np.abs(v1[same]).astype(np.float32)).astype(np.float64)
    assert np.all(np.abs(v1[same].astype(np.float64) - vref[same]) <= ulp)
