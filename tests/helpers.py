"""Shared helpers of the GPU parity tests: tolerances and comparisons."""
import ctypes

import numpy as np

# Velocity tolerance of the FP64 form: per particle,
# |v_gpu - v_oracle|_inf <= 1e-12 * max(|v_oracle|_inf, sqrt(kT/m)).
FP64_REL = 1e-12


def vel_err_fp64(v_gpu, v_ora, kT=1.0, m=1.0):
    scale = np.maximum(np.abs(v_ora).max(axis=1), np.sqrt(kT / m))
    return (np.abs(v_gpu - v_ora).max(axis=1) / scale).max() if v_ora.size else 0.0


def periodic_dist(a, b, L):
    d = np.abs(a - b)
    return np.minimum(d, L - d)


def ulp_diff_f32(a, b):
    """Distance in units in the last place between two float32 arrays."""
    ai = np.asarray(a, dtype=np.float32).view(np.int32).astype(np.int64)
    bi = np.asarray(b, dtype=np.float32).view(np.int32).astype(np.int64)
    ai = np.where(ai < 0, -(ai & 0x7FFFFFFF), ai)
    bi = np.where(bi < 0, -(bi & 0x7FFFFFFF), bi)
    return np.abs(ai - bi)


# Absolute resolution of the FP32 form's fixed-point cell sums (one limb,
# 2^-40): a term that is an FP64 value (an AT kick, a relative kinetic energy)
# is rounded to it, so a cell mean carries an absolute error of at most 2^-41.
# Against the oracle's FP64 sums an FP32 result is then within one ulp, or,
# for results within ~1e-6 of zero, where an ulp is below that error, within
# 2^-40 absolute.
FP32_FIXED_ABS = 2.0 ** -40

# The FP32 form draws AT kicks in single precision (logf, sqrtf, sincospif,
# cospif and three products); the oracle evaluates the same formula from the
# same uniforms exactly. With the device library's single-precision functions
# within 2 ulps and correctly rounded products and square root, a kick is
# within about 5 ulps of the exact value; 8 ulps (2^-20 relative) is the
# bound used.
AT32_KICK_REL = 2.0 ** -20


def at32_close(g, v, info):
    """FP32 form under the AT rule, elementwise: within one ulp of the
    emulation, or within one ulp plus 2^-20 of the particle's own kick and of
    the largest kick in its cell (the kick enters the velocity once and the
    cell's mean kick once), plus 2^-40."""
    g = np.asarray(g, dtype=np.float64)
    v32 = np.asarray(v, dtype=np.float32)
    kick = np.abs(info["kick"])
    cell = info["cell"]
    kmax = np.zeros((int(cell.max()) + 1 if cell.size else 1, 3))
    np.maximum.at(kmax, cell, kick)
    tol = (np.spacing(np.abs(v32)).astype(np.float64) +
           AT32_KICK_REL * (kick + kmax[cell]) + FP32_FIXED_ABS)
    return (ulp_diff_f32(g.astype(np.float32), v32) <= 1) | (np.abs(g - v32.astype(np.float64)) <= tol)


def at32_kick_units(g, v, info):
    """For reports: the largest difference beyond one ulp of the velocity, in
    FP32 ulps of the kicks it may come from (|own kick| + largest in the
    cell); at32_close allows 8."""
    v32 = np.asarray(v, dtype=np.float32)
    kick = np.abs(info["kick"])
    cell = info["cell"]
    kmax = np.zeros((int(cell.max()) + 1 if cell.size else 1, 3))
    np.maximum.at(kmax, cell, kick)
    d = np.abs(np.asarray(g, dtype=np.float64) - v32.astype(np.float64))
    excess = np.maximum(d - np.spacing(np.abs(v32)).astype(np.float64), 0.0)
    return float((excess / (2.0 ** -23 * (kick + kmax[cell]))).max()) if d.size else 0.0


def f32_close(a, b, abs_tol=FP32_FIXED_ABS):
    """Elementwise: within one FP32 ulp, or within abs_tol absolute."""
    a = np.asarray(a, dtype=np.float32)
    b = np.asarray(b, dtype=np.float32)
    absd = np.abs(a.astype(np.float64) - b.astype(np.float64))
    return (ulp_diff_f32(a, b) <= 1) | (absd <= abs_tol)


def fp32_step_matches(gpos0, gvel0, gpos1, gvel1, gcells1, mass, p, step, fp32form):
    """One FP32-form step checked element by element from the GPU's own state
    before it (read back exactly: h a + o and FP32 velocities are exact in
    FP64 for a = 1): cells and positions bit-exact, every velocity component
    within one FP32 ulp of the oracle's emulation of that step, or within
    2^-40 absolute (the resolution of the form's one-limb cell sums, which
    exceeds an ulp only for results within ~1e-6 of zero). Checking each
    step from the GPU's state keeps the check strict over many steps, where a
    one-ulp difference could otherwise move a particle across a cell face and
    part the two trajectories."""
    h, o, v = fp32form.from_double(gpos0, gvel0, p)
    assert np.array_equal(fp32form.to_double(h, o, p), gpos0), "FP32 state does not round-trip"
    assert np.array_equal(v.astype(np.float64), gvel0)
    h1, o1, v1, info = fp32form.step32(h, o, v, mass, p, step)
    assert np.array_equal(gcells1, info["cell"])
    assert np.array_equal(gpos1, fp32form.to_double(h1, o1, p))
    close = f32_close(gvel1, v1)
    if not np.all(close):
        bad = ~close
        g32 = np.asarray(gvel1, dtype=np.float32)
        raise AssertionError(
            f"step {step}: {bad.sum()} velocity components beyond one ulp and 2^-40: "
            f"ulps {ulp_diff_f32(g32[bad], v1[bad])[:8]}, oracle {v1[bad][:8]}, "
            f"gpu {g32[bad][:8]}")
    return info


def banner(msg):
    print(f"[gpu-test] {msg}", flush=True)


class PoolHighWater:
    """High-water mark of the device's default stream-ordered memory pool
    (where the library's allocations come from), read through the HIP
    runtime that torch loaded."""

    def __init__(self):
        import torch
        torch.cuda.init()
        self.hip = ctypes.CDLL("libamdhip64.so")
        self.pool = ctypes.c_void_p()
        dev = torch.cuda.current_device()
        assert self.hip.hipDeviceGetDefaultMemPool(ctypes.byref(self.pool), dev) == 0

    def reset(self):
        zero = ctypes.c_uint64(0)
        assert self.hip.hipMemPoolSetAttribute(self.pool, 8, ctypes.byref(zero)) == 0  # UsedMemHigh

    def used(self, attr):
        v = ctypes.c_uint64(0)
        assert self.hip.hipMemPoolGetAttribute(self.pool, attr, ctypes.byref(v)) == 0
        return v.value

    def current(self):
        return self.used(7)  # UsedMemCurrent

    def high(self):
        return self.used(8)  # UsedMemHigh since the last reset
