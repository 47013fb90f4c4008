"""Shared helpers of the GPU parity tests: tolerances and comparisons."""
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


def f32_close(a, b, abs_tol=FP32_FIXED_ABS):
    """Elementwise: within one FP32 ulp, or within abs_tol absolute."""
    a = np.asarray(a, dtype=np.float32)
    b = np.asarray(b, dtype=np.float32)
    absd = np.abs(a.astype(np.float64) - b.astype(np.float64))
    return (ulp_diff_f32(a, b) <= 1) | (absd <= abs_tol)


def banner(msg):
    print(f"[gpu-test] {msg}", flush=True)
