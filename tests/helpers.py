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


def banner(msg):
    print(f"[gpu-test] {msg}", flush=True)
