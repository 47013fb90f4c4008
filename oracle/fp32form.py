"""Emulation of the FP32 cell-relative storage form (test infrastructure).

The paper's mixed-precision model stores positions and velocities in single
precision and upcasts to FP64 for the cell reductions and the rotation
(sec. 3.5, sec. 3.6 and Alg. 1, sec. 4.1). The GPU form checked here keeps
each particle's position as an integer home cell h (per axis) plus an FP32
offset o in [0, a) inside it, so that the offset keeps full single precision
anywhere in a large box; velocities are FP32.

Every single-precision operation below is a numpy float32 operation (IEEE
binary32, round to nearest, one rounding per operation, no contraction):
  stream: t = v*dt32; o1 = o + t; k = floor(o1*inv_a32); o2 = o1 - k*a32;
          o2 >= a32 -> o2 = 0, k += 1;  o2 < 0 -> o2 = 0;  h = (h + k) mod n
  bin:    q = o + s32; j = floor(q*inv_a32) clamped to [-1, 1];
          cell = (h + j) mod n per axis
  collide: v upcast to FP64; sums, draws and rotation in FP64 exactly as the
          FP64 oracle; the result rounded once to FP32. Under the AT rule the
          kicks are the form's single-precision ones (at_kicks32).
with dt32 = fl32(dt), a32 = fl32(a), inv_a32 = fl32(fl64(1/a)), s32 = fl32(s).
"""
import math

import numpy as np

from . import srd
from .philox import TAG_AT, philox4x32_10, seed_key


def uniform23(w):
    """The FP32 form's uniforms: u = (floor(w / 2^9) + 1/2) 2^-23, from the top
    23 bits of a 32-bit word; exact in FP32, strictly inside (0, 1)."""
    return ((np.asarray(w, dtype=np.uint64) >> np.uint64(9)).astype(np.float64) + 0.5) * 2.0 ** -23


def at_kicks32(tags, step, mass, p):
    """Random velocities of the AT rule in the FP32 form (sec. 3.7 with the
    mixed-precision model of sec. 4.1, which keeps double precision for the
    cell sums and the rotation only): the words of counter (tag, step,
    TAG_AT, 0) as in the FP64 form, uniforms by uniform23, the same
    Box-Muller pairing, and the scale sqrt(kT / m) rounded to FP32. Returned
    as the exact value of that formula (FP64 evaluation from the same
    uniforms and scale); the GPU evaluates it in single precision, which
    differs from it by the rounding of a few single-precision operations."""
    tags = np.asarray(tags, dtype=np.uint64)
    n = tags.size
    ctr = np.stack([tags, np.full(n, step, dtype=np.uint64),
                    np.full(n, TAG_AT, dtype=np.uint64), np.zeros(n, dtype=np.uint64)],
                   axis=1).astype(np.uint32)
    w = philox4x32_10(ctr, seed_key(p.seed))
    u = uniform23(w)
    r0 = np.sqrt(-2.0 * np.log(u[:, 0]))
    r2 = np.sqrt(-2.0 * np.log(u[:, 2]))
    g = np.stack([r0 * np.cos((2.0 * math.pi) * u[:, 1]),
                  r0 * np.sin((2.0 * math.pi) * u[:, 1]),
                  r2 * np.cos((2.0 * math.pi) * u[:, 3])], axis=1)
    scale = np.sqrt(p.kT / np.asarray(mass, dtype=np.float64)).astype(np.float32).astype(np.float64)
    return scale[:, None] * g


def constants32(p):
    return np.float32(p.dt), np.float32(p.a), np.float32(p.inv_a)


def from_double(pos, vel, p):
    """FP64 positions -> (home cell per axis, FP32 offset): h = floor(x/a)
    clamped to [0, n-1]; o = fl32(x - h*a) with the subtraction in FP64; an
    offset that rounds up to a32 moves to the next cell at offset 0, and a
    negative one becomes 0."""
    n = np.array(p.n_cells, dtype=np.int64)
    _, a32, _ = constants32(p)
    h = np.floor(pos * p.inv_a).astype(np.int64)
    h = np.clip(h, 0, n - 1)
    o = (pos - h.astype(np.float64) * p.a).astype(np.float32)
    over = o >= a32
    o = np.where(over, np.float32(0.0), o)
    h = np.where(over, (h + 1) % n, h)
    o = np.maximum(o, np.float32(0.0))
    return h, o.astype(np.float32), vel.astype(np.float32)


def to_double(h, o, p):
    """Position in FP64: x = h*a + o (FP64 multiply, then FP64 add)."""
    return h.astype(np.float64) * p.a + o.astype(np.float64)


def stream32(h, o, v, p):
    dt32, a32, inv_a32 = constants32(p)
    n = np.array(p.n_cells, dtype=np.int64)
    t = v * dt32
    o1 = o + t
    k = np.floor(o1 * inv_a32)
    o2 = o1 - k * a32
    over = o2 >= a32
    o2 = np.where(over, np.float32(0.0), o2)
    k = k.astype(np.int64) + over.astype(np.int64)
    o2 = np.where(o2 < np.float32(0.0), np.float32(0.0), o2).astype(np.float32)
    h = np.mod(h + k, n)
    return h, o2


def bin32(h, o, shift, p):
    _, _, inv_a32 = constants32(p)
    n = np.array(p.n_cells, dtype=np.int64)
    s32 = np.asarray(shift, dtype=np.float64).astype(np.float32)
    q = o + s32
    j = np.floor(q * inv_a32).astype(np.int64)
    j = np.clip(j, -1, 1)
    c = np.mod(h + j, n)
    nx, ny, _ = p.n_cells
    return c[:, 0] + nx * (c[:, 1] + ny * c[:, 2])


def collide32(h, o, v, mass, p, step):
    s = srd.grid_shift(p, step)
    cell = bin32(h, o, s, p)
    v64 = v.astype(np.float64)
    if p.rule == "at":
        vnew, info = srd.collide_at(cell, v64, mass, p, step, kicks=at_kicks32)
        info.update(shift=s, cell=cell)
        return vnew.astype(np.float32), info
    count, M, P, u, ek = srd.cell_sums(cell, v64, mass, p.ncells)
    all_cells = np.arange(p.ncells, dtype=np.uint64)
    axis = srd.cell_axes(all_cells, step, p)
    if p.thermostat:
        xi = srd.thermostat_xi(count, ek, all_cells, step, p)
    else:
        xi = np.ones(p.ncells)
    vnew = srd.rotate(v64, cell, u, axis, xi, p).astype(np.float32)
    info = dict(shift=s, cell=cell, count=count, mass=M, momentum=P, u=u,
                ek=ek, axis=axis, xi=xi, vnew64=None)
    return vnew, info


def step32(h, o, v, mass, p, step):
    h, o = stream32(h, o, v, p)
    v, info = collide32(h, o, v, mass, p, step)
    return h, o, v, info


def run32(h, o, v, mass, p, step0, nsteps):
    info = None
    for k in range(nsteps):
        h, o, v, info = step32(h, o, v, mass, p, step0 + k)
    return h, o, v, info
