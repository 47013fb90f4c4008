"""Pure-Python brute force of one SRD step for boxes of a few cells.

Particle by particle and cell by cell, with Python floats for the
per-particle arithmetic and exact rational arithmetic (fractions.Fraction)
for the cell sums, so the centre-of-mass velocity is the correctly rounded
value of the exact mass-weighted mean (sec. 3.5). The random numbers come
from the scalar Philox. Cross products and dot products are written out
component by component. Used only to pin the vectorised oracle on tiny
inputs; it is far too slow for anything else.
"""
from fractions import Fraction
import math

from .philox import (TAG_AT, TAG_AXIS, TAG_SHIFT, TAG_THERMO, philox_scalar, seed_key,
                     uniform01_scalar)
from .srd import GAMMA_MAX_ATTEMPTS


def _wrap(w, L):
    if w >= L:
        w = w - L
    elif w < 0.0:
        w = w + L
        if w >= L:
            w = 0.0
    return w


def _gamma(k, cell, step, p):
    d = k - 1.0 / 3.0
    c = 1.0 / math.sqrt(9.0 * d)
    key = seed_key(p.seed)
    for j in range(GAMMA_MAX_ATTEMPTS):
        w = philox_scalar((cell, step, TAG_THERMO, j), key)
        u0, u1, u2 = (uniform01_scalar(x) for x in w[:3])
        g = math.sqrt(-2.0 * math.log(u0)) * math.cos((2.0 * math.pi) * u1)
        t = 1.0 + c * g
        if t <= 0.0:
            continue
        V = t * t * t
        sq = g * g
        if u2 < 1.0 - 0.0331 * (sq * sq):
            return d * V * p.kT
        if math.log(u2) < 0.5 * g * g + d - d * V + d * math.log(V):
            return d * V * p.kT
    raise RuntimeError("Gamma sampler exceeded its attempt cap")


def brute_step(pos, vel, mass, p, step):
    """pos, vel: lists of [x, y, z]; mass: list. Returns (pos', vel', cells,
    per-cell dict). Follows eq. 1, the shifted binning of sec. 3.4, eq. 3,
    the draws of sec. 3.6 and Alg. 1."""
    L = [n * p.a for n in p.n_cells]
    nx, ny, nz = p.n_cells
    key = seed_key(p.seed)
    # stream (eq. 1)
    newpos = []
    for r, v in zip(pos, vel):
        newpos.append([_wrap(r[d] + v[d] * p.dt, L[d]) for d in range(3)])
    # shift and bin
    if p.grid_shift:
        w = philox_scalar((0, step, TAG_SHIFT, 0), key)
        s = [(uniform01_scalar(w[d]) - 0.5) * p.a for d in range(3)]
    else:
        s = [0.0, 0.0, 0.0]
    cells = []
    for r in newpos:
        ijk = []
        for d in range(3):
            wd = _wrap(r[d] + s[d], L[d])
            ijk.append(min(int(math.floor(wd * p.inv_a)), p.n_cells[d] - 1))
        cells.append(ijk[0] + nx * (ijk[1] + ny * ijk[2]))
    members = {}
    for i, c in enumerate(cells):
        members.setdefault(c, []).append(i)
    newvel = [list(v) for v in vel]
    props = {}
    for c, idx in members.items():
        M = sum(Fraction(mass[i]) for i in idx)
        P = [sum(Fraction(mass[i]) * Fraction(vel[i][d]) for i in idx)
             for d in range(3)]
        u = [float(P[d] / M) for d in range(3)]
        ek = 0.5 * math.fsum(mass[i] * ((vel[i][0] - u[0]) ** 2 +
                                         (vel[i][1] - u[1]) ** 2 +
                                         (vel[i][2] - u[2]) ** 2)
                             for i in idx)
        w = philox_scalar((c, step, TAG_AXIS, 0), key)
        z = 2.0 * uniform01_scalar(w[0]) - 1.0
        phi = (2.0 * math.pi) * uniform01_scalar(w[1])
        rr = math.sqrt(max(0.0, 1.0 - z * z))
        n = [rr * math.cos(phi), rr * math.sin(phi), z]
        xi = 1.0
        if p.thermostat and len(idx) >= 2 and ek > 0.0:
            xi = math.sqrt(_gamma(1.5 * (len(idx) - 1), c, step, p) / ek)
        for i in idx:
            dv = [vel[i][d] - u[d] for d in range(3)]
            ndv = n[0] * dv[0] + n[1] * dv[1] + n[2] * dv[2]
            nxd = [n[1] * dv[2] - n[2] * dv[1],
                   n[2] * dv[0] - n[0] * dv[2],
                   n[0] * dv[1] - n[1] * dv[0]]
            for d in range(3):
                rot = (dv[d] * p.cos_a + nxd[d] * p.sin_a
                       + n[d] * ndv * (1.0 - p.cos_a))
                newvel[i][d] = u[d] + xi * rot
        props[c] = dict(count=len(idx), mass=float(M), u=u, ek=ek, axis=n,
                        xi=xi)
    return newpos, newvel, cells, s, props


def brute_at_step(pos, vel, mass, p, step):
    """One step with the Andersen-thermostat rule (eq. 4, sec. 3.7), particle
    by particle: stream and bin as brute_step, then per particle a random
    velocity from the scalar Philox (counter (tag, step, TAG_AT, 0), tag =
    list index) by Box-Muller, and v <- u + dv - (sum_j m_j dv_j) / M_c with
    u and the random mean as exact rational sums rounded once."""
    L = [n * p.a for n in p.n_cells]
    nx, ny, _ = p.n_cells
    key = seed_key(p.seed)
    newpos = [[_wrap(r[d] + v[d] * p.dt, L[d]) for d in range(3)] for r, v in zip(pos, vel)]
    if p.grid_shift:
        w = philox_scalar((0, step, TAG_SHIFT, 0), key)
        s = [(uniform01_scalar(w[d]) - 0.5) * p.a for d in range(3)]
    else:
        s = [0.0, 0.0, 0.0]
    cells = []
    for r in newpos:
        ijk = [min(int(math.floor(_wrap(r[d] + s[d], L[d]) * p.inv_a)), p.n_cells[d] - 1)
               for d in range(3)]
        cells.append(ijk[0] + nx * (ijk[1] + ny * ijk[2]))
    kicks = []
    for i in range(len(pos)):
        u = [uniform01_scalar(x) for x in philox_scalar((i, step, TAG_AT, 0), key)]
        r0 = math.sqrt(-2.0 * math.log(u[0]))
        r2 = math.sqrt(-2.0 * math.log(u[2]))
        g = [r0 * math.cos((2.0 * math.pi) * u[1]), r0 * math.sin((2.0 * math.pi) * u[1]),
             r2 * math.cos((2.0 * math.pi) * u[3])]
        sc = math.sqrt(p.kT / mass[i])
        kicks.append([sc * x for x in g])
    members = {}
    for i, c in enumerate(cells):
        members.setdefault(c, []).append(i)
    newvel = [list(v) for v in vel]
    for c, idx in members.items():
        M = sum(Fraction(mass[i]) for i in idx)
        u = [float(sum(Fraction(mass[i]) * Fraction(vel[i][d]) for i in idx) / M) for d in range(3)]
        wm = [float(sum(Fraction(mass[i]) * Fraction(kicks[i][d]) for i in idx) / M) for d in range(3)]
        for i in idx:
            newvel[i] = [u[d] + kicks[i][d] - wm[d] for d in range(3)]
    return newpos, newvel, cells
