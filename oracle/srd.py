"""One SRD-MPCD time step in plain FP64 numpy (test infrastructure only).

Follows the paper's order of work for one step (sec. 3, flow diagram Fig. 1):
stream (eq. 1) -> random grid shift and binning into cubic cells (sec. 2,
sec. 3.4) -> cell properties (sec. 3.5, eq. 3) -> per-cell rotation axis and,
optionally, the Maxwell-Boltzmann scale factor (sec. 3.6) -> rotation of the
velocities relative to the cell centre-of-mass velocity (eq. 2, Alg. 1).

Readings of points the paper leaves open:
* box [0, L) per axis with L = n*a, periodic;
* stream uses one FP64 multiply then one FP64 add (no fused multiply-add);
* a wrapped coordinate that rounds to L is set to 0;
* one shift vector per step, each component uniform on (-a/2, a/2), added to
  the positions for binning only;
* cell index x-fastest: c = ix + nx*(iy + ny*iz) on the shifted grid; it is
  the "global cell index" that keys the cell's random numbers;
* Philox4x32-10 counters: (cell, step, purpose, attempt), key = seed;
* axis by the cylindrical (Archimedes) projection z = 2u1 - 1, phi = 2 pi u2;
* thermostat draws E ~ Gamma(3(Nc-1)/2, kT) (centre-of-mass motion removed)
  by Marsaglia-Tsang (with its squeeze test) and a Box-Muller normal (cos
  branch), at most 64 attempts; xi = 1 for Nc < 2 or E_k = 0;
* rotation by +alpha, right-handed (Rodrigues' formula);
* Andersen-thermostat rule (eq. 4, sec. 3.7): per particle a Philox counter
  (tag, step, TAG_AT, 0), Box-Muller on words (0, 1) for two components (cos
  and sin branches) and on words (2, 3) for the third (cos branch), scaled by
  sqrt(kT / m); the cell's mean random velocity is mass-weighted, which is
  the paper's 1/N_c sum for equal masses and conserves momentum with beads.
"""
from dataclasses import dataclass, field
import math

import numpy as np

from .philox import (TAG_AT, TAG_AXIS, TAG_SHIFT, TAG_THERMO, philox4x32_10, seed_key,
                     uniform01)

GAMMA_MAX_ATTEMPTS = 64


@dataclass
class Params:
    """Problem parameters as the paper states them (sec. 2, sec. 4):
    cubic cells of edge a, rotation angle alpha, collision time dt,
    temperature kT, user seed, solvent mass m, thermostat switch."""
    n_cells: tuple
    a: float = 1.0
    alpha: float = 130.0 * math.pi / 180.0
    dt: float = 0.1
    kT: float = 1.0
    seed: int = 1
    solvent_mass: float = 1.0
    thermostat: bool = False
    grid_shift: bool = True
    rule: str = "srd"        # collision rule: "srd" (eq. 2) or "at" (eq. 4)
    # derived constants, computed once on the host (both sides take these
    # values rather than re-deriving them)
    L: np.ndarray = field(init=False)
    inv_a: float = field(init=False)
    cos_a: float = field(init=False)
    sin_a: float = field(init=False)

    def __post_init__(self):
        self.n_cells = tuple(int(x) for x in self.n_cells)
        self.L = np.array([n * self.a for n in self.n_cells], dtype=np.float64)
        self.inv_a = 1.0 / self.a
        self.cos_a = math.cos(self.alpha)
        self.sin_a = math.sin(self.alpha)

    @property
    def ncells(self):
        nx, ny, nz = self.n_cells
        return nx * ny * nz


# ---------------------------------------------------------------- streaming
def wrap(w, L):
    """Map w in (-L, 2L) into [0, L). The subtraction branch is exact
    (Sterbenz); the addition branch can round up to L, which becomes 0."""
    w = np.where(w >= L, w - L, w)
    w = np.where(w < 0.0, w + L, w)
    return np.where(w >= L, 0.0, w)


def stream(pos, vel, p, moving=None):
    """Ballistic streaming r <- r + v*dt in a periodic box (eq. 1). With a
    boolean mask `moving`, only those particles stream; the others (solutes
    integrated by molecular dynamics between collisions, sec. 3.6) keep
    their positions."""
    step = vel * p.dt
    if np.any(np.abs(step) >= p.L):
        raise ValueError("a particle moves a whole box length in one step")
    out = wrap(pos + step, p.L)
    if moving is not None:
        out = np.where(np.asarray(moving)[:, None], out, pos)
    return out


# ------------------------------------------------------------- grid shift
def grid_shift(p, step):
    """Random shift of the collision grid for this step (sec. 2, sec. 3.4):
    one vector, each component uniform on (-a/2, a/2)."""
    if not p.grid_shift:
        return np.zeros(3)
    w = philox4x32_10(np.array([0, step, TAG_SHIFT, 0], dtype=np.uint64),
                      np.array(seed_key(p.seed), dtype=np.uint64))
    u = uniform01(w[:3])
    return (u - 0.5) * p.a


# ----------------------------------------------------------------- binning
def bin_cells(pos, shift, p):
    """Collision cell of each particle: shifted position wrapped into the
    box, per-axis index floor(w / a) (multiplying by the host's 1/a), clamped
    to n - 1, then the x-fastest linear index (sec. 3.4)."""
    w = wrap(pos + shift, p.L)
    idx = np.floor(w * p.inv_a).astype(np.int64)
    n = np.array(p.n_cells, dtype=np.int64)
    idx = np.minimum(idx, n - 1)
    nx, ny, _ = p.n_cells
    return idx[:, 0] + nx * (idx[:, 1] + ny * idx[:, 2])


# ---------------------------------------------------------- cell properties
def cell_sums(cell, vel, mass, ncells):
    """Per-cell particle count N_c, mass M_c, momentum P_c, centre-of-mass
    velocity u = P_c / M_c, and kinetic energy in the centre-of-mass frame
    E_k = 1/2 sum m |v - u|^2 (sec. 3.5, eq. 3), mass-weighted so that
    embedded particles of other masses count correctly (sec. 2, solutes)."""
    count = np.bincount(cell, minlength=ncells)
    M = np.bincount(cell, weights=mass, minlength=ncells)
    P = np.stack([np.bincount(cell, weights=mass * vel[:, d], minlength=ncells)
                  for d in range(3)], axis=1)
    u = np.zeros((ncells, 3))
    occ = M > 0
    u[occ] = P[occ] / M[occ, None]
    dv = vel - u[cell]
    ek = 0.5 * np.bincount(cell, weights=mass * (dv * dv).sum(axis=1),
                           minlength=ncells)
    return count, M, P, u, ek


# -------------------------------------------------------- per-cell draws
def cell_axes(cells, step, p):
    """Random rotation axis of each listed cell, uniform on the unit sphere
    by the cylindrical projection from two uniforms (sec. 3.6)."""
    cells = np.asarray(cells, dtype=np.uint64)
    ctr = np.zeros((cells.size, 4), dtype=np.uint64)
    ctr[:, 0] = cells
    ctr[:, 1] = step
    ctr[:, 2] = TAG_AXIS
    w = philox4x32_10(ctr, np.array(seed_key(p.seed), dtype=np.uint64))
    u1 = uniform01(w[:, 0])
    u2 = uniform01(w[:, 1])
    z = 2.0 * u1 - 1.0
    phi = (2.0 * math.pi) * u2
    r = np.sqrt(np.maximum(0.0, 1.0 - z * z))
    return np.stack([r * np.cos(phi), r * np.sin(phi), z], axis=1)


def gamma_marsaglia_tsang(shape_k, cells, step, p, theta):
    """Gamma(shape_k, scale theta) by Marsaglia and Tsang's rejection method
    with a Box-Muller normal (sec. 3.6, thermostat). Attempt j of a cell uses
    Philox counter (cell, step, TAG_THERMO, j): words 0 and 1 make the normal
    g, word 2 the acceptance uniform U. With t = 1 + c g > 0 and V = t^3 the
    attempt is accepted if U < 1 - 0.0331 g^4 (the method's squeeze, a subset
    of the acceptance region) or log U < g^2/2 + d - d V + d log V; the draw is
    d V theta. Valid for shape_k >= 1 (here >= 1.5).
    Returns (draw, attempts); a cell still rejected after 64 attempts gets
    NaN, which callers treat as an error."""
    shape_k = np.asarray(shape_k, dtype=np.float64)
    cells = np.asarray(cells, dtype=np.uint64)
    d = shape_k - 1.0 / 3.0
    c = 1.0 / np.sqrt(9.0 * d)
    out = np.full(shape_k.shape, np.nan)
    attempts = np.zeros(shape_k.shape, dtype=np.int64)
    todo = np.arange(shape_k.size)
    key = np.array(seed_key(p.seed), dtype=np.uint64)
    for j in range(GAMMA_MAX_ATTEMPTS):
        if todo.size == 0:
            break
        ctr = np.zeros((todo.size, 4), dtype=np.uint64)
        ctr[:, 0] = cells[todo]
        ctr[:, 1] = step
        ctr[:, 2] = TAG_THERMO
        ctr[:, 3] = j
        w = philox4x32_10(ctr, key)
        u0 = uniform01(w[:, 0])
        u1 = uniform01(w[:, 1])
        u2 = uniform01(w[:, 2])
        g = np.sqrt(-2.0 * np.log(u0)) * np.cos((2.0 * math.pi) * u1)
        t = 1.0 + c[todo] * g
        pos = t > 0.0
        V = t * t * t
        dd = d[todo]
        sq = g * g
        squeeze = u2 < 1.0 - 0.0331 * (sq * sq)
        with np.errstate(invalid="ignore", divide="ignore"):
            rhs = 0.5 * g * g + dd - dd * V + dd * np.log(np.where(pos, V, 1.0))
        acc = pos & (squeeze | (np.log(u2) < rhs))
        attempts[todo] = j + 1
        hit = todo[acc]
        out[hit] = dd[acc] * V[acc] * theta
        todo = todo[~acc]
    return out, attempts


def thermostat_xi(count, ek, cells, step, p):
    """Maxwell-Boltzmann cell thermostat scale factor xi = sqrt(E_hat / E_k)
    with E_hat ~ Gamma(3(N_c - 1)/2, kT) (sec. 2, sec. 3.6). Cells with
    fewer than two particles, or with no relative kinetic energy, get 1."""
    xi = np.ones(cells.size)
    act = (count >= 2) & (ek > 0.0)
    if np.any(act):
        k = 1.5 * (count[act] - 1).astype(np.float64)
        e_hat, _ = gamma_marsaglia_tsang(k, cells[act], step, p, p.kT)
        if np.any(np.isnan(e_hat)):
            raise RuntimeError("Gamma sampler exceeded its attempt cap")
        xi[act] = np.sqrt(e_hat / ek[act])
    return xi


# ---------------------------------------------------------------- rotation
def rotate(vel, cell, u, axis, xi, p):
    """SRD collision (eq. 2, Alg. 1): relative velocity dv = v - u rotated by
    +alpha about the cell axis with Rodrigues' formula, scaled by the
    thermostat factor, and added back to u."""
    uc = u[cell]
    n = axis[cell]
    dv = vel - uc
    ndv = (n * dv).sum(axis=1)
    nxd = np.cross(n, dv)
    dvr = dv * p.cos_a + nxd * p.sin_a + n * (ndv * (1.0 - p.cos_a))[:, None]
    dvr = dvr * xi[cell][:, None]
    return uc + dvr


# ------------------------------------------------- Andersen thermostat rule
def at_kicks(tags, step, mass, p):
    """Random velocities of the AT rule (sec. 3.7): per particle the Philox
    words of counter (tag, step, TAG_AT, 0) -> uniforms u0..u3; Box-Muller
    g0 = r0 cos(2 pi u1), g1 = r0 sin(2 pi u1) with r0 = sqrt(-2 ln u0), and
    g2 = sqrt(-2 ln u2) cos(2 pi u3); velocity sqrt(kT / m) (g0, g1, g2)."""
    tags = np.asarray(tags, dtype=np.uint64)
    n = tags.size
    ctr = np.stack([tags, np.full(n, step, dtype=np.uint64),
                    np.full(n, TAG_AT, dtype=np.uint64), np.zeros(n, dtype=np.uint64)],
                   axis=1).astype(np.uint32)
    w = philox4x32_10(ctr, seed_key(p.seed))
    u = uniform01(w)
    r0 = np.sqrt(-2.0 * np.log(u[:, 0]))
    r2 = np.sqrt(-2.0 * np.log(u[:, 2]))
    g = np.stack([r0 * np.cos((2.0 * math.pi) * u[:, 1]),
                  r0 * np.sin((2.0 * math.pi) * u[:, 1]),
                  r2 * np.cos((2.0 * math.pi) * u[:, 3])], axis=1)
    return np.sqrt(p.kT / np.asarray(mass, dtype=np.float64))[:, None] * g


def collide_at(cell, vel, mass, p, step, tags=None, kicks=None):
    """AT collision (eq. 4): v_i <- u + dv_i - sum_j m_j dv_j / M_c, the sums
    over the particles of the cell. `kicks` draws the random velocities
    (default at_kicks; the FP32 form passes its own)."""
    n = vel.shape[0]
    tags = np.arange(n) if tags is None else tags
    count, M, P, u, ek = cell_sums(cell, vel, mass, p.ncells)
    dv = (at_kicks if kicks is None else kicks)(tags, step, mass, p)
    Q = np.stack([np.bincount(cell, weights=mass * dv[:, d], minlength=p.ncells)
                  for d in range(3)], axis=1)
    wmean = np.zeros((p.ncells, 3))
    occ = M > 0
    wmean[occ] = Q[occ] / M[occ, None]
    vnew = u[cell] + dv - wmean[cell]
    return vnew, dict(count=count, mass=M, momentum=P, u=u, ek=ek, kick=dv, kick_mean=wmean)


# -------------------------------------------------------------- whole step
def collide(pos_streamed, vel, mass, p, step):
    """Bin, cell properties, draws and rotation (or the AT rule) for step
    `step`, given already streamed positions. Returns (new velocities, info
    dict)."""
    s = grid_shift(p, step)
    cell = bin_cells(pos_streamed, s, p)
    if p.rule == "at":
        vnew, info = collide_at(cell, vel, mass, p, step)
        info.update(shift=s, cell=cell)
        return vnew, info
    count, M, P, u, ek = cell_sums(cell, vel, mass, p.ncells)
    all_cells = np.arange(p.ncells, dtype=np.uint64)
    axis = cell_axes(all_cells, step, p)
    if p.thermostat:
        xi = thermostat_xi(count, ek, all_cells, step, p)
    else:
        xi = np.ones(p.ncells)
    vnew = rotate(vel, cell, u, axis, xi, p)
    info = dict(shift=s, cell=cell, count=count, mass=M, momentum=P, u=u,
                ek=ek, axis=axis, xi=xi)
    return vnew, info


def srd_step(pos, vel, mass, p, step, moving=None):
    """One full MPCD step: stream (the particles in `moving`, default all),
    then collide with counter `step`."""
    pos1 = stream(pos, vel, p, moving)
    vel1, info = collide(pos1, vel, mass, p, step)
    return pos1, vel1, info


def run(pos, vel, mass, p, step0, nsteps):
    """nsteps consecutive steps with counters step0, step0+1, ..."""
    info = None
    for k in range(nsteps):
        pos, vel, info = srd_step(pos, vel, mass, p, step0 + k)
    return pos, vel, info


# ------------------------------------------------------------ diagnostics
def velocity_field(pos, vel, mass, p):
    """Cell-averaged velocity of a state on the unshifted grid: every particle
    counts in its home cell (the binning of sec. 3.4 with zero shift); per
    cell the mass-weighted mean velocity sum(m v) / sum(m), 0 where the cell
    is empty, and the cell's mass (sec. 3.5 cell properties)."""
    cell = bin_cells(pos, np.zeros(3), p)
    _, M, P, u, _ = cell_sums(cell, vel, mass, p.ncells)
    return u, M


def totals(vel, mass):
    """Net momentum, kinetic energy, and the kinetic temperature of the
    motion relative to the centre of mass, 2 (KE - |P|^2 / 2M) / (3 (N - 1))
    (sec. 3.5, net properties by a reduction over the system)."""
    P = (mass[:, None] * vel).sum(axis=0)
    ke = 0.5 * (mass * (vel * vel).sum(axis=1)).sum()
    n = vel.shape[0]
    M = mass.sum()
    kT = 2.0 * (ke - 0.5 * (P * P).sum() / M) / (3.0 * (n - 1)) if n > 1 else 0.0
    return P, ke, kT
