"""Seeded synthetic inputs shared by the oracle tests and the GPU tests.

This module only draws random inputs; it holds none of the method's
arithmetic. The recipe follows the paper's benchmark fluid (sec. 4): point
particles of mass m placed uniformly at random in a cubic periodic box,
Gaussian velocities at temperature kT, and a constant shift that removes the
net momentum. Embedded beads (sec. 2, solutes) are laid out as random walks.

Everything is drawn from numpy.random.default_rng(seed) in a fixed order, so
the same seed gives the same input on every machine.
"""
import math

import numpy as np

DEG130 = 130.0 * math.pi / 180.0


def _uniform_positions(rng, n, L):
    pos = rng.random((n, 3)) * L
    # rng.random() < 1, but the product can round up to L for some L
    return np.where(pos >= L, 0.0, pos)


def fluid(n_cells, density, kT=1.0, mass=1.0, seed=1, a=1.0):
    """Uniform positions in [0, L)^3, velocities N(0, kT/m) per component,
    then the mean velocity subtracted so the net momentum is zero (sec. 4.1:
    a constant correction on every particle). N = round(density * cells)."""
    n_cells = tuple(int(x) for x in np.broadcast_to(n_cells, (3,)))
    L = np.array(n_cells, dtype=np.float64) * a
    n = int(round(density * n_cells[0] * n_cells[1] * n_cells[2]))
    rng = np.random.default_rng(seed)
    pos = _uniform_positions(rng, n, L)
    vel = rng.normal(0.0, math.sqrt(kT / mass), size=(n, 3))
    vel -= vel.mean(axis=0)
    return pos, vel


def beads(n_cells, n_chains, chain_len, bond=0.97, kT=1.0, mass=5.0, seed=2,
          a=1.0):
    """Random-walk chains of beads: the first bead uniform in the box, each
    next bead one bond length away in a uniformly random direction, wrapped
    into the box; velocities N(0, kT/mass). Returns (pos, vel, mass)."""
    n_cells = tuple(int(x) for x in np.broadcast_to(n_cells, (3,)))
    L = np.array(n_cells, dtype=np.float64) * a
    rng = np.random.default_rng(seed)
    n = n_chains * chain_len
    start = _uniform_positions(rng, n_chains, L)
    steps = rng.normal(size=(n_chains, chain_len - 1, 3))
    steps *= bond / np.linalg.norm(steps, axis=2, keepdims=True)
    walk = np.concatenate([start[:, None, :],
                           start[:, None, :] + np.cumsum(steps, axis=1)], axis=1)
    pos = np.mod(walk.reshape(n, 3), L)
    pos = np.where(pos >= L, 0.0, pos)
    vel = rng.normal(0.0, math.sqrt(kT / mass), size=(n, 3))
    return pos, vel, np.full(n, float(mass))


def zero_net_momentum(vel_list, mass_list):
    """Subtract the common centre-of-mass velocity from every group so the
    total momentum of all groups together is zero."""
    P = sum((m[:, None] * v).sum(axis=0) for v, m in zip(vel_list, mass_list))
    M = sum(m.sum() for m in mass_list)
    return [v - P / M for v in vel_list]


def non_gaussian_fluid(n_cells, density, kT=1.0, mass=1.0, seed=1, a=1.0):
    """Same positions as `fluid`, but every speed equal to sqrt(3 kT / m)
    with uniformly random directions (a far-from-Maxwellian start), then the
    net momentum removed."""
    n_cells = tuple(int(x) for x in np.broadcast_to(n_cells, (3,)))
    L = np.array(n_cells, dtype=np.float64) * a
    n = int(round(density * n_cells[0] * n_cells[1] * n_cells[2]))
    rng = np.random.default_rng(seed)
    pos = _uniform_positions(rng, n, L)
    d = rng.normal(size=(n, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    vel = d * math.sqrt(3.0 * kT / mass)
    vel -= vel.mean(axis=0)
    return pos, vel


def replica_boxes(n_rep=256, seed=1, side=(8, 64), density=(5.0, 10.0), kT=(0.5, 2.0)):
    """Parameters of a batch of independent boxes: side n_r uniform on the
    integers side[0]..side[1], density uniform, kT uniform, seed 1 + r (the
    box's Philox key). Returns dicts with n_cells, density, kT, seed; the
    particles come from fluid() with seed 1000 + r."""
    rng = np.random.default_rng(seed)
    n = rng.integers(side[0], side[1] + 1, size=n_rep)
    rho = rng.uniform(density[0], density[1], size=n_rep)
    t = rng.uniform(kT[0], kT[1], size=n_rep)
    return [dict(n_cells=(int(n[r]),) * 3, density=float(rho[r]), kT=float(t[r]),
                 seed=1 + r) for r in range(n_rep)]


def replica_inputs(boxes):
    """Add pos/vel drawn by fluid() (seed 1000 + r) to each box dict."""
    out = []
    for r, b in enumerate(boxes):
        pos, vel = fluid(b["n_cells"], b["density"], kT=b["kT"], seed=1000 + r)
        out.append(dict(b, pos=pos, vel=vel))
    return out


def serve_requests(rate=50.0, duration=60.0, seed=1, n_range=(1e4, 1e7),
                   density=(5.0, 10.0), steps=(100, 2000)):
    """Open-loop request stream: Poisson arrivals at `rate` per second over
    `duration` seconds (exponential gaps); per request N log-uniform on
    n_range, density uniform, cells per axis max(2, round((N / rho)^(1/3))),
    steps uniform on the integers steps[0]..steps[1], seed 1 + i. Returns a
    list of dicts (t, n_cells, density, steps, seed); particles come from
    fluid() with seed 5000 + i."""
    rng = np.random.default_rng(seed)
    out = []
    t = 0.0
    i = 0
    while True:
        t += rng.exponential(1.0 / rate)
        if t >= duration:
            break
        N = math.exp(rng.uniform(math.log(n_range[0]), math.log(n_range[1])))
        rho = rng.uniform(density[0], density[1])
        n = max(2, int(round((N / rho) ** (1.0 / 3.0))))
        k = int(rng.integers(steps[0], steps[1] + 1))
        out.append(dict(t=t, n_cells=(n, n, n), density=float(rho), steps=k, seed=1 + i))
        i += 1
    return out


# Named workloads of the benchmark suite (sizes of the paper's benchmark
# fluid, sec. 4 and Table 1, scaled to one GPU).
CONFIGS = {
    "srd_20c_rho5_fp64": dict(n_cells=(20, 20, 20), density=5, kT=1.0,
                              thermostat=False, steps=100, seed=1),
    "srd_100c_rho10_mbthermo": dict(n_cells=(100, 100, 100), density=10,
                                    kT=1.0, thermostat=True, steps=1000,
                                    seed=1),
    "srd_400c_rho5_beads": dict(n_cells=(400, 400, 400), density=5, kT=1.0,
                                thermostat=False, steps=200, seed=1,
                                chains=20000, chain_len=50, bead_mass=5.0),
    # the same box with the beads coupled to MD (MPCD_FLAG_MD_SOLUTE): 50
    # velocity-Verlet steps of 0.002 per collision, state exchanged on device
    # buffers every collision
    "srd_400c_rho5_md": dict(n_cells=(400, 400, 400), density=5, kT=1.0,
                             thermostat=False, steps=50, seed=1,
                             chains=20000, chain_len=50, bead_mass=5.0),
    # 256 independent boxes (replica_boxes): sides 8..64 cells, densities
    # 5..10, kT 0.5..2, Maxwell-Boltzmann thermostat, FP32
    "srd_batch256_fp32": dict(n_rep=256, thermostat=True, steps=500, seed=1),
    # open-loop serving (serve_requests): 50 requests/s for 60 s, each a
    # thermostatted FP32 box returning its cell-averaged velocity field
    "srd_serve_poisson50": dict(rate=50.0, duration=60.0, seed=1, thermostat=True, kT=1.0),
}
