"""A small molecular-dynamics integrator for bead chains, standing in for the
external MD engine that moves solutes between MPCD collisions (sec. 3.6):
harmonic bonds U = k/2 (|r_{i+1} - r_i| - b)^2 along each chain (minimum
image in the periodic box), velocity Verlet. Test infrastructure, used the
same way in the oracle run and the GPU run."""
import numpy as np


def bond_forces(pos, chain_len, L, k=30.0, b=0.97):
    n = pos.shape[0]
    f = np.zeros_like(pos)
    idx = np.arange(n).reshape(-1, chain_len)
    i, j = idx[:, :-1].ravel(), idx[:, 1:].ravel()
    d = pos[j] - pos[i]
    d -= L * np.round(d / L)
    r = np.linalg.norm(d, axis=1)
    fmag = -k * (r - b) / r
    fij = fmag[:, None] * d          # force on j
    np.add.at(f, j, fij)
    np.add.at(f, i, -fij)
    return f


def verlet(pos, vel, mass, chain_len, L, dt, nsteps):
    """nsteps velocity-Verlet steps of size dt; positions wrapped into [0, L)."""
    pos, vel = pos.copy(), vel.copy()
    m = mass[:, None]
    f = bond_forces(pos, chain_len, L)
    for _ in range(nsteps):
        vel += 0.5 * dt * f / m
        pos = np.mod(pos + dt * vel, L)
        pos = np.where(pos >= L, 0.0, pos)
        f = bond_forces(pos, chain_len, L)
        vel += 0.5 * dt * f / m
    return pos, vel
