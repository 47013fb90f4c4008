"""Philox4x32-10 and the mapping from 32-bit words to uniforms.

The paper draws its per-cell random numbers from a counter-based hash
generator keyed on (global cell index, timestep, user seed) so that any cell's
numbers can be reproduced on any rank without communication (sec. 3.6, refs.
Phillips et al. 2011 and Salmon et al. 2011). It names Saru; this oracle uses
Philox4x32-10 from Salmon et al., "Parallel random numbers: as easy as 1, 2,
3" (SC'11), which the paper cites for the same idea.

Philox4x32-10: a 128-bit counter (c0, c1, c2, c3) and a 64-bit key (k0, k1).
One round multiplies c0 and c2 by two odd 32-bit constants, forms the 64-bit
products' high and low halves, and permutes/xors them with c1, c3 and the
round key; the key is bumped by two Weyl constants between rounds. Ten rounds.

Uniform mapping (a reading; the paper does not say how words become reals):
u = (w + 1/2) * 2**-32, which is exact in FP64 and lies in the open interval
(0, 1), so log(u) and log(1 - u) are always finite.
"""
import numpy as np

PHILOX_M0 = 0xD2511F53
PHILOX_M1 = 0xCD9E8D57
PHILOX_W0 = 0x9E3779B9
PHILOX_W1 = 0xBB67AE85
_MASK32 = np.uint64(0xFFFFFFFF)

# Counter word c2 carries the purpose of a draw, so the streams never overlap.
TAG_AXIS = 0
TAG_THERMO = 1
TAG_SHIFT = 2
TAG_AT = 3      # per-particle random velocities of the Andersen-thermostat rule


def philox4x32_10(ctr, key):
    """Vectorised Philox4x32-10.

    ctr: array (..., 4) of uint32-valued integers; key: array (..., 2) or a
    pair broadcastable against ctr[..., :2]. Returns (..., 4) uint32.
    """
    ctr = np.asarray(ctr, dtype=np.uint64)
    key = np.asarray(key, dtype=np.uint64)
    c0, c1, c2, c3 = (ctr[..., j] & _MASK32 for j in range(4))
    k0 = key[..., 0] & _MASK32
    k1 = key[..., 1] & _MASK32
    m0 = np.uint64(PHILOX_M0)
    m1 = np.uint64(PHILOX_M1)
    sh = np.uint64(32)
    for r in range(10):
        p0 = m0 * c0          # < 2**64: exact in uint64
        p1 = m1 * c2
        n0 = (p1 >> sh) ^ c1 ^ k0
        n1 = p1 & _MASK32
        n2 = (p0 >> sh) ^ c3 ^ k1
        n3 = p0 & _MASK32
        c0, c1, c2, c3 = n0, n1, n2, n3
        if r < 9:
            k0 = (k0 + np.uint64(PHILOX_W0)) & _MASK32
            k1 = (k1 + np.uint64(PHILOX_W1)) & _MASK32
    return np.stack([c0, c1, c2, c3], axis=-1).astype(np.uint32)


def philox_scalar(ctr, key):
    """Same generator on Python ints, one block at a time (used by the
    brute-force tier so that it does not depend on numpy's uint64 rules)."""
    c0, c1, c2, c3 = (int(x) & 0xFFFFFFFF for x in ctr)
    k0, k1 = (int(x) & 0xFFFFFFFF for x in key)
    for r in range(10):
        p0 = PHILOX_M0 * c0
        p1 = PHILOX_M1 * c2
        c0, c1, c2, c3 = ((p1 >> 32) ^ c1 ^ k0) & 0xFFFFFFFF, p1 & 0xFFFFFFFF, \
                         ((p0 >> 32) ^ c3 ^ k1) & 0xFFFFFFFF, p0 & 0xFFFFFFFF
        if r < 9:
            k0 = (k0 + PHILOX_W0) & 0xFFFFFFFF
            k1 = (k1 + PHILOX_W1) & 0xFFFFFFFF
    return (c0, c1, c2, c3)


def seed_key(seed):
    """64-bit user seed -> Philox key (low word, high word)."""
    seed = int(seed) & 0xFFFFFFFFFFFFFFFF
    return (seed & 0xFFFFFFFF, seed >> 32)


def uniform01(words):
    """u = (w + 0.5) * 2**-32 in FP64 (exact, open interval (0, 1))."""
    return (np.asarray(words, dtype=np.float64) + 0.5) * (2.0 ** -32)


def uniform01_scalar(w):
    return (float(int(w)) + 0.5) * (2.0 ** -32)
