"""Pins of the oracle's Philox4x32-10 and uniform mapping (CPU only)."""
import json
import os

import numpy as np
import pytest

from oracle.philox import (philox4x32_10, philox_scalar, seed_key, uniform01,
                           uniform01_scalar)


def _kat(golden_dir):
    with open(os.path.join(golden_dir, "philox4x32_10_kat.json")) as f:
        return json.load(f)["vectors"]


def test_known_answer_vectors_vectorised(golden_dir):
    for v in _kat(golden_dir):
        ctr = np.array([int(x, 16) for x in v["ctr"]], dtype=np.uint64)
        key = np.array([int(x, 16) for x in v["key"]], dtype=np.uint64)
        out = philox4x32_10(ctr, key)
        assert [int(x) for x in out] == [int(x, 16) for x in v["out"]]


def test_known_answer_vectors_scalar(golden_dir):
    for v in _kat(golden_dir):
        out = philox_scalar([int(x, 16) for x in v["ctr"]],
                            [int(x, 16) for x in v["key"]])
        assert list(out) == [int(x, 16) for x in v["out"]]


def test_vectorised_equals_scalar_on_random_counters():
    rng = np.random.default_rng(7)
    ctr = rng.integers(0, 2**32, size=(200, 4), dtype=np.uint64)
    key = rng.integers(0, 2**32, size=(200, 2), dtype=np.uint64)
    out = philox4x32_10(ctr, key)
    for i in range(200):
        assert tuple(int(x) for x in out[i]) == philox_scalar(ctr[i], key[i])


def test_seed_key_split():
    assert seed_key(1) == (1, 0)
    assert seed_key(0x0123456789ABCDEF) == (0x89ABCDEF, 0x01234567)


def test_uniform_mapping_endpoints_exact():
    assert uniform01_scalar(0) == 2.0 ** -33
    assert uniform01_scalar(2**32 - 1) == 1.0 - 2.0 ** -33
    u = uniform01(np.array([0, 1, 2**31, 2**32 - 1], dtype=np.uint64))
    assert np.all((u > 0.0) & (u < 1.0))
    # exact: (w + 1/2) has at most 33 significant bits
    assert u[2] == 0.5 + 2.0 ** -33


def test_output_words_uniform_chi2():
    from scipy import stats
    ctr = np.zeros((50000, 4), dtype=np.uint64)
    ctr[:, 0] = np.arange(50000)
    ctr[:, 1] = 17
    w = philox4x32_10(ctr, np.array(seed_key(1), dtype=np.uint64)).ravel()
    hist = np.bincount((w >> 24).astype(np.int64), minlength=256)
    chi2 = ((hist - w.size / 256) ** 2 / (w.size / 256)).sum()
    # 255 dof; p < 1e-4 false-alarm threshold
    assert chi2 < stats.chi2.ppf(1 - 1e-4, 255)


def test_counter_avalanche():
    """One flipped counter bit changes about half of the 128 output bits."""
    rng = np.random.default_rng(3)
    ctr = rng.integers(0, 2**32, size=(2000, 4), dtype=np.uint64)
    key = np.array([5, 9], dtype=np.uint64)
    a = philox4x32_10(ctr, key)
    ctr2 = ctr.copy()
    ctr2[:, 1] ^= np.uint64(1 << 13)
    b = philox4x32_10(ctr2, key)
    x = np.bitwise_xor(a, b).view(np.uint8)
    flips = np.unpackbits(x).reshape(2000, 128).sum(axis=1)
    assert abs(flips.mean() - 64.0) < 1.0
