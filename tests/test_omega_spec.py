"""Pins for the oracle's sketch-matrix generator (oracle/omega.py).

The generator is Philox4x64-10 + Box-Muller with its own ln/cos/sin.  It is
pinned against NumPy's independent Philox implementation, against NumPy's
libm for the elementary functions, and by distribution checks.
"""

import numpy as np
import pytest
from scipy import stats

from oracle import omega as om


@pytest.mark.parametrize("key", [(0, 0), (123, 7), (2**64 - 1, 1), (0xDEADBEEF, 3)])
def test_philox_matches_numpy_bitgenerator(key):
    # NumPy's Philox (a 4x64-10 implementation of the same SC'11 generator)
    # increments its 256-bit counter before each block, so its first block
    # is counter value 1.
    g = np.random.Philox(key=np.array(key, dtype=np.uint64), counter=0)
    ref = g.random_raw(4 * 64).reshape(64, 4)
    ctr = np.zeros((64, 4), dtype=np.uint64)
    ctr[:, 0] = np.arange(1, 65, dtype=np.uint64)
    got = om.philox4x64_10(ctr, key)
    assert np.array_equal(got, ref)


def test_philox_high_counter_words():
    # counter words 1..3 enter the rounds too: compare a counter with all
    # four words set against NumPy started one below it
    c = [2**64 - 1, 5, 0, 9]
    g = np.random.Philox(key=np.array([1, 2], dtype=np.uint64), counter=np.array(c, dtype=np.uint64))
    ref = g.random_raw(4)
    ctr = np.array([[0, 6, 0, 9]], dtype=np.uint64)   # c + 1 with carry
    assert np.array_equal(om.philox4x64_10(ctr, (1, 2))[0], ref)


def test_ln_against_libm():
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.random(200000), 2.0 ** -np.arange(0, 54, dtype=float),
                        [1.0, 0.5, 2.0 ** -53, 1 - 2.0 ** -53, 0.7071067811865476]])
    x = x[x > 0]
    got, ref = om.ln(x), np.log(x)
    err = np.abs(got - ref)
    assert np.all(err <= 2.5e-16 * np.maximum(np.abs(ref), 1.0))
    assert om.ln(np.array([1.0]))[0] == 0.0


def test_cos_sin_2pi_against_libm():
    rng = np.random.default_rng(1)
    u = np.concatenate([rng.random(200000), np.arange(64) / 64.0,
                        [1 - 2.0 ** -53, 2.0 ** -53]])
    c, s = om.cos_sin_2pi(u)
    assert np.max(np.abs(c - np.cos(2 * np.pi * u))) < 2e-15
    assert np.max(np.abs(s - np.sin(2 * np.pi * u))) < 2e-15
    # quarter turns are exact
    c4, s4 = om.cos_sin_2pi(np.array([0.0, 0.25, 0.5, 0.75]))
    assert np.array_equal(np.abs(c4), [1, 0, 1, 0]) and np.array_equal(np.abs(s4), [0, 1, 0, 1])


def test_box_muller_pairs():
    # z0^2 + z1^2 = -2 ln u1 and atan2(z1, z0) = 2 pi u2 for each pair
    seed, nctr = 99, 1000
    ctr = np.zeros((nctr, 4), dtype=np.uint64)
    ctr[:, 0] = np.arange(nctr, dtype=np.uint64)
    w = om.philox4x64_10(ctr, (seed, om.STREAM_OMEGA))
    z = om.gaussians(seed, om.STREAM_OMEGA, 4 * nctr).reshape(nctr, 4)
    u1 = ((w[:, 0] >> np.uint64(11)) + np.uint64(1)).astype(float) * 2.0 ** -53
    u2 = (w[:, 1] >> np.uint64(11)).astype(float) * 2.0 ** -53
    assert np.allclose(z[:, 0] ** 2 + z[:, 1] ** 2, -2 * np.log(u1), rtol=1e-13, atol=1e-14)
    ang = np.mod(np.arctan2(z[:, 1], z[:, 0]), 2 * np.pi)
    d = np.abs(ang - 2 * np.pi * u2)
    d = np.minimum(d, 2 * np.pi - d)
    assert np.max(d) < 1e-10


def test_gaussian_distribution():
    z = om.gaussians(7, om.STREAM_OMEGA, 1_000_000)
    assert abs(z.mean()) < 5e-3
    assert abs(z.var() - 1.0) < 5e-3
    assert stats.kstest(z, "norm").pvalue > 1e-3
    # independent streams and seeds differ
    assert not np.array_equal(z[:100], om.gaussians(8, om.STREAM_OMEGA, 100))
    assert not np.array_equal(z[:100], om.gaussians(7, 2, 100))


def test_omega_layout():
    l, n = 5, 13
    O = om.omega(42, l, n)
    flat = om.gaussians(42, om.STREAM_OMEGA, l * n)
    assert O.shape == (l, n)
    assert np.array_equal(O.reshape(-1), flat)
    assert om.omega(42, 0, 7).shape == (0, 7)
