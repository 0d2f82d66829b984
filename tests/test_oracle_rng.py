"""Pins for the oracle's Philox4x64-10 and probe generators (Sec. 3 distributions)."""
import numpy as np

from oracle import philox


def test_scalar_philox_matches_numpy_bit_generator():
    # numpy's Philox (4x64, 10 rounds) increments its counter before each block,
    # so block c of ours is numpy's first block after counter c - 1.
    for key, ctr in [((0, 0), (1, 0, 0, 0)),
                     ((12345, 678), (7, 3, 2, 0)),
                     ((2**64 - 1, 2**63), (2**40 + 5, 2**33, 9, 1))]:
        g = np.random.Philox(key=np.array(key, dtype=np.uint64),
                             counter=np.array([(ctr[0] - 1) % 2**64] + list(ctr[1:]),
                                              dtype=np.uint64))
        ref = [int(v) for v in g.random_raw(4)]
        assert philox.philox4x64_scalar(ctr, key) == ref


def test_vectorised_philox_matches_scalar():
    rng = np.random.default_rng(0)
    c = rng.integers(0, 2**63, size=(4, 50), dtype=np.uint64)
    for k0, k1 in [(0, 0), (99, 2**62 + 3)]:
        words = philox.philox4x64(c[0], c[1], c[2], c[3], k0, k1)
        for j in range(50):
            ref = philox.philox4x64_scalar([int(c[i, j]) for i in range(4)], (k0, k1))
            assert [int(w[j]) for w in words] == ref


def test_rademacher_bit_layout_by_enumeration():
    n, seed, k, lvl = 600, 11, 4, 2
    x = philox.rademacher(n, seed, k, lvl)
    for i in range(n):
        words = philox.philox4x64_scalar((i // 256, k, lvl, philox.STREAM_PROBE), (seed, 0))
        bit = (words[(i // 64) % 4] >> (i % 64)) & 1
        assert x[i] == (1.0 if bit == 0 else -1.0)


def test_z4_bit_layout_by_enumeration():
    n, seed, k, lvl = 300, 5, 9, 1
    x = philox.z4(n, seed, k, lvl, problem=3)
    table = [1, 1j, -1, -1j]
    for i in range(n):
        words = philox.philox4x64_scalar((i // 128, k, lvl, philox.STREAM_PROBE), (seed, 3))
        f = (words[(i // 32) % 4] >> (2 * (i % 32))) & 3
        assert x[i] == table[f]


def test_probe_moments():
    # E[x_i] = 0 and E[conj(x_i) x_j] = delta_ij (eq. P_assumptions); Z4 also E[x^2] = 0.
    n = 1 << 16
    r = philox.rademacher(n, 1, 0, 1)
    assert set(np.unique(r)) == {-1.0, 1.0}
    assert abs(r.mean()) < 4.0 / np.sqrt(n)
    assert abs(np.mean(r[:-1] * r[1:])) < 4.0 / np.sqrt(n)
    z = philox.z4(n, 1, 0, 1)
    assert np.all(np.abs(z) == 1.0)
    assert abs(z.mean()) < 4.0 / np.sqrt(n)
    assert abs(np.mean(z * z)) < 4.0 / np.sqrt(n)
    assert abs(np.mean(np.conj(z[:-1]) * z[1:])) < 4.0 / np.sqrt(n)
    # different samples, levels, streams and seeds give uncorrelated probes
    for other in [philox.rademacher(n, 1, 1, 1), philox.rademacher(n, 1, 0, 2),
                  philox.rademacher(n, 1, 0, 1, stream=1), philox.rademacher(n, 2, 0, 1)]:
        assert abs(np.mean(r * other)) < 4.0 / np.sqrt(n)
