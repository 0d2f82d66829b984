"""Philox4x64-10 counter-based generator and the probe distributions.

Test infrastructure (see the package docstring).

The paper fixes only the distributions of the probe components (Sec. 3,
eqs. iid_components1 and iid_components2: Rademacher +-1 and Z4 {+-1, +-i},
both with E[x_i] = 0 and E[conj(x_i) x_j] = delta_ij, eq. P_assumptions).  It
names no generator.  Reading taken: Philox4x64-10 of Salmon, Moraes, Dror and
Shaw ("Parallel random numbers: as easy as 1, 2, 3", SC'11), so that sample k
on level l is a pure function of (seed, l, k) and both the CPU and the GPU can
produce the same bits independently.

Counter / key layout (shared convention; each side implements it on its own):
    key     = (seed, problem)
    counter = (block, sample k, level l, stream)
Rademacher entry i of a probe: bit (i mod 64) of word ((i >> 6) mod 4) of block
i >> 8; a 0 bit gives +1, a 1 bit gives -1.
Z4 entry i: the 2-bit field at bit 2(i mod 32) of word ((i >> 5) mod 4) of
block i >> 7; values 0, 1, 2, 3 give 1, i, -1, -i.
Streams: 0 level-difference probes, 1 pilot Hutchinson probes, 2 near-null
test-vector starts, 3 plain Hutchinson probes, 5 training-crop positions.
"""
import numpy as np

MASK64 = (1 << 64) - 1
# Philox4x64 round multipliers and Weyl key increments (Salmon et al. 2011).
M0 = 0xD2E7470EE14C6C93
M1 = 0xCA5A826395121157
W0 = 0x9E3779B97F4A7C15
W1 = 0xBB67AE8584CAA73B

STREAM_PROBE = 0
STREAM_PILOT = 1
STREAM_TESTVEC = 2
STREAM_HUTCH = 3
STREAM_CROPS = 5


def philox4x64_scalar(ctr, key, rounds=10):
    """One Philox4x64 block with Python integers: 4 counter words, 2 key words."""
    c0, c1, c2, c3 = (int(v) & MASK64 for v in ctr)
    k0, k1 = (int(v) & MASK64 for v in key)
    for _ in range(rounds):
        p0 = M0 * c0
        p1 = M1 * c2
        hi0, lo0 = p0 >> 64, p0 & MASK64
        hi1, lo1 = p1 >> 64, p1 & MASK64
        c0, c1, c2, c3 = hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0
        k0 = (k0 + W0) & MASK64
        k1 = (k1 + W1) & MASK64
    return [c0, c1, c2, c3]


def _mulhilo64(a, b):
    """Full 64x64 -> 128-bit product of uint64 arrays, as (hi, lo)."""
    m32 = np.uint64(0xFFFFFFFF)
    s32 = np.uint64(32)
    a0, a1 = a & m32, a >> s32
    b0, b1 = b & m32, b >> s32
    p00 = a0 * b0
    p01 = a0 * b1
    p10 = a1 * b0
    p11 = a1 * b1
    mid = (p00 >> s32) + (p01 & m32) + (p10 & m32)
    hi = p11 + (p01 >> s32) + (p10 >> s32) + (mid >> s32)
    lo = a * b
    return hi, lo


def philox4x64(c0, c1, c2, c3, k0, k1, rounds=10):
    """Vectorised Philox4x64 over broadcastable uint64 arrays; returns 4 words."""
    with np.errstate(over="ignore"):
        c0, c1, c2, c3 = (np.asarray(v, dtype=np.uint64) for v in (c0, c1, c2, c3))
        c0, c1, c2, c3 = np.broadcast_arrays(c0, c1, c2, c3)
        c0, c1, c2, c3 = (v.copy() for v in (c0, c1, c2, c3))
        k0 = np.uint64(int(k0) & MASK64)
        k1 = np.uint64(int(k1) & MASK64)
        m0, m1 = np.uint64(M0), np.uint64(M1)
        w0, w1 = np.uint64(W0), np.uint64(W1)
        for _ in range(rounds):
            hi0, lo0 = _mulhilo64(m0, c0)
            hi1, lo1 = _mulhilo64(m1, c2)
            c0, c1, c2, c3 = hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0
            k0 = k0 + w0
            k1 = k1 + w1
    return c0, c1, c2, c3


def _words(nblocks, seed, sample, level, stream, problem):
    blocks = np.arange(nblocks, dtype=np.uint64)
    w = philox4x64(blocks, np.uint64(sample), np.uint64(level), np.uint64(stream),
                   seed, problem)
    return np.stack(w, axis=1)  # [nblocks, 4]


def rademacher(n, seed, sample, level, stream=STREAM_PROBE, problem=0):
    """Probe x in {+1,-1}^n, distribution iid_components1 (Sec. 3)."""
    nblocks = (n + 255) // 256
    words = _words(nblocks, seed, sample, level, stream, problem).reshape(-1)
    i = np.arange(n, dtype=np.int64)
    w = words[i >> 6]
    bits = (w >> (i & 63).astype(np.uint64)) & np.uint64(1)
    return 1.0 - 2.0 * bits.astype(np.float64)


def z4(n, seed, sample, level, stream=STREAM_PROBE, problem=0):
    """Probe x in {1, i, -1, -i}^n, distribution iid_components2 (Sec. 3)."""
    nblocks = (n + 127) // 128
    words = _words(nblocks, seed, sample, level, stream, problem).reshape(-1)
    i = np.arange(n, dtype=np.int64)
    w = words[i >> 5]
    f = ((w >> (2 * (i & 31)).astype(np.uint64)) & np.uint64(3)).astype(np.int64)
    table = np.array([1.0 + 0.0j, 1.0j, -1.0 + 0.0j, -1.0j])
    return table[f]


def probe(n, seed, sample, level, complex_probe, stream=STREAM_PROBE, problem=0):
    """Rademacher for real operators, Z4 for complex ones."""
    if complex_probe:
        return z4(n, seed, sample, level, stream, problem)
    return rademacher(n, seed, sample, level, stream, problem)
