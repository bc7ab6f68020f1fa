"""Philox4x64-10 counter-based random numbers (oracle side).

Written from the published definition of the Philox family (Salmon, Moraes,
Dror & Shaw, "Parallel random numbers: as easy as 1, 2, 3", SC'11): a
four-word counter is mixed with a two-word key through ten rounds of
64x64->128-bit multiplications; the key is advanced by Weyl constants between
rounds.  Pinned against ``numpy.random.Philox`` (the same published generator)
in ``tests/test_oracle_philox.py``.

The random draws of the method (mode amplitudes and phases, particle
positions, momenta) are defined as functions of (seed, stream, index) so that
any subset of particles or modes can be regenerated independently.
"""
import numpy as np

_M0 = np.uint64(0xD2E7470EE14C6C93)
_M1 = np.uint64(0xCA5A826395121157)
_W0 = np.uint64(0x9E3779B97F4A7C15)
_W1 = np.uint64(0xBB67AE8584CAA73B)
_MASK32 = np.uint64(0xFFFFFFFF)
_S32 = np.uint64(32)

# Stream tags: the second key word separates independent uses of one seed.
STREAM_FIELD = 0x46       # delta_0(k) amplitude and phase, counter = mode index
STREAM_POSITION = 0x50    # particle positions, counter = particle id
STREAM_MOMENTUM = 0x51    # |q| rejection sampling, counter = (id, trial)
STREAM_DIRECTION = 0x44   # isotropic direction, counter = particle id


def _mulhilo(a, b):
    """Full 128-bit product of uint64 arrays, returned as (hi, lo)."""
    a = np.asarray(a, dtype=np.uint64)
    b = np.asarray(b, dtype=np.uint64)
    a_lo, a_hi = a & _MASK32, a >> _S32
    b_lo, b_hi = b & _MASK32, b >> _S32
    ll = a_lo * b_lo
    lh = a_lo * b_hi
    hl = a_hi * b_lo
    hh = a_hi * b_hi
    mid = (ll >> _S32) + (lh & _MASK32) + (hl & _MASK32)
    hi = hh + (lh >> _S32) + (hl >> _S32) + (mid >> _S32)
    lo = a * b  # uint64 multiplication wraps modulo 2^64
    return hi, lo


def philox4x64(ctr, key):
    """Philox4x64 with 10 rounds.

    ctr : (..., 4) uint64 counters; key : (..., 2) uint64 keys (broadcast).
    Returns (..., 4) uint64.
    """
    with np.errstate(over="ignore"):
        ctr = np.asarray(ctr, dtype=np.uint64)
        key = np.asarray(key, dtype=np.uint64)
        shape = np.broadcast_shapes(ctr.shape[:-1], key.shape[:-1])
        x0 = np.broadcast_to(ctr[..., 0], shape).copy()
        x1 = np.broadcast_to(ctr[..., 1], shape).copy()
        x2 = np.broadcast_to(ctr[..., 2], shape).copy()
        x3 = np.broadcast_to(ctr[..., 3], shape).copy()
        k0 = np.broadcast_to(key[..., 0], shape).copy()
        k1 = np.broadcast_to(key[..., 1], shape).copy()
        for rnd in range(10):
            if rnd > 0:
                k0 = k0 + _W0
                k1 = k1 + _W1
            hi0, lo0 = _mulhilo(_M0, x0)
            hi1, lo1 = _mulhilo(_M1, x2)
            x0, x1, x2, x3 = hi1 ^ x1 ^ k0, lo1, hi0 ^ x3 ^ k1, lo0
        return np.stack([x0, x1, x2, x3], axis=-1)


def draw(seed, stream, index, trial=0):
    """Four uint64 words for (seed, stream, index, trial).

    Counter = (index, trial, 0, 0), key = (seed, stream).
    """
    index = np.asarray(index, dtype=np.uint64)
    ctr = np.zeros(index.shape + (4,), dtype=np.uint64)
    ctr[..., 0] = index
    ctr[..., 1] = np.uint64(trial)
    key = np.array([np.uint64(seed), np.uint64(stream)], dtype=np.uint64)
    return philox4x64(ctr, key)


def to_unit_open(words):
    """Map uint64 words to doubles in (0, 1): (floor(w / 2^12) + 1/2) * 2^-52.

    The value (2j+1) 2^-53 with j < 2^52 is exact in binary64.
    """
    j = (np.asarray(words, dtype=np.uint64) >> np.uint64(12)).astype(np.float64)
    return (j + 0.5) * 2.0 ** -52
