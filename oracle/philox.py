"""Philox4x32-10 counter-based generator and the samplers built on it.

The paper says only that null-collision Monte Carlo is used (Sec. 2.5); it fixes no
generator.  The oracle and the GPU path each implement Philox4x32-10 as published by
Salmon, Moraes, Dror and Shaw ("Parallel random numbers: as easy as 1, 2, 3", SC'11):
ten rounds of two 32x32->64 multiplications with the round multipliers below, the
key bumped by the two Weyl constants between rounds.

Counter layout (a reading; the paper is silent): (particle id, 0, step, tag) with
tag = (species << 8) | stream; key = (seed mod 2^32, seed >> 32).
"""
import numpy as np

_MASK = np.uint64(0xFFFFFFFF)
_M0 = np.uint64(0xD2511F53)
_M1 = np.uint64(0xCD9E8D57)
_W0 = np.uint64(0x9E3779B9)
_W1 = np.uint64(0xBB67AE85)

# streams of one (id, step, species) counter family
STREAM_COLLISION = 0    # candidate test and process selection
STREAM_TARGET = 1       # velocity of the gas atom hit by an ion
STREAM_SCATTER = 2      # two isotropic directions
STREAM_NEWION = 3       # velocity of the ion created by ionisation
STREAM_LOAD = 0xFF      # initial load


def philox4x32_10(c0, c1, c2, c3, k0, k1):
    """Return the four 32-bit output words (as uint64 arrays) for counters (c0..c3), key (k0, k1)."""
    c0 = np.asarray(c0, dtype=np.uint64) & _MASK
    c1 = np.asarray(c1, dtype=np.uint64) & _MASK
    c2 = np.asarray(c2, dtype=np.uint64) & _MASK
    c3 = np.asarray(c3, dtype=np.uint64) & _MASK
    c0, c1, c2, c3 = np.broadcast_arrays(c0, c1, c2, c3)
    k0 = np.uint64(int(k0) & 0xFFFFFFFF)
    k1 = np.uint64(int(k1) & 0xFFFFFFFF)
    for _ in range(10):
        p0 = _M0 * c0            # exact: both factors < 2^32
        p1 = _M1 * c2
        hi0, lo0 = p0 >> np.uint64(32), p0 & _MASK
        hi1, lo1 = p1 >> np.uint64(32), p1 & _MASK
        c0, c1, c2, c3 = (hi1 ^ c1 ^ k0), lo1, (hi0 ^ c3 ^ k1), lo0
        k0 = (k0 + _W0) & _MASK
        k1 = (k1 + _W1) & _MASK
    return c0, c1, c2, c3


def key_of(seed):
    seed = int(seed)
    return seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF


def draw(ids, step, species, stream, seed):
    """Philox words for counters (id, 0, step, (species << 8) | stream)."""
    k0, k1 = key_of(seed)
    tag = ((int(species) & 0xFFFFFF) << 8) | (int(stream) & 0xFF)
    return philox4x32_10(ids, 0, int(step) & 0xFFFFFFFF, tag, k0, k1)


def uniform(w):
    """u = ((w >> 9) + 1/2) * 2^-23, in (0, 1); exact in both FP32 and FP64."""
    w = np.asarray(w, dtype=np.uint64)
    return ((w >> np.uint64(9)).astype(np.float64) + 0.5) * 2.0 ** -23


def normal_pair(wa, wb):
    """Box-Muller: (sqrt(-2 ln ua) cos(2 pi ub), sqrt(-2 ln ua) sin(2 pi ub))."""
    ua, ub = uniform(wa), uniform(wb)
    r = np.sqrt(-2.0 * np.log(ua))
    return r * np.cos(2.0 * np.pi * ub), r * np.sin(2.0 * np.pi * ub)


def direction(wa, wb):
    """Isotropic unit vector: cos(chi) = 1 - 2 ua, phi = 2 pi ub; the field axis is x."""
    ua, ub = uniform(wa), uniform(wb)
    c = 1.0 - 2.0 * ua
    s = np.sqrt(np.maximum(0.0, 1.0 - c * c))
    ph = 2.0 * np.pi * ub
    return np.stack([c, s * np.cos(ph), s * np.sin(ph)], axis=-1)
