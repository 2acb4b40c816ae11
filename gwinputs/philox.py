"""Counter-based random numbers for the synthetic inputs.

Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as easy
as 1, 2, 3", SC'11) written from its published definition, vectorised in
NumPy.  One normal deviate per counter by the Box-Muller transform
(Box & Muller, Ann. Math. Stat. 29, 610 (1958)).

Every generated tensor element is a pure function of (seed, stream, index),
so any brick of the three-center tensor can be regenerated on its own, on the
host here or on the device by the HIP generator in ``csrc/gwgen.hip``, which
implements the same definition.

Conventions (shared with the device generator):
  key     = (seed, stream)                       two 32-bit words
  counter = (idx & 0xffffffff, idx >> 32, 0, 0)  idx is a 64-bit element index
  u1 = (x0 + 1) * 2**-32  in (0, 1]
  u2 =  x1      * 2**-32  in [0, 1)
  z  = sqrt(-2 ln u1) * cos(2 pi u2)
so |z| <= sqrt(64 ln 2) = Z_MAX exactly.
"""
from __future__ import annotations

import numpy as np

M0 = np.uint64(0xD2511F53)
M1 = np.uint64(0xCD9E8D57)
W0 = 0x9E3779B9
W1 = 0xBB67AE85
MASK32 = np.uint64(0xFFFFFFFF)
TWO_M32 = 2.0 ** -32
Z_MAX = float(np.sqrt(64.0 * np.log(2.0)))


def philox4x32_10(c0, c1, c2, c3, k0: int, k1: int):
    """Ten Philox rounds on uint32 counter words (arrays of equal shape).

    Returns the four output words as uint64 arrays holding 32-bit values.
    """
    c0 = np.asarray(c0, dtype=np.uint64) & MASK32
    c1 = np.asarray(c1, dtype=np.uint64) & MASK32
    c2 = np.asarray(c2, dtype=np.uint64) & MASK32
    c3 = np.asarray(c3, dtype=np.uint64) & MASK32
    k0 = int(k0) & 0xFFFFFFFF
    k1 = int(k1) & 0xFFFFFFFF
    for r in range(10):
        if r:
            k0 = (k0 + W0) & 0xFFFFFFFF
            k1 = (k1 + W1) & 0xFFFFFFFF
        p0 = M0 * c0
        p1 = M1 * c2
        hi0, lo0 = p0 >> np.uint64(32), p0 & MASK32
        hi1, lo1 = p1 >> np.uint64(32), p1 & MASK32
        c0, c1, c2, c3 = (hi1 ^ c1 ^ np.uint64(k0), lo1,
                          hi0 ^ c3 ^ np.uint64(k1), lo0)
    return c0, c1, c2, c3


def _words(idx):
    idx = np.asarray(idx, dtype=np.uint64)
    return idx & MASK32, idx >> np.uint64(32)


def normal(seed: int, stream: int, idx) -> np.ndarray:
    """Standard normal deviates, one per 64-bit counter index (float64)."""
    lo, hi = _words(idx)
    z0 = np.zeros_like(lo)
    x0, x1, _, _ = philox4x32_10(lo, hi, z0, z0, seed, stream)
    u1 = (x0.astype(np.float64) + 1.0) * TWO_M32
    u2 = x1.astype(np.float64) * TWO_M32
    return np.sqrt(-2.0 * np.log(u1)) * np.cos(2.0 * np.pi * u2)


def uniform(seed: int, stream: int, idx) -> np.ndarray:
    """Uniform deviates in [0, 1), one per 64-bit counter index."""
    lo, hi = _words(idx)
    z0 = np.zeros_like(lo)
    x0, _, _, _ = philox4x32_10(lo, hi, z0, z0, seed, stream)
    return x0.astype(np.float64) * TWO_M32
