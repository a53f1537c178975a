"""Philox4x32-10 and Z4 probe vectors (oracle; test infrastructure only).

The paper draws Hutchinson probe entries i.i.d. from Z4 = {1, -1, i, -i} with
equal probability (Sec. 1, eq. z4).  It does not name a generator; this
project uses the counter-based Philox4x32-10 of Salmon, Moraes, Dror and Shaw,
"Parallel random numbers: as easy as 1, 2, 3" (SC'11), so that any entry of any
probe can be drawn independently and reproduced bit for bit on both sides.

Convention (shared with the GPU library, written independently there):
  key     = (seed & 0xffffffff, seed >> 32)
  counter = (i & 0xffffffff, i >> 32, probe, stream)
  x_i     = (1, i, -1, -i)[word0 >> 30]
where i is the dof index within the level vector and
stream = 256 * level + kind, kind in {0 plain, 1 O_l, 2 F_l, 3 M_l,
4 coarsest, 5 correlator source, 6 loop source, 7 test vector, 8 network
training input, 9 deflation basis start, 10 deflated-estimator probe}.

Parity status: pinned by the generator's published known-answer vectors
(tests/golden/philox4x32_10_kat.txt) and by frequency tests of the Z4 map.
"""
from __future__ import annotations

import numpy as np

M0 = np.uint64(0xD2511F53)
M1 = np.uint64(0xCD9E8D57)
W0 = np.uint32(0x9E3779B9)
W1 = np.uint32(0xBB67AE85)
MASK32 = np.uint64(0xFFFFFFFF)

KIND_PLAIN, KIND_O, KIND_F, KIND_M, KIND_COARSEST = 0, 1, 2, 3, 4
KIND_CORR, KIND_LOOP, KIND_TV = 5, 6, 7


def stream_id(level: int, kind: int) -> int:
    return 256 * int(level) + int(kind)


def philox4x32_10(ctr, key):
    """Ten Philox4x32 rounds.

    ctr: tuple of 4 uint32 arrays (broadcastable), key: tuple of 2 uint32.
    Returns a tuple of 4 uint32 arrays.
    """
    c0, c1, c2, c3 = (np.asarray(c, dtype=np.uint32) for c in ctr)
    k0 = np.uint32(key[0])
    k1 = np.uint32(key[1])
    with np.errstate(over="ignore"):
        for r in range(10):
            if r > 0:
                k0 = np.uint32(k0 + W0)
                k1 = np.uint32(k1 + W1)
            p0 = M0 * c0.astype(np.uint64)
            p1 = M1 * c2.astype(np.uint64)
            hi0 = (p0 >> np.uint64(32)).astype(np.uint32)
            lo0 = (p0 & MASK32).astype(np.uint32)
            hi1 = (p1 >> np.uint64(32)).astype(np.uint32)
            lo1 = (p1 & MASK32).astype(np.uint32)
            c0, c1, c2, c3 = hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0
    return c0, c1, c2, c3


_Z4 = np.array([1.0, 1.0j, -1.0, -1.0j], dtype=np.complex128)


def z4_codes_at(idx, seed: int, stream: int, probe: int) -> np.ndarray:
    """The 2-bit Z4 codes (0:1, 1:i, 2:-1, 3:-i) of entries idx (uint64)."""
    i = np.asarray(idx, dtype=np.uint64)
    ctr = ((i & MASK32).astype(np.uint32), (i >> np.uint64(32)).astype(np.uint32),
           np.uint32(probe), np.uint32(stream))
    key = (int(seed) & 0xFFFFFFFF, (int(seed) >> 32) & 0xFFFFFFFF)
    return (philox4x32_10(ctr, key)[0] >> np.uint32(30)).astype(np.uint8)


def z4_codes(n: int, seed: int, stream: int, probe: int) -> np.ndarray:
    return z4_codes_at(np.arange(n, dtype=np.uint64), seed, stream, probe)


def z4_vector(n: int, seed: int, stream: int, probe: int) -> np.ndarray:
    """Probe vector x in Z4^n for (seed, stream, probe); entries i = 0..n-1."""
    return _Z4[z4_codes(n, seed, stream, probe).astype(np.int64)]
