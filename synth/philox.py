"""Counter-based uniform random numbers (Philox4x32-10).

The method draws its random pivots and accept/reject thresholds from a
uniform distribution on [0, 1) (Algorithm 2: iid proposals from the
residual-diagonal distribution; Algorithm 3: z uniform in [0, 1)).  Both
implementations receive the same stream of doubles as an input array, so the
stream itself is generated here, once.

Generator: Philox4x32 with 10 rounds, as published by Salmon, Moraes, Dror and
Shaw, "Parallel random numbers: as easy as 1, 2, 3" (SC'11).  The 128-bit
counter of draw i is (i mod 2^32, i div 2^32, 0, 0) and the 64-bit key is the
seed.  Draw i is the double  ((w0 >> 5) * 2^26 + (w1 >> 6)) * 2^-53, i.e. 53
random bits from the first two output words, which lies in [0, 1).
"""
import numpy as np

_M0 = np.uint64(0xD2511F53)
_M1 = np.uint64(0xCD9E8D57)
_W0 = np.uint32(0x9E3779B9)
_W1 = np.uint32(0xBB67AE85)
_MASK32 = np.uint64(0xFFFFFFFF)


def _mulhilo(a, m):
    p = a.astype(np.uint64) * m
    return (p >> np.uint64(32)).astype(np.uint32), (p & _MASK32).astype(np.uint32)


def philox4x32_10(ctr, key):
    """Philox4x32-10 block function.

    ctr: uint32 array of shape (n, 4); key: uint32 array of shape (2,) or (n, 2).
    Returns the uint32 array of shape (n, 4).
    """
    c = np.array(ctr, dtype=np.uint32).reshape(-1, 4)
    k = np.broadcast_to(np.array(key, dtype=np.uint32).reshape(-1, 2), (c.shape[0], 2))
    c0, c1, c2, c3 = (c[:, i].copy() for i in range(4))
    k0, k1 = k[:, 0].copy(), k[:, 1].copy()
    with np.errstate(over="ignore"):
        for rnd in range(10):
            if rnd > 0:
                k0 = k0 + _W0
                k1 = k1 + _W1
            hi0, lo0 = _mulhilo(c0, _M0)
            hi1, lo1 = _mulhilo(c2, _M1)
            c0, c1, c2, c3 = hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0
    return np.stack([c0, c1, c2, c3], axis=1)


def uniform_stream(n, seed, offset=0):
    """n doubles in [0, 1) from draws offset .. offset+n-1 of the stream `seed`."""
    idx = np.arange(offset, offset + n, dtype=np.uint64)
    ctr = np.zeros((n, 4), dtype=np.uint32)
    ctr[:, 0] = (idx & _MASK32).astype(np.uint32)
    ctr[:, 1] = (idx >> np.uint64(32)).astype(np.uint32)
    seed = int(seed) & 0xFFFFFFFFFFFFFFFF
    key = np.array([seed & 0xFFFFFFFF, seed >> 32], dtype=np.uint32)
    w = philox4x32_10(ctr, key)
    hi = (w[:, 0] >> np.uint32(5)).astype(np.uint64)
    lo = (w[:, 1] >> np.uint32(6)).astype(np.uint64)
    bits = (hi << np.uint64(26)) | lo
    return bits.astype(np.float64) * (2.0 ** -53)
