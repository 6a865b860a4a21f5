"""Philox4x32-10 counter-based generator and Box-Muller normals (numpy).

Definition followed: J. K. Salmon, M. A. Moraes, R. O. Dror, D. E. Shaw,
"Parallel random numbers: as easy as 1, 2, 3", SC'11 -- Philox4x32 with
multipliers 0xD2511F53 / 0xCD9E8D57, Weyl key increments 0x9E3779B9 /
0xBB67AE85 and 10 rounds.

Stream layout used by every consumer (host and device must agree):

* key   = (seed mod 2^32, stream mod 2^32)
* counter = (block mod 2^32, block >> 32, purpose, tick)
* one block yields four 32-bit words w0..w3; the 53-bit uniforms of that block
  are u_a = ((w0 >> 5) * 2^26 + (w1 >> 6)) / 2^53 and likewise u_b from
  (w2, w3); both lie in [0, 1).
* normals: Box-Muller on one block, r = sqrt(-2 ln(1 - u_a)),
  phi = 2 pi u_b, giving normal[2*block] = r cos phi and
  normal[2*block + 1] = r sin phi.
"""
import numpy as np

_M0 = np.uint64(0xD2511F53)
_M1 = np.uint64(0xCD9E8D57)
_W0 = np.uint64(0x9E3779B9)
_W1 = np.uint64(0xBB67AE85)
_MASK = np.uint64(0xFFFFFFFF)
_S32 = np.uint64(32)


def philox4x32_10(c0, c1, c2, c3, k0, k1):
    """Philox4x32 with 10 rounds on broadcastable uint32-valued arrays.

    Returns four uint64 arrays holding the 32-bit output words."""
    c0, c1, c2, c3 = (np.asarray(c, dtype=np.uint64) & _MASK for c in (c0, c1, c2, c3))
    k0 = np.asarray(k0, dtype=np.uint64) & _MASK
    k1 = np.asarray(k1, dtype=np.uint64) & _MASK
    c0, c1, c2, c3 = np.broadcast_arrays(c0, c1, c2, c3)
    for r in range(10):
        if r > 0:
            k0 = (k0 + _W0) & _MASK
            k1 = (k1 + _W1) & _MASK
        p0 = _M0 * c0
        p1 = _M1 * c2
        hi0, lo0 = p0 >> _S32, p0 & _MASK
        hi1, lo1 = p1 >> _S32, p1 & _MASK
        c0, c1, c2, c3 = (hi1 ^ c1 ^ k0), lo1, (hi0 ^ c3 ^ k1), lo0
    return c0, c1, c2, c3


def _blocks(seed, stream, purpose, ticks, nblocks):
    ticks = np.asarray(ticks, dtype=np.uint64).reshape(-1, 1)
    b = np.arange(nblocks, dtype=np.uint64).reshape(1, -1)
    return philox4x32_10(b & _MASK, b >> _S32, np.uint64(purpose), ticks,
                         np.uint64(seed), np.uint64(stream))


def _u53(hi_word, lo_word):
    a = (hi_word >> np.uint64(5)).astype(np.float64)
    b = (lo_word >> np.uint64(6)).astype(np.float64)
    return (a * 67108864.0 + b) * (1.0 / 9007199254740992.0)


def uniforms(seed, stream, purpose, ticks, count):
    """Uniforms in [0,1): array of shape (len(ticks), count)."""
    nb = (count + 1) // 2
    w0, w1, w2, w3 = _blocks(seed, stream, purpose, ticks, nb)
    out = np.empty((w0.shape[0], 2 * nb))
    out[:, 0::2] = _u53(w0, w1)
    out[:, 1::2] = _u53(w2, w3)
    return out[:, :count]


def normals(seed, stream, purpose, ticks, count):
    """Standard normals: array of shape (len(ticks), count)."""
    nb = (count + 1) // 2
    w0, w1, w2, w3 = _blocks(seed, stream, purpose, ticks, nb)
    ua = _u53(w0, w1)
    ub = _u53(w2, w3)
    r = np.sqrt(-2.0 * np.log(1.0 - ua))
    phi = 6.283185307179586 * ub
    out = np.empty((w0.shape[0], 2 * nb))
    out[:, 0::2] = r * np.cos(phi)
    out[:, 1::2] = r * np.sin(phi)
    return out[:, :count]
