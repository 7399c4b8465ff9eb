"""Oracle: counter-based Gaussian noise n ~ N(0, I) (test infrastructure).

The paper draws the stochastic driving term as eta = Q n with n a vector of independent
standard normals every iteration (eqs. J_QQ and def_Q_GS).  To make the GPU path and this
oracle consume the same n, both sides implement the same published counter-based
generator independently: Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random
numbers: as easy as 1, 2, 3", SC'11).  One Philox call maps a 128-bit counter and a 64-bit
key to four 32-bit words through ten rounds; each round multiplies words 0 and 2 by the
two Philox constants, splits each 64-bit product into high and low halves, and forms
(hi1 ^ w1 ^ k0, lo1, hi0 ^ w3 ^ k1, lo0); the key is advanced by the two Weyl constants
between rounds.

Counter layout (shared convention of this project):
  key  = (seed mod 2^32, seed >> 32)
  ctr0 = call index (a site pair: sites 2q and 2q+1 use call q)
  ctr1 = level | slot << 4 | colour << 12 | comp << 16 | kind << 24
  ctr2 = cycle mod 2^32, ctr3 = cycle >> 32
Words (w0, w1) and (w2, w3) give two uniforms u = (((w_a 2^32 + w_b) >> 11) + 1/2) 2^-53
in (0, 1] (the
half-ulp offset rounds away for the largest words); Box-Muller turns them into z0 = sqrt(-2 ln u1) cos(2 pi u2) (even site) and
z1 = sqrt(-2 ln u1) sin(2 pi u2) (odd site).
"""
import numpy as np

MASK32 = np.uint64(0xFFFFFFFF)
PHILOX_M0 = np.uint64(0xD2511F53)
PHILOX_M1 = np.uint64(0xCD9E8D57)
PHILOX_W0 = 0x9E3779B9
PHILOX_W1 = 0xBB67AE85

KIND_SMOOTH = 0
KIND_COARSEST = 1


def philox4x32_10(c0, c1, c2, c3, k0, k1):
    """Vectorised Philox4x32-10.  Counters are arrays (or scalars) of values < 2^32."""
    c0 = np.asarray(c0, dtype=np.uint64) & MASK32
    c1 = np.asarray(c1, dtype=np.uint64) & MASK32
    c2 = np.asarray(c2, dtype=np.uint64) & MASK32
    c3 = np.asarray(c3, dtype=np.uint64) & MASK32
    k0 = int(k0) & 0xFFFFFFFF
    k1 = int(k1) & 0xFFFFFFFF
    for r in range(10):
        p0 = PHILOX_M0 * c0
        p1 = PHILOX_M1 * c2
        hi0, lo0 = p0 >> np.uint64(32), p0 & MASK32
        hi1, lo1 = p1 >> np.uint64(32), p1 & MASK32
        c0, c1, c2, c3 = (hi1 ^ c1 ^ np.uint64(k0), lo1, hi0 ^ c3 ^ np.uint64(k1), lo0)
        k0 = (k0 + PHILOX_W0) & 0xFFFFFFFF
        k1 = (k1 + PHILOX_W1) & 0xFFFFFFFF
    return c0, c1, c2, c3


def stream_id(level, slot, colour, comp, kind):
    assert 0 <= level < 16 and 0 <= slot < 256 and 0 <= colour < 16
    assert 0 <= comp < 256 and 0 <= kind < 256
    return level | (slot << 4) | (colour << 12) | (comp << 16) | (kind << 24)


def uniforms_from_words(wa, wb):
    v = ((wa << np.uint64(32)) | wb) >> np.uint64(11)
    return (v.astype(np.float64) + 0.5) * 2.0 ** -53


def box_muller(u1, u2):
    r = np.sqrt(-2.0 * np.log(u1))
    return r * np.cos(2.0 * np.pi * u2), r * np.sin(2.0 * np.pi * u2)


def normals(seed, cycle, level, slot, colour, comp, kind, sites):
    """Standard normals for the given site indices of one noise stream."""
    sites = np.asarray(sites, dtype=np.int64)
    calls = (sites >> 1).astype(np.uint64)
    sid = stream_id(level, slot, colour, comp, kind)
    w0, w1, w2, w3 = philox4x32_10(calls, sid, cycle & 0xFFFFFFFF, cycle >> 32,
                                   seed & 0xFFFFFFFF, seed >> 32)
    z0, z1 = box_muller(uniforms_from_words(w0, w1), uniforms_from_words(w2, w3))
    return np.where(sites & 1, z1, z0)


class PhiloxNoise:
    """Noise source used by the oracle's cycles: draws from the counter-based stream."""

    def __init__(self, seed):
        self.seed = int(seed)

    def draw(self, cycle, level, slot, colour, comp, kind, sites):
        return normals(self.seed, int(cycle), level, slot, colour, comp, kind, sites)
