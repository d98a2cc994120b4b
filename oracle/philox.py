"""Philox4x32-10 counter-based generator and the random draws of one move.

Philox4x32-10 is the generator of Salmon, Moraes, Dror and Shaw (SC'11,
"Parallel random numbers: as easy as 1, 2, 3"): ten rounds of two 32x32->64
multiplies, xor with the key, and a Weyl-sequence key schedule.  It is
written here from that definition.

The paper does not state its Markov-chain move (Appendix A says only that
configurations are drawn by MCMC).  Reading used throughout: single-electron
moves, proposal r' = r + sigma z with z ~ N(0, I_3), accept iff u < q.

Counter layout of one draw (same on the GPU side, implemented separately):
  key     = (seed & 0xffffffff, seed >> 32)
  counter = (walker id, sweep index, electron | purpose << 16, 0)
  purpose 0 -> three normals by Box-Muller from the four words
  purpose 1 -> one uniform in [0, 1) from 53 bits of the first two words
"""
import numpy as np

MASK = np.uint64(0xFFFFFFFF)
M0 = np.uint64(0xD2511F53)
M1 = np.uint64(0xCD9E8D57)
W0 = np.uint64(0x9E3779B9)
W1 = np.uint64(0xBB67AE85)

PURPOSE_NORMAL = 0
PURPOSE_UNIFORM = 1


def philox4x32_10(c0, c1, c2, c3, k0, k1):
    """Apply ten Philox rounds; inputs are integer arrays (values < 2**32)."""
    c0, c1, c2, c3 = (np.asarray(x, dtype=np.uint64) & MASK for x in (c0, c1, c2, c3))
    k0 = np.asarray(k0, dtype=np.uint64) & MASK
    k1 = np.asarray(k1, dtype=np.uint64) & MASK
    for _ in range(10):
        p0 = c0 * M0
        p1 = c2 * M1
        hi0, lo0 = p0 >> np.uint64(32), p0 & MASK
        hi1, lo1 = p1 >> np.uint64(32), p1 & MASK
        c0, c1, c2, c3 = hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0
        k0 = (k0 + W0) & MASK
        k1 = (k1 + W1) & MASK
    return c0, c1, c2, c3


def _words(seed, walker_ids, sweep, electron, purpose):
    seed = int(seed)
    k0 = seed & 0xFFFFFFFF
    k1 = (seed >> 32) & 0xFFFFFFFF
    w = np.asarray(walker_ids, dtype=np.uint64)
    c1 = np.full_like(w, int(sweep) & 0xFFFFFFFF)
    c2 = np.full_like(w, (int(electron) & 0xFFFF) | (int(purpose) << 16))
    c3 = np.zeros_like(w)
    return philox4x32_10(w, c1, c2, c3, k0, k1)


def box_muller(w_a, w_b):
    """Two normals from two 32-bit words: u1 in (0,1], u2 in [0,1)."""
    u1 = (w_a.astype(np.float64) + 1.0) * 2.0 ** -32
    u2 = w_b.astype(np.float64) * 2.0 ** -32
    rad = np.sqrt(-2.0 * np.log(u1))
    ang = 2.0 * np.pi * u2
    return rad * np.cos(ang), rad * np.sin(ang)


def move_normals(seed, walker_ids, sweep, electron):
    """z[W][3] for the proposal of `electron` in `sweep`."""
    x0, x1, x2, x3 = _words(seed, walker_ids, sweep, electron, PURPOSE_NORMAL)
    z0, z1 = box_muller(x0, x1)
    z2, _ = box_muller(x2, x3)
    return np.stack([z0, z1, z2], axis=-1)


def move_uniform(seed, walker_ids, sweep, electron):
    """u[W] in [0, 1) with 53 random bits for the accept test."""
    x0, x1, _, _ = _words(seed, walker_ids, sweep, electron, PURPOSE_UNIFORM)
    bits = (x0 << np.uint64(21)) | (x1 >> np.uint64(11))
    return bits.astype(np.float64) * 2.0 ** -53
