"""Philox4x32-10 counter-based generator and Box-Muller Gaussians (CPU, numpy).

TEST INFRASTRUCTURE ONLY: part of the FP64 CPU oracle.  Nothing in the
product path imports this module.

Philox4x32-10 follows its published definition (Salmon, Moraes, Dror, Shaw,
"Parallel random numbers: as easy as 1, 2, 3", SC'11): ten rounds on a
128-bit counter (c0, c1, c2, c3) with a 64-bit key (k0, k1).  One round takes
the two 32x32->64-bit products M0*c0 and M1*c2 and returns
(hi(M1*c2) ^ c1 ^ k0, lo(M1*c2), hi(M0*c0) ^ c3 ^ k1, lo(M0*c0)); the key is
bumped by the Weyl constants between rounds.

Noise layout (the reading of the paper's zero-mean Gaussian noise used in
the training quantisation proxy, Section IV-C, eq. q-train): the draw for
latent i of grid k at iteration t uses counter (t, k, i, 0) and key
(seed & 0xffffffff, seed >> 32); with r0, r1 its first two words,
u1 = ((r0 >> 8) + 0.5) * 2^-24, u2 = (r1 >> 8) * 2^-24 and
n = sqrt(-2 ln u1) cos(2 pi u2).
"""
import numpy as np

M0 = np.uint64(0xD2511F53)
M1 = np.uint64(0xCD9E8D57)
W0 = 0x9E3779B9
W1 = 0xBB67AE85
MASK = np.uint64(0xFFFFFFFF)


def philox4x32_10(c0, c1, c2, c3, k0, k1):
    """Vectorised Philox4x32-10. Counter words are arrays (broadcast),
    key words are Python ints. Returns four uint32 arrays."""
    c0 = np.asarray(c0, dtype=np.uint64) & MASK
    c1 = np.asarray(c1, dtype=np.uint64) & MASK
    c2 = np.asarray(c2, dtype=np.uint64) & MASK
    c3 = np.asarray(c3, dtype=np.uint64) & MASK
    c0, c1, c2, c3 = np.broadcast_arrays(c0, c1, c2, c3)
    k0 = int(k0) & 0xFFFFFFFF
    k1 = int(k1) & 0xFFFFFFFF
    for r in range(10):
        if r > 0:
            k0 = (k0 + W0) & 0xFFFFFFFF
            k1 = (k1 + W1) & 0xFFFFFFFF
        p0 = M0 * c0
        p1 = M1 * c2
        hi0, lo0 = p0 >> np.uint64(32), p0 & MASK
        hi1, lo1 = p1 >> np.uint64(32), p1 & MASK
        c0, c1, c2, c3 = (hi1 ^ c1 ^ np.uint64(k0), lo1,
                          hi0 ^ c3 ^ np.uint64(k1), lo0)
    return tuple(x.astype(np.uint32) for x in (c0, c1, c2, c3))


def box_muller(r0, r1):
    """Standard normal deviates (float64) from two uint32 words."""
    u1 = ((np.asarray(r0, dtype=np.uint64) >> np.uint64(8)).astype(np.float64)
          + 0.5) * 2.0 ** -24
    u2 = (np.asarray(r1, dtype=np.uint64) >> np.uint64(8)).astype(np.float64) \
        * 2.0 ** -24
    return np.sqrt(-2.0 * np.log(u1)) * np.cos(2.0 * np.pi * u2)


def latent_noise(seed: int, t: int, k: int, n: int) -> np.ndarray:
    """Gaussian noise for the n latents of grid k at iteration t (float64)."""
    i = np.arange(n, dtype=np.uint64)
    r0, r1, _, _ = philox4x32_10(t, k, i, 0, seed & 0xFFFFFFFF,
                                 (seed >> 32) & 0xFFFFFFFF)
    return box_muller(r0, r1)
