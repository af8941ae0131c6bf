"""Philox4x32-10 counter-based generator and the detector's word layout (test oracle).

TEST INFRASTRUCTURE ONLY: nothing in the product path may import this module.

Philox is not part of the paper; the paper only says that the proposal is sampled
(Algorithm 1, "Sample x'_n ~ q_n") and that u ~ U(0,1) is drawn for the MH test.
A counter-based generator is used so that the oracle and the GPU kernels can draw
the same random numbers independently.  The generator is written from its
published definition: Salmon, Moraes, Dror, Shaw, "Parallel Random Numbers: As
Easy as 1, 2, 3", SC'11 (the Philox-4x32 S-box: two 32x32->64 multiplications
per round, the outputs' high halves xor-ed with the other counter words and the
round key; the key advanced between rounds by a Weyl sequence).

Word layout (shared convention, implemented separately on each side):
  key     = (seed mod 2^32, seed >> 32)
  counter = (block, t, chain, instance); a block yields 4 words
  word j of the stream of (instance, chain, t) = block j>>2, lane j&3
  * t = 0: initial state, real dimension n takes word n; level index
    k = ((w >> 8) * Q) >> 24  (a uniform 24-bit fraction times Q, floored)
  * t >= 1 (transition t): real dimension n takes word n, the uniform of its
    draw is ((w >> 9) + 1/2) * 2^-23 (the midpoint of the word's 23-bit cell:
    in (0, 1), so the inverse CDF never compares against an exact zero, and
    exact in fp32); the MH uniform is the 24-bit number formed from the low
    bytes of words 0, 1, 2 (word 0 least significant), times 2^-24; the kernel
    mixture uniform is formed the same way from the low bytes of words 4, 5, 6.
  The real dimensions are interleaved per antenna: n = 2m is Re x_m, n = 2m+1 is
  Im x_m.  At least two blocks (8 words) are generated per (instance, chain, t).
"""
import numpy as np

M0 = np.uint64(0xD2511F53)
M1 = np.uint64(0xCD9E8D57)
W0 = np.uint64(0x9E3779B9)
W1 = np.uint64(0xBB67AE85)
MASK32 = np.uint64(0xFFFFFFFF)


def philox4x32_10(c0, c1, c2, c3, k0, k1):
    """Philox4x32 with 10 rounds on broadcastable uint32 arrays.

    Returns a tuple of 4 uint32 arrays (the output words in order).
    """
    c0 = np.asarray(c0, dtype=np.uint64) & MASK32
    c1 = np.asarray(c1, dtype=np.uint64) & MASK32
    c2 = np.asarray(c2, dtype=np.uint64) & MASK32
    c3 = np.asarray(c3, dtype=np.uint64) & MASK32
    k0 = np.asarray(k0, dtype=np.uint64) & MASK32
    k1 = np.asarray(k1, dtype=np.uint64) & MASK32
    for r in range(10):
        if r > 0:  # Weyl key schedule between rounds
            k0 = (k0 + W0) & MASK32
            k1 = (k1 + W1) & MASK32
        p0 = M0 * c0  # exact: both factors < 2^32, product < 2^64
        p1 = M1 * c2
        hi0, lo0 = p0 >> np.uint64(32), p0 & MASK32
        hi1, lo1 = p1 >> np.uint64(32), p1 & MASK32
        c0, c1, c2, c3 = (hi1 ^ c1 ^ k0), lo1, (hi0 ^ c3 ^ k1), lo0
    return tuple(v.astype(np.uint32) for v in (c0, c1, c2, c3))


def seed_key(seed):
    seed = int(seed) & ((1 << 64) - 1)
    return seed & 0xFFFFFFFF, seed >> 32


def words(seed, instance, chains, t, n_words):
    """Words 0..n_words-1 of the stream of (instance, chain, t) for every chain.

    chains: 1-D int array.  Returns uint32 array of shape (len(chains), n_words').
    n_words is rounded up to a multiple of 4 and to at least 8.
    """
    chains = np.asarray(chains, dtype=np.uint64)
    nb = max(2, (int(n_words) + 3) // 4)
    k0, k1 = seed_key(seed)
    blocks = np.arange(nb, dtype=np.uint64)
    b, c = np.meshgrid(blocks, chains)  # (C, nb)
    out = philox4x32_10(b, np.uint64(t), c, np.uint64(instance), k0, k1)
    w = np.stack(out, axis=-1)  # (C, nb, 4)
    return w.reshape(len(chains), nb * 4)


def uniform24(w):
    """High 24 bits of a word as a fraction in [0, 1) (exact in fp32 and fp64)."""
    return (np.asarray(w, dtype=np.uint32) >> np.uint32(8)).astype(np.float64) * 2.0 ** -24


def uniform_draw(w):
    """Uniform of a proposal draw: ((w >> 9) + 1/2) * 2^-23, in (0, 1), exact in fp32 and fp64."""
    return ((np.asarray(w, dtype=np.uint32) >> np.uint32(9)).astype(np.float64) + 0.5) * 2.0 ** -23


def low_byte_uniform(w, j0):
    """24-bit uniform assembled from the low bytes of words j0, j0+1, j0+2."""
    w = np.asarray(w, dtype=np.uint32)
    v = (w[..., j0] & np.uint32(0xFF)).astype(np.uint64)
    v |= (w[..., j0 + 1] & np.uint32(0xFF)).astype(np.uint64) << np.uint64(8)
    v |= (w[..., j0 + 2] & np.uint32(0xFF)).astype(np.uint64) << np.uint64(16)
    return v.astype(np.float64) * 2.0 ** -24


def init_level_index(w, Q):
    """Initial level index floor(u * Q) with u the high 24 bits of the word."""
    w = np.asarray(w, dtype=np.uint32)
    return (((w >> np.uint32(8)).astype(np.uint64) * np.uint64(Q)) >> np.uint64(24)).astype(np.int64)
