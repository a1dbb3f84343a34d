"""Philox4x32-10 counter-based random numbers (Salmon, Moraes, Dror, Shaw,
"Parallel random numbers: as easy as 1, 2, 3", SC'11), written from that
definition in plain numpy uint64 arithmetic.

One block maps a 128-bit counter (c0, c1, c2, c3) and a 64-bit key (k0, k1) to
four 32-bit words by ten rounds of
    (hi0, lo0) = M0 * c0,  (hi1, lo1) = M1 * c2     (32x32 -> 64-bit products)
    c <- (hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0)
with the key bumped by the Weyl constants (W0, W1) between rounds.

Stream convention shared with the device generator: element i of a stream
(seed, stream) is word (i mod 4) of the block with counter (i div 4, stream, 0, 0)
and key (seed mod 2^32, seed div 2^32).  ``uniform01`` maps a word x to
(x + 0.5) / 2^32, exact in FP64.
"""
import numpy as np

M0, M1 = 0xD2511F53, 0xCD9E8D57
W0, W1 = 0x9E3779B9, 0xBB67AE85
_MASK = 0xFFFFFFFF


def philox4x32(ctr, key, rounds=10):
    """ctr: uint array [..., 4]; key: (k0, k1).  Returns uint64 array [..., 4] of words."""
    c = np.asarray(ctr, dtype=np.uint64) & _MASK
    c0, c1, c2, c3 = (c[..., i].copy() for i in range(4))
    k0, k1 = np.uint64(key[0] & _MASK), np.uint64(key[1] & _MASK)
    for r in range(rounds):
        if r:
            k0 = np.uint64((int(k0) + W0) & _MASK)
            k1 = np.uint64((int(k1) + W1) & _MASK)
        p0 = c0 * np.uint64(M0)
        p1 = c2 * np.uint64(M1)
        hi0, lo0 = p0 >> np.uint64(32), p0 & np.uint64(_MASK)
        hi1, lo1 = p1 >> np.uint64(32), p1 & np.uint64(_MASK)
        c0, c1, c2, c3 = hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0
    return np.stack([c0, c1, c2, c3], axis=-1)


def stream_words(seed, stream, n):
    """First n 32-bit words of stream (seed, stream)."""
    nblk = (n + 3) // 4
    ctr = np.zeros((nblk, 4), dtype=np.uint64)
    ctr[:, 0] = np.arange(nblk, dtype=np.uint64)
    ctr[:, 1] = stream & _MASK
    words = philox4x32(ctr, (seed & _MASK, (seed >> 32) & _MASK))
    return words.reshape(-1)[:n]


def uniform01(seed, stream, n):
    """n FP64 uniforms in (0, 1): (word + 0.5) / 2^32."""
    return (stream_words(seed, stream, n).astype(np.float64) + 0.5) / 4294967296.0
