"""Philox4x32-10 counter-based generator and the probe laws built on it.

Philox is the published generator of Salmon, Moraes, Dror and Shaw, "Parallel
random numbers: as easy as 1, 2, 3" (SC'11): 10 rounds of a bijection on four
32-bit words, each round two 32x32->64 multiplications by fixed odd constants
whose high halves are xored with the other words and the round key, the key
advanced by a Weyl sequence between rounds.  This implementation is written
from that definition and pinned by the published known-answer vectors.

Probe stream (same definition on the HIP side, written independently there):
element (i, j) of an n x M row-major block has linear index e = i*M + j; it is
word e mod 4 of Philox(counter = (q mod 2^32, q div 2^32, stream, 0),
key = (seed mod 2^32, seed div 2^32)) with q = e div 4.
  * Rademacher: 1 - 2 * (word >> 31).
  * Gaussian (the isotropic probes of Alg. 1): Box-Muller on the word pairs
    (0,1) and (2,3): u = (word + 1/2) 2^-32, r = sqrt(-2 ln u_even),
    theta = 2 pi u_odd, values r cos(theta) (even slot), r sin(theta) (odd slot),
    evaluated in float64.
Test infrastructure: see the package docstring.
"""

import numpy as np

M0 = np.uint64(0xD2511F53)
M1 = np.uint64(0xCD9E8D57)
W0 = np.uint64(0x9E3779B9)
W1 = np.uint64(0xBB67AE85)
MASK = np.uint64(0xFFFFFFFF)
SH = np.uint64(32)


def philox4x32_10(ctr, key):
    """ctr: (..., 4) uint32-valued array, key: (..., 2).  Returns (..., 4) uint32."""
    c = [np.asarray(ctr[..., i], dtype=np.uint64) for i in range(4)]
    k0 = np.asarray(key[..., 0], dtype=np.uint64) & MASK
    k1 = np.asarray(key[..., 1], dtype=np.uint64) & MASK
    for r in range(10):
        p0 = M0 * c[0]
        p1 = M1 * c[2]
        hi0, lo0 = p0 >> SH, p0 & MASK
        hi1, lo1 = p1 >> SH, p1 & MASK
        c = [hi1 ^ c[1] ^ k0, lo1, hi0 ^ c[3] ^ k1, lo0]
        k0 = (k0 + W0) & MASK
        k1 = (k1 + W1) & MASK
    return np.stack(c, axis=-1).astype(np.uint32)


def probe_words(n, M, seed, stream=0):
    """The raw 32-bit word for every element of an n x M block (row-major)."""
    total = n * M
    nq = (total + 3) // 4
    q = np.arange(nq, dtype=np.uint64)
    ctr = np.stack([q & MASK, q >> SH, np.full(nq, stream, dtype=np.uint64), np.zeros(nq, dtype=np.uint64)], axis=-1)
    seed = np.uint64(seed)
    key = np.broadcast_to(np.array([seed & MASK, seed >> SH], dtype=np.uint64), (nq, 2))
    words = philox4x32_10(ctr, key).reshape(-1)[:total]
    return words.reshape(n, M)


def rademacher(n, M, seed, stream=0):
    w = probe_words(n, M, seed, stream).astype(np.int64)
    return (1 - 2 * (w >> 31)).astype(np.float64)


def gaussian(n, M, seed, stream=0):
    total = n * M
    nq = (total + 3) // 4
    q = np.arange(nq, dtype=np.uint64)
    ctr = np.stack([q & MASK, q >> SH, np.full(nq, stream, dtype=np.uint64), np.zeros(nq, dtype=np.uint64)], axis=-1)
    s = np.uint64(seed)
    key = np.broadcast_to(np.array([s & MASK, s >> SH], dtype=np.uint64), (nq, 2))
    w = philox4x32_10(ctr, key).astype(np.float64)
    u = (w + 0.5) * 2.0 ** -32
    out = np.empty((nq, 4))
    for a, b in ((0, 1), (2, 3)):
        r = np.sqrt(-2.0 * np.log(u[:, a]))
        th = 2.0 * np.pi * u[:, b]
        out[:, a] = r * np.cos(th)
        out[:, b] = r * np.sin(th)
    return out.reshape(-1)[:total].reshape(n, M)
