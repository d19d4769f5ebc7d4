"""Philox4x32-10 and the Gaussian sketch matrix.

Philox4x32 with 10 rounds is the counter-based generator of Salmon, Moraes,
Dror and Shaw ("Parallel random numbers: as easy as 1, 2, 3", SC 2011).
One round maps counter (c0, c1, c2, c3) under key (k0, k1) to
    (hi(M1*c2) ^ c1 ^ k0, lo(M1*c2), hi(M0*c0) ^ c3 ^ k1, lo(M0*c0))
with M0 = 0xD2511F53 and M1 = 0xCD9E8D57; between rounds the key is bumped
by the Weyl constants (0x9E3779B9, 0xBB67AE85).

The randomized step-1 solver needs an N x k Gaussian matrix Omega (section
3.2.3).  Entry (j, c) (row j, column c) is defined as follows: the counter
(j // 4, c, 0, 0) under key (seed mod 2^32, seed >> 32) gives four words a0..a3;
each word maps to u = (a + 1/2) / 2^32 in (0, 1); Box-Muller on (u0, u1) gives
rows 4q, 4q+1 as r cos(2 pi u1), r sin(2 pi u1) with r = sqrt(-2 ln u0), and
(u2, u3) gives rows 4q+2, 4q+3 the same way.
"""
import numpy as np

M0, M1 = 0xD2511F53, 0xCD9E8D57
W0, W1 = 0x9E3779B9, 0xBB67AE85
MASK = 0xFFFFFFFF


def _mulhilo(a, b):
    p = a.astype(np.uint64) * np.uint64(b)
    return (p >> np.uint64(32)).astype(np.uint32), (p & np.uint64(MASK)).astype(np.uint32)


def philox4x32(ctr, key, rounds=10):
    """ctr: uint32 array (..., 4); key: (k0, k1) python ints.  Returns (..., 4)."""
    c = [np.asarray(ctr[..., i], dtype=np.uint32) for i in range(4)]
    k0, k1 = key[0] & MASK, key[1] & MASK
    for rnd in range(rounds):
        if rnd:
            k0 = (k0 + W0) & MASK
            k1 = (k1 + W1) & MASK
        hi0, lo0 = _mulhilo(c[0], M0)
        hi1, lo1 = _mulhilo(c[2], M1)
        c = [hi1 ^ c[1] ^ np.uint32(k0), lo1, hi0 ^ c[3] ^ np.uint32(k1), lo0]
    return np.stack(c, axis=-1)


def gaussian_sketch(N, k, seed):
    """The N x k matrix Omega defined in the module docstring (FP64)."""
    nq = (N + 3) // 4
    q, col = np.meshgrid(np.arange(nq, dtype=np.uint32),
                         np.arange(k, dtype=np.uint32), indexing="ij")
    ctr = np.stack([q, col, np.zeros_like(q), np.zeros_like(q)], axis=-1)
    a = philox4x32(ctr, (seed & MASK, (seed >> 32) & MASK))
    u = (a.astype(np.float64) + 0.5) * (1.0 / 4294967296.0)
    out = np.empty((nq, 4, k))
    for pair in range(2):
        r = np.sqrt(-2.0 * np.log(u[..., 2 * pair]))
        t = 2.0 * np.pi * u[..., 2 * pair + 1]
        out[:, 2 * pair, :] = r * np.cos(t)
        out[:, 2 * pair + 1, :] = r * np.sin(t)
    return out.reshape(4 * nq, k)[:N]
