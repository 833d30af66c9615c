"""Philox-4x32-10, written from its published definition (Salmon, Moraes, Dror & Shaw,
"Parallel Random Numbers: As Easy as 1, 2, 3", SC'11, section 4 "Philox").

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

The paper keeps only pseudorandom keys of accepted assignments and regenerates an
assignment from its key on demand (section 2.1, "Key-only storage"; section 4, "Reducing
memory pressure": a key of L = 2 integers).  It does not name the generator; the per-draw
stream used here is Philox-4x32-10, a counter-based generator, so that any draw can be
regenerated from (seed, draw index) without replaying the stream.

Definition (SC'11): the state is a 128-bit counter (x0, x1, x2, x3) and a 64-bit key
(k0, k1), all 32-bit words.  One round computes the two full 64-bit products
    M0 * x0 = (hi0, lo0),   M1 * x2 = (hi1, lo1)
and returns (hi1 ^ x1 ^ k0, lo1, hi0 ^ x3 ^ k1, lo0).  Between rounds the key is bumped
by the Weyl constants, k0 += W0, k1 += W1 (mod 2^32).  Philox-4x32-10 applies 10 rounds,
the first with the key as given.
"""

import numpy as np

M0 = 0xD2511F53
M1 = 0xCD9E8D57
W0 = 0x9E3779B9
W1 = 0xBB67AE85
ROUNDS = 10
_MASK = 0xFFFFFFFF


def philox4x32_10(counter, key):
    """One Philox-4x32-10 block in Python integers.

    counter: 4 ints in [0, 2^32); key: 2 ints in [0, 2^32).  Returns a tuple of 4 ints.
    """
    x0, x1, x2, x3 = (int(c) & _MASK for c in counter)
    k0, k1 = (int(k) & _MASK for k in key)
    for r in range(ROUNDS):
        if r > 0:
            k0 = (k0 + W0) & _MASK
            k1 = (k1 + W1) & _MASK
        p0 = M0 * x0
        p1 = M1 * x2
        hi0, lo0 = p0 >> 32, p0 & _MASK
        hi1, lo1 = p1 >> 32, p1 & _MASK
        x0, x1, x2, x3 = hi1 ^ x1 ^ k0, lo1, hi0 ^ x3 ^ k1, lo0
    return x0, x1, x2, x3


def philox4x32_10_np(x0, x1, x2, x3, k0, k1):
    """The same block function applied elementwise to NumPy arrays.

    Counters are broadcastable integer arrays with values in [0, 2^32); the key is two
    Python ints.  Arithmetic is done in uint64 so that the 32x32 -> 64-bit products are
    exact.  Returns four uint64 arrays holding 32-bit words.
    """
    mask = np.uint64(_MASK)
    sh = np.uint64(32)
    x0 = np.asarray(x0, dtype=np.uint64) & mask
    x1 = np.asarray(x1, dtype=np.uint64) & mask
    x2 = np.asarray(x2, dtype=np.uint64) & mask
    x3 = np.asarray(x3, dtype=np.uint64) & mask
    k0 = int(k0) & _MASK
    k1 = int(k1) & _MASK
    m0 = np.uint64(M0)
    m1 = np.uint64(M1)
    for r in range(ROUNDS):
        if r > 0:
            k0 = (k0 + W0) & _MASK
            k1 = (k1 + W1) & _MASK
        p0 = x0 * m0
        p1 = x2 * m1
        n0 = (p1 >> sh) ^ x1 ^ np.uint64(k0)
        n1 = p1 & mask
        n2 = (p0 >> sh) ^ x3 ^ np.uint64(k1)
        n3 = p0 & mask
        x0, x1, x2, x3 = n0, n1, n2, n3
    return x0, x1, x2, x3
