"""Candidate assignments from keys: Monte Carlo draws and exact enumeration.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

Section 2.3 ("generate_randomizations()") describes two generation modes: Monte Carlo
draws of complete randomizations with n1 of n units treated, filtered by balance, and
exact enumeration of all C(n, n1) assignments when that is feasible.  Section 2.1
("Key-only storage") keeps a key per accepted draw from which the assignment is
regenerated.  The paper fixes neither the stream layout nor the order of enumeration;
the readings implemented here are:

Monte Carlo (key = draw index b, plus a 64-bit seed shared by the whole pool):
  * unit i reads word r = (i // 64) % 4 of Philox-4x32-10 block j = 64 * (i // 256) + i % 64,
    with counter (j, 0, lo32(b), hi32(b)) and key (lo32(seed), hi32(seed));
  * the treated set is the n1 units with the smallest (u_i, i) pairs, i.e. ties between
    equal 32-bit words go to the smaller unit index.
  Ranking n iid uniform keys and treating the n1 smallest gives every n1-subset the same
  probability, which is complete randomization.

Exact enumeration (key = colex rank r in [0, C(n, n1))):
  * the treated set {i_1 < ... < i_n1} has rank r = sum_t C(i_t, t) (combinatorial
    number system, co-lexicographic order).

Bitmask format: bit (i % 32) of 32-bit word (i // 32) is 1 iff unit i is treated.
"""

from math import comb

import numpy as np

from .philox import philox4x32_10, philox4x32_10_np

_MASK = 0xFFFFFFFF


def unit_block_word(i):
    """(Philox block j, output word r) that unit i reads."""
    return 64 * (i // 256) + i % 64, (i // 64) % 4


def unit_keys(seed, b, n):
    """The n 32-bit unit keys u_0..u_{n-1} of Monte Carlo draw b (Python ints)."""
    key = (seed & _MASK, (seed >> 32) & _MASK)
    cache = {}
    u = []
    for i in range(n):
        j, r = unit_block_word(i)
        if j not in cache:
            cache[j] = philox4x32_10((j, 0, b & _MASK, (b >> 32) & _MASK), key)
        u.append(cache[j][r])
    return u


def smallest_set(u, n1):
    """Indices of the n1 smallest (u_i, i) pairs, ascending by index."""
    order = sorted(range(len(u)), key=lambda i: (u[i], i))
    return sorted(order[:n1])


def mc_assignment(seed, b, n, n1):
    """0/1 treatment vector (numpy uint8) of Monte Carlo draw b; scalar reference."""
    w = np.zeros(n, dtype=np.uint8)
    w[smallest_set(unit_keys(seed, b, n), n1)] = 1
    return w


def unit_keys_batch(seed, keys, n):
    """Unit keys for many draws at once: (len(keys), n) uint32 array (NumPy)."""
    keys = np.asarray(keys, dtype=np.uint64)
    i = np.arange(n)
    jj = (64 * (i // 256) + i % 64).astype(np.uint64)
    rr = (i // 64) % 4
    nblk = int(jj.max()) + 1 if n > 0 else 0
    blocks = np.arange(nblk, dtype=np.uint64)
    lo = (keys & np.uint64(_MASK))[:, None]
    hi = (keys >> np.uint64(32))[:, None]
    out = philox4x32_10_np(blocks[None, :], np.uint64(0), lo, hi,
                           seed & _MASK, (seed >> 32) & _MASK)
    words = np.stack(out, axis=-1)            # (B, nblk, 4)
    return words[:, jj, rr].astype(np.uint32)


def mc_assignments_batch(seed, keys, n, n1):
    """(len(keys), n) uint8 treatment matrix; a stable sort on u puts ties in index order."""
    u = unit_keys_batch(seed, keys, n)
    order = np.argsort(u, axis=1, kind="stable")[:, :n1]
    w = np.zeros(u.shape, dtype=np.uint8)
    np.put_along_axis(w, order, 1, axis=1)
    return w


def colex_rank(treated):
    """Rank of a treated set (iterable of distinct unit indices) in colex order."""
    return sum(comb(i, t + 1) for t, i in enumerate(sorted(treated)))


def colex_unrank(r, n, n1):
    """Treated set (ascending indices) of colex rank r; the inverse of ``colex_rank``."""
    if not 0 <= r < comb(n, n1):
        raise ValueError("rank out of range")
    out = []
    hi = n
    for t in range(n1, 0, -1):
        i = hi - 1
        while comb(i, t) > r:
            i -= 1
        out.append(i)
        r -= comb(i, t)
        hi = i
    return sorted(out)


def exact_assignment(r, n, n1):
    w = np.zeros(n, dtype=np.uint8)
    w[colex_unrank(r, n, n1)] = 1
    return w


def exact_assignments(n, n1):
    """All C(n, n1) assignments, row r = colex rank r (uint8 matrix)."""
    total = comb(n, n1)
    w = np.zeros((total, n), dtype=np.uint8)
    for r in range(total):
        w[r, colex_unrank(r, n, n1)] = 1
    return w


def pack_bits(w):
    """Pack 0/1 rows into 32-bit words: bit i % 32 of word i // 32 is w[i]."""
    w = np.atleast_2d(np.asarray(w, dtype=np.uint8))
    B, n = w.shape
    nw = (n + 31) // 32
    pad = np.zeros((B, nw * 32), dtype=np.uint64)
    pad[:, :n] = w
    weights = (np.uint64(1) << np.arange(32, dtype=np.uint64))
    return (pad.reshape(B, nw, 32) * weights).sum(axis=2).astype(np.uint32)


def unpack_bits(words, n):
    words = np.atleast_2d(np.asarray(words, dtype=np.uint32)).astype(np.uint64)
    bits = (words[:, :, None] >> np.arange(32, dtype=np.uint64)) & np.uint64(1)
    return bits.reshape(words.shape[0], -1)[:, :n].astype(np.uint8)
