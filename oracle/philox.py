"""Philox4x32-10 counter-based generator, written from its published definition
(J. K. Salmon, M. A. Moraes, R. O. Dror, D. E. Shaw, "Parallel random numbers:
as easy as 1, 2, 3", SC'11, Section 4 and its Philox-4x32 parameter table).

The paper draws Pi with i.i.d. N(0, 1/k) entries (Alg. 1 step 2) and samples each
entry of the n1 x n2 grid independently (Alg. 1 step 3) but names no generator.
Both sides of the parity check therefore implement this one generator from its
definition; nothing is shared between them.

Definition restated:
  state: four 32-bit counter words (x0, x1, x2, x3) and a 2-word key (k0, k1)
  one round:  (hi0, lo0) = 0xD2511F53 * x0   (full 64-bit product)
              (hi1, lo1) = 0xCD9E8D57 * x2
              (x0, x1, x2, x3) <- (hi1 ^ x1 ^ k0, lo1, hi0 ^ x3 ^ k1, lo0)
  key schedule: round r (r = 0..9) uses (k0 + r*0x9E3779B9, k1 + r*0xBB67AE85) mod 2^32
  output: the four counter words after ten rounds.

Streams used by SMP-PCA (the "counter spec"):
  key = (seed mod 2^32, seed >> 32)
  counter = (col_block, row mod 2^32, tag, row >> 32)
  where a call serves four consecutive columns 4*col_block .. 4*col_block + 3.
  Tags: TAG_PI = 1 (Pi, row = d index l, col = sketch row c),
        TAG_SAMPLE = 2 (row = i, col = j), TAG_SPLIT = 3 (row = i, col = j).

Parity: pinned against rocRAND's independent Philox4x32-10 (tests/test_oracle_rng.py).
"""

import numpy as np

_MASK = np.uint64(0xFFFFFFFF)
_M0 = np.uint64(0xD2511F53)
_M1 = np.uint64(0xCD9E8D57)
_W0 = 0x9E3779B9
_W1 = 0xBB67AE85

TAG_PI = 1
TAG_SAMPLE = 2
TAG_SPLIT = 3


def philox4x32_10(x0, x1, x2, x3, k0, k1):
    """Ten Philox-4x32 rounds on counter words (x0..x3) under key (k0, k1).

    x0..x3 are integer arrays (broadcastable) holding values < 2^32; k0, k1 are
    Python ints < 2^32. Returns four uint32 arrays.
    """
    c0 = np.asarray(x0, dtype=np.uint64)
    c1 = np.asarray(x1, dtype=np.uint64)
    c2 = np.asarray(x2, dtype=np.uint64)
    c3 = np.asarray(x3, dtype=np.uint64)
    c0, c1, c2, c3 = np.broadcast_arrays(c0, c1, c2, c3)
    key0 = int(k0) & 0xFFFFFFFF
    key1 = int(k1) & 0xFFFFFFFF
    for _ in range(10):
        p0 = _M0 * c0          # < 2^64, exact in uint64
        p1 = _M1 * c2
        hi0, lo0 = p0 >> np.uint64(32), p0 & _MASK
        hi1, lo1 = p1 >> np.uint64(32), p1 & _MASK
        c0, c1, c2, c3 = (hi1 ^ c1 ^ np.uint64(key0), lo1,
                          hi0 ^ c3 ^ np.uint64(key1), lo0)
        key0 = (key0 + _W0) & 0xFFFFFFFF
        key1 = (key1 + _W1) & 0xFFFFFFFF
    return (c0.astype(np.uint32), c1.astype(np.uint32),
            c2.astype(np.uint32), c3.astype(np.uint32))


def seed_key(seed):
    """Split a 64-bit seed into the Philox key words."""
    seed = int(seed) & 0xFFFFFFFFFFFFFFFF
    return seed & 0xFFFFFFFF, seed >> 32


def stream_words(seed, tag, rows, col_blocks):
    """Philox output for counters (col_block, row_lo, tag, row_hi).

    rows, col_blocks: integer arrays, broadcast against each other.
    Returns the four output words, each of the broadcast shape.
    """
    k0, k1 = seed_key(seed)
    rows = np.asarray(rows, dtype=np.uint64)
    cb = np.asarray(col_blocks, dtype=np.uint64)
    rows, cb = np.broadcast_arrays(rows, cb)
    return philox4x32_10(cb, rows & _MASK, np.uint64(tag), rows >> np.uint64(32), k0, k1)


def stream_word_at(seed, tag, rows, cols):
    """The 32-bit word that the counter spec assigns to (row, col): output word
    (col mod 4) of the call with col_block = col // 4."""
    rows = np.asarray(rows, dtype=np.int64)
    cols = np.asarray(cols, dtype=np.int64)
    rows, cols = np.broadcast_arrays(rows, cols)
    w = stream_words(seed, tag, rows, cols // 4)
    lane = cols % 4
    return np.choose(lane, w).astype(np.uint32)
