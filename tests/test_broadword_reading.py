"""The reading of Section 3.3's broadword maximisation that the 5-bit register kernels use,
checked on the CPU with Python integers (no GPU, no library code).

A counter's registers are k-bit fields of one long bit string (register j at bits
kj .. kj+k-1, little-endian). The paper's comparison sets the high bit of every field where
x < y; a mask built from it selects x or y per field. The bit string is processed in 64-bit
words with multi-precision subtraction and shifts, so fields that straddle two words must
come out right through the borrows alone. These tests evaluate the formulas on whole
Python integers (exact multi-precision) and also word by word with explicit borrows, and
compare both with the plain register-wise max.
"""
import numpy as np
import pytest


def _consts(k, nbits):
    L = sum(1 << (k * i) for i in range(nbits // k))
    return L, L << (k - 1)


def _pack(fields, k):
    return sum(int(f) << (k * j) for j, f in enumerate(fields))


def _unpack(x, k, count):
    return [(x >> (k * j)) & ((1 << k) - 1) for j in range(count)]


def broadword_max(x, y, k, nbits):
    """Section 3.3 on one multi-word bit string held as a Python integer."""
    full = (1 << nbits) - 1
    L, H = _consts(k, nbits)
    lt = ((((x | H) - (y & ~H & full)) | (x ^ y)) ^ (x | (~y & full))) & H
    mask = ((((lt >> (k - 1)) | H) - L) | H) ^ lt
    return (x & mask) | (y & ~mask & full)


def broadword_max_words(xw, yw, k):
    """The same on a list of 64-bit words with explicit borrow and shift chains."""
    n = len(xw)
    M = (1 << 64) - 1
    L, H = _consts(k, 64 * n)
    Lw = [(L >> (64 * i)) & M for i in range(n)]
    Hw = [(H >> (64 * i)) & M for i in range(n)]
    lt, borrow = [], 0
    for i in range(n):
        a, b = xw[i] | Hw[i], yw[i] & ~Hw[i] & M
        d = (a - b - borrow) & M
        borrow = 1 if a < b + borrow else 0
        lt.append(((d | (xw[i] ^ yw[i])) ^ (xw[i] | (~yw[i] & M))) & Hw[i])
    out, borrow = [], 0
    for i in range(n):
        sh = (lt[i] >> (k - 1)) | ((lt[i + 1] << (65 - k)) & M if i + 1 < n else 0)
        a = sh | Hw[i]
        d = (a - Lw[i] - borrow) & M
        borrow = 1 if a < Lw[i] + borrow else 0
        mask = (d | Hw[i]) ^ lt[i]
        out.append((xw[i] & mask) | (yw[i] & ~mask & M))
    return out


def _words(x, n):
    return [(x >> (64 * i)) & ((1 << 64) - 1) for i in range(n)]


@pytest.mark.parametrize("k,count", [(5, 64), (5, 128), (8, 8), (8, 16), (4, 16), (6, 32)])
def test_broadword_max_is_registerwise_max(k, count):
    rng = np.random.default_rng(k * 1000 + count)
    nbits = k * count
    nw = -(-nbits // 64)
    for _ in range(300):
        a = rng.integers(0, 1 << k, count)
        b = rng.integers(0, 1 << k, count)
        # half the fields equal, to exercise ties next to differing fields
        eq = rng.random(count) < 0.3
        b[eq] = a[eq]
        x, y = _pack(a, k), _pack(b, k)
        want = np.maximum(a, b)
        got = broadword_max(x, y, k, nbits)
        assert _unpack(got, k, count) == list(want)
        if nbits % 64 == 0:  # the paper's word-aligned case: word-by-word chains
            gw = broadword_max_words(_words(x, nw), _words(y, nw), k)
            assert _unpack(sum(w << (64 * i) for i, w in enumerate(gw)), k, count) == list(want)


def test_broadword_max5_every_pair_at_every_position():
    """Every pair of 5-bit values in every field of a 320-bit (five-word) group, the others
    random: the straddling fields 12, 25, 38 and 51 included."""
    rng = np.random.default_rng(5)
    vals = np.arange(32)
    for j in range(64):
        for a in vals:
            xa = rng.integers(0, 32, 64)
            yb = rng.integers(0, 32, 64)
            for b in vals:
                xa[j], yb[j] = a, b
                gw = broadword_max_words(_words(_pack(xa, 5), 5), _words(_pack(yb, 5), 5), 5)
                got = _unpack(sum(w << (64 * i) for i, w in enumerate(gw)), 5, 64)
                assert got[j] == max(a, b)
                assert got == list(np.maximum(xa, yb))


def test_straddling_fields_are_where_expected():
    """With 64 five-bit registers per five words, exactly fields 12, 25, 38 and 51 cross a
    64-bit word boundary."""
    cross = [j for j in range(64) if (5 * j) // 64 != (5 * j + 4) // 64]
    assert cross == [12, 25, 38, 51]


def test_comparison_bits():
    """The comparison alone: the high bit of field j is set exactly where x_j < y_j."""
    k, count = 5, 64
    nbits = k * count
    full = (1 << nbits) - 1
    L, H = _consts(k, nbits)
    rng = np.random.default_rng(9)
    for _ in range(200):
        a = rng.integers(0, 32, count)
        b = rng.integers(0, 32, count)
        x, y = _pack(a, k), _pack(b, k)
        lt = ((((x | H) - (y & ~H & full)) | (x ^ y)) ^ (x | (~y & full))) & H
        assert [(lt >> (k * j + k - 1)) & 1 for j in range(count)] == list((a < b).astype(int))
