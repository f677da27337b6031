"""Register saturation on the GPU (Section 3.1: rho+ of the bits after the register index,
kept in 5-bit registers, so saturated at 31). A random node reaches 30 or more leading
zeroes with probability about 2^-30, so the cap and the all-zero tail are reached here by
choosing the hash seed: splitmix64's output mixing is a bijection (xor-shifts and odd
multipliers, each invertible), so for a chosen node v and a chosen 64-bit hash h the seed
whose (v+1)-th output is h is computed by inverting it. Each crafted run is compared with the
oracle at every iteration, for b = 4..8, with byte and 5-bit registers.

The CPU test pins the inversion itself: the oracle's hash of the crafted seed is h."""
import sys

import numpy as np
import pytest

import graphgen
import oracle

hanf = None

GAMMA = 0x9E3779B97F4A7C15
M1 = 0xBF58476D1CE4E5B9
M2 = 0x94D049BB133111EB
MASK = (1 << 64) - 1


def _unxorshift(y, s):
    """x with x ^ (x >> s) == y (64-bit)."""
    x = y
    k = s
    while k < 64:
        x = y ^ (x >> s)
        k += s
    return x & MASK


def seed_for(h, v):
    """The splitmix64 seed whose output number v + 1 is h: undo z ^ (z >> 31), the
    multiplication by M2, z ^ (z >> 27), the multiplication by M1 and z ^ (z >> 30), then
    subtract the v + 1 increments of the state."""
    z = _unxorshift(h, 31)
    z = (z * pow(M2, -1, 1 << 64)) & MASK
    z = _unxorshift(z, 27)
    z = (z * pow(M1, -1, 1 << 64)) & MASK
    z = _unxorshift(z, 30)
    return (z - (v + 1) * GAMMA) & MASK


def crafted_hash(b, idx, zeros):
    """Register index idx in the leftmost b bits; the remaining 64 - b bits start with
    exactly `zeros` zeroes (all zero when zeros >= 64 - b); the bits after the first one
    are ones, to show that they do not matter."""
    tail = 64 - b
    h = idx << tail
    if zeros < tail:
        h |= (1 << (tail - zeros)) - 1
    return h


CASES = [29, 30, 31, 32, 40, 64]  # leading zeroes of the tail (64: all zero)


@pytest.mark.parametrize("b", [4, 5, 6, 7, 8])
def test_crafted_seed_gives_the_chosen_hash(b):
    rng = np.random.default_rng(b)
    for zeros in CASES:
        idx = int(rng.integers(0, 1 << b))
        h = crafted_hash(b, idx, zeros)
        v = int(rng.integers(0, 5000))
        s = seed_for(h, v)
        assert oracle.hash64(s, v) == h
        assert oracle.register_index(h, b) == idx
        assert min(oracle.rho_plus(h, b), 31) == min(zeros + 1 if zeros < 64 - b else 64 - b + 1, 31)
        M = np.zeros(1 << b, np.uint8)
        oracle.add(M, b, s, v)
        assert M[idx] == min(zeros + 1, 31) and M.sum() == M[idx]


@pytest.mark.gpu
@pytest.mark.parametrize("b", [4, 5, 6, 7, 8])
@pytest.mark.parametrize("packed", [0, 1])
def test_saturated_registers_on_the_gpu(b, packed):
    global hanf
    hanf = pytest.importorskip("paper_1011_5599_amd")
    if packed and b < 6:
        pytest.skip("5-bit registers need m >= 64")
    rp, ci = graphgen.rmat(11, 12_000, seed=77)
    n = len(rp) - 1
    rng = np.random.default_rng(100 + b)
    for zeros in CASES:
        v = int(rng.integers(0, n))
        idx = int(rng.integers(0, 1 << b))
        seed = seed_for(crafted_hash(b, idx, zeros), v)
        print(f"[saturation] b={b} packed={packed} zeros={zeros} node={v} seed={seed:#x}", flush=True)
        sys.stdout.flush()
        ref = list(oracle.run_steps(rp, ci, b, seed))
        assert ref[0][1][v, idx] == min(zeros + 1, 31)
        with hanf.HyperANF(0, packed5=packed) as h:
            h.load(rp, ci).init(b, seed)
            for t, c, _ in ref:
                assert np.array_equal(h.registers(), c), (zeros, t)
                st, _, _ = h.step(1)
            assert st == hanf.HANF_DONE
            np.testing.assert_allclose(h.nt(), [s for _, _, s in ref], rtol=1e-12, atol=0)
