"""Host check of the FP32 path's fixed-point deposit arithmetic (no GPU).

The particle passes convert a contribution u*x (two FP32 factors, |u*x| at
most 2^32 after scaling) to fixed point with one FP64 operation,
u*x + 1.5*2^52, and add the resulting bit patterns into 64-bit LDS words
without subtracting the constant.  The claim: the low 48 bits of such a sum,
read as a signed 48-bit integer, equal the sum of the rounded products
whenever that sum stays below 2^47 in magnitude.  Here the arithmetic is
replayed in numpy (the FP32 product is exact in FP64, so adding the constant
rounds once, as the fused operation does) and compared with exact integer
sums.
"""
import numpy as np
import pytest

MAGIC = np.float64(6755399441055744.0)  # 1.5 * 2^52
MASK64 = (1 << 64) - 1


def bit_pattern(u, x):
    p = u.astype(np.float64) * x.astype(np.float64)  # exact: 24 + 24 bits
    return (p + MAGIC).view(np.int64)


def word_sum(patterns):
    return int(sum(int(v) & MASK64 for v in patterns)) & MASK64


def read_sum(word):
    low = word & ((1 << 48) - 1)
    return low - (1 << 48) if low >= 1 << 47 else low


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_bit_pattern_sums_equal_rounded_sums(seed):
    rng = np.random.default_rng(seed)
    n = 8192  # two contributions per particle of a 4096-particle work item
    u = rng.uniform(-1.0, 1.0, n).astype(np.float32)
    x = (rng.uniform(-1.0, 1.0, n) * 2.0**32).astype(np.float32)
    pats = bit_pattern(u, x)
    # each pattern is the constant's bits plus the product rounded to nearest (even)
    exact = np.rint(u.astype(np.float64) * x.astype(np.float64)).astype(np.int64)
    assert np.all(pats - MAGIC.view(np.int64) == exact)
    assert read_sum(word_sum(pats)) == int(exact.sum())


def test_sum_at_the_bound_and_sign():
    # 8192 contributions of +2^32 (and then of -2^32) reach 2^45 in magnitude,
    # inside the +-2^47 the low 48 bits hold
    n = 8192
    u = np.ones(n, np.float32)
    for sign in (1.0, -1.0):
        x = np.full(n, sign * 2.0**32, np.float32)
        assert read_sum(word_sum(bit_pattern(u, x))) == int(sign) * n * 2**32


def test_mixed_signs_cancel_exactly():
    rng = np.random.default_rng(7)
    x = (rng.uniform(0.0, 1.0, 4096) * 2.0**30).astype(np.float32)
    u = np.ones(4096, np.float32)
    pats = np.concatenate([bit_pattern(u, x), bit_pattern(-u, x)])
    rng.shuffle(pats)  # the order of the atomics does not matter
    assert read_sum(word_sum(pats)) == 0
