"""Pins for the oracle's randomness: Philox4x64-10, Feistel bijections,
sign vector and nested row sets (SRHT of Sec. 2.1, nested sets of Sec. 2.2)."""
import numpy as np
import pytest

from oracle.feistel import feistel_forward, feistel_inverse
from oracle.philox import MASK64, philox4x64, philox4x64_ref
from oracle.sketch import (STREAM_PI, STREAM_PIHAT, hat_slot_rows, input_perm, padded_bits,
                           sign_vector, slot_rows)


def _numpy_philox_block(counter, key):
    """numpy.random.Philox (independent library code, 4x64 with 10 rounds)
    increments its 256-bit counter before producing a block, so the first
    block it returns for counter c is Philox(c + 1)."""
    bg = np.random.Philox(counter=np.array(counter, dtype=np.uint64),
                          key=np.array(key, dtype=np.uint64))
    return tuple(int(v) for v in bg.random_raw(4))


def _add_one(counter):
    c = list(counter)
    for i in range(4):
        c[i] = (c[i] + 1) & MASK64
        if c[i] != 0:
            break
    return c


@pytest.mark.parametrize("counter,key", [
    ((0, 0, 0, 0), (0, 0)),
    ((1, 2, 3, 4), (5, 6)),
    ((MASK64, 7, 0, 0), (1, 2)),                       # carry into word 1
    ((0x243F6A8885A308D3, 0x13198A2E03707344, 0xA4093822299F31D0, 0x082EFA98EC4E6C89),
     (0x452821E638D01377, 0xBE5466CF34E90C6C)),
    ((123456789, 0, 0, 0), (20261203, 3)),
])
def test_philox_matches_numpy(counter, key):
    got = philox4x64_ref(_add_one(counter), key)
    assert got == _numpy_philox_block(counter, key)


def test_philox_vectorised_equals_reference():
    rng = np.random.default_rng(5)
    c = rng.integers(0, 2**63, size=(4, 64), dtype=np.uint64) * np.uint64(2) + np.uint64(1)
    k = rng.integers(0, 2**63, size=(2, 64), dtype=np.uint64)
    out = philox4x64(c[0], c[1], c[2], c[3], k[0], k[1])
    for i in range(64):
        ref = philox4x64_ref([int(c[j, i]) for j in range(4)], [int(k[0, i]), int(k[1, i])])
        assert tuple(int(o[i]) for o in out) == ref


@pytest.mark.parametrize("L", list(range(1, 17)) + [20])
def test_feistel_is_a_bijection(L):
    x = np.arange(1 << L, dtype=np.uint64)
    y = feistel_forward(x, L, 1234, STREAM_PI)
    assert y.max() < (1 << L)
    assert np.unique(y).size == 1 << L
    assert np.array_equal(feistel_inverse(y, L, 1234, STREAM_PI), x)


def test_feistel_depends_on_seed_and_stream():
    x = np.arange(4096, dtype=np.uint64)
    a = feistel_forward(x, 12, 1, STREAM_PI)
    b = feistel_forward(x, 12, 2, STREAM_PI)
    c = feistel_forward(x, 12, 1, STREAM_PIHAT)
    assert (a != b).mean() > 0.99 and (a != c).mean() > 0.99


def test_nested_sets_are_prefixes_of_distinct_rows():
    L = 15
    big = slot_rows(7, L, 12800)
    for m in (200, 400, 800, 1600, 3200, 6400):
        assert np.array_equal(slot_rows(7, L, m), big[:m])
    assert np.unique(big).size == big.size
    assert hat_slot_rows(7, L, 300).size == 300


def test_sampled_rows_look_uniform():
    # chi-square over 64 bins of the first 2^14 sampled rows of a 2^20 domain
    L = 20
    t = slot_rows(11, L, 1 << 14)
    counts = np.bincount(t >> (L - 6), minlength=64)
    exp = t.size / 64
    chi2 = ((counts - exp) ** 2 / exp).sum()
    assert chi2 < 120  # 63 dof: P(chi2 > 120) ~ 2e-5


def test_sign_vector_balance_and_packing():
    L = 16
    s = sign_vector(3, L)
    assert set(np.unique(s)) == {-1.0, 1.0}
    frac = (s < 0).mean()
    assert abs(frac - 0.5) < 5 * 0.5 / np.sqrt(s.size)
    # the sign of a subset of rows equals the full vector at those rows
    rows = np.array([0, 1, 255, 256, 257, 40000, 65535])
    assert np.array_equal(sign_vector(3, L, rows), s[rows])
    # bit j of word w of block b decides row 256 b + 64 w + j
    w = philox4x64(np.uint64(156), 0, 0, 0, np.uint64(3), np.uint64(1))
    row = 156 * 256 + 2 * 64 + 17
    bit = (int(w[2]) >> 17) & 1
    assert s[row] == (-1.0 if bit else 1.0)


def test_input_perm_is_a_permutation():
    p = input_perm(9, 12)
    assert np.array_equal(np.sort(p), np.arange(4096))


def test_padded_bits():
    assert padded_bits(1) == (1, 2)
    assert padded_bits(2) == (1, 2)
    assert padded_bits(3) == (2, 4)
    assert padded_bits(20000) == (15, 32768)
    assert padded_bits(1 << 20) == (20, 1 << 20)
    assert padded_bits(4_000_000) == (22, 1 << 22)
