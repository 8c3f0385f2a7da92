"""Pins of the oracle's rounding, border and random-number primitives.

Each check compares the oracle with something other than itself: exact
rational arithmetic (fractions), numpy's own reflect padding, and numpy's
Philox4x64-10 bit generator.
"""
from fractions import Fraction

import numpy as np
import pytest

import oracle


def round_half_even(fr: Fraction) -> int:
    fl = fr.numerator // fr.denominator
    rem = fr - fl
    if rem > Fraction(1, 2) or (rem == Fraction(1, 2) and fl % 2 == 1):
        return fl + 1
    return fl


def test_rdiv_he_matches_exact_rational_rounding():
    rng = np.random.default_rng(1)
    cases = [(n, d) for n in range(-40, 41) for d in (1, 2, 3, 4, 7, 16, 1024)]
    cases += [(int(rng.integers(-2**40, 2**40)), int(rng.integers(1, 2**20))) for _ in range(3000)]
    for n, d in cases:
        assert oracle.rdiv_he(n, d) == round_half_even(Fraction(n, d)), (n, d)


def test_rdiv_he_ties_go_to_even_including_negative_numerators():
    assert [oracle.rdiv_he(n, 2) for n in (-5, -3, -1, 1, 3, 5)] == [-2, -2, 0, 0, 2, 2]
    assert oracle.rshr_he(-512, 10) == 0 and oracle.rshr_he(-1536, 10) == -2 and oracle.rshr_he(1536, 10) == 2


@pytest.mark.parametrize("n", [1, 2, 3, 5, 8])
def test_reflect101_matches_numpy_reflect_padding(n):
    if n == 1:
        assert all(oracle.reflect101(i, 1) == 0 for i in range(-5, 6))
        return
    pad = 4 * n
    ref = np.pad(np.arange(n), pad, mode="reflect")  # numpy 'reflect' does not repeat the edge
    for k, i in enumerate(range(-pad, n + pad)):
        assert oracle.reflect101(i, n) == ref[k], (i, n)


def test_philox_matches_numpy_bit_generator():
    # numpy's Philox increments the 256-bit counter before each block, so a
    # generator started at counter c - 1 yields the block of counter c.
    rng = np.random.default_rng(7)
    for _ in range(50):
        key = [int(x) for x in rng.integers(0, 2**63, size=2, dtype=np.uint64)]
        ctr = [int(x) for x in rng.integers(1, 2**63, size=4, dtype=np.uint64)]
        prev = list(ctr)
        prev[0] -= 1
        g = np.random.Philox(counter=prev, key=key)
        expect = g.random_raw(4)
        got = oracle.philox4x64_10(ctr, key)
        assert [int(x) for x in got] == [int(x) for x in expect]


def test_draw_is_word0_of_the_stream_block():
    seed, stream, index, draw = 1809068391, 0, 17, 3
    g = np.random.Philox(counter=[draw - 1, index, 0, stream], key=[seed, 0])
    assert oracle.draw_u64(seed, stream, index, draw) == int(g.random_raw(4)[0])


def test_noise16_unpacks_16_bit_words_of_the_noise_stream():
    seed, index, field = 5, 3, 1
    for e in (0, 1, 5, 15, 16, 31, 12345):
        blk = e // 16
        if blk > 0:
            prev = [blk - 1, index, field, 4]
        else:  # counter word 0 == 0: borrow through the 256-bit counter
            prev = [2**64 - 1, index - 1, field, 4]
        g = np.random.Philox(counter=np.array(prev, dtype=np.uint64), key=np.array([seed, 0], dtype=np.uint64))
        words = g.random_raw(4)
        w = int(words[(e % 16) // 4])
        expect = ((w >> (16 * (e % 4))) & 0xFFFF) - 32768
        assert oracle.noise16(seed, index, field, e) == expect


def test_sampler_ranges_and_frequencies():
    flags, ab = oracle.sample_d4bc(1809068391, 0, 20000)
    for j in (0, 1, 3):
        assert set(np.unique(flags[:, j])) == {0, 1}
        assert abs(flags[:, j].mean() - 0.5) < 0.02
    assert set(np.unique(flags[:, 2])) == {0, 1, 2, 3}
    assert np.all(np.abs(np.bincount(flags[:, 2]) / 20000 - 0.25) < 0.02)
    assert ab[:, 0].min() >= 0.8 and ab[:, 0].max() <= 1.2
    assert ab[:, 1].min() >= -51 and ab[:, 1].max() <= 51
    from scipy import stats
    assert stats.kstest((ab[:, 0] - 0.8) / 0.4, "uniform").pvalue > 1e-4
    assert stats.kstest((ab[:, 1] + 51) / 102, "uniform").pvalue > 1e-4
    # draws are independent of batch composition (counter-based)
    f2, ab2 = oracle.sample_d4bc(1809068391, 137, 10)
    assert np.array_equal(f2, flags[137:147]) and np.array_equal(ab2, ab[137:147])


def test_sampler_c2_ranges():
    f, k = oracle.sample_c2(1809068392, 0, 20000)
    assert f[:, 0].min() >= -45 and f[:, 0].max() <= 45
    assert f[:, 1].min() >= 0.9 and f[:, 1].max() <= 1.1
    assert np.abs(f[:, 2:4]).max() <= 0.0625
    assert k[:, 0].min() == 0 and k[:, 0].max() == 64 and k[:, 1].max() == 64
    assert k[:, 2].min() == -20 and k[:, 2].max() == 20
    assert k[:, 3].min() == -30 and k[:, 3].max() == 30
    assert abs(k[:, 4].mean() - 0.3) < 0.02
    assert f[:, 4].min() >= 0.8 and f[:, 4].max() <= 1.2


def test_sampler_wc_and_grid_ranges():
    f = oracle.sample_wc(1809068394, 0, 5000)
    lo = [-45, 0.9, -0.0625, -0.0625, 0.8, -0.2, 0.8]
    hi = [45, 1.1, 0.0625, 0.0625, 1.2, 0.2, 1.2]
    assert np.all(f.min(0) >= lo) and np.all(f.max(0) <= hi)
    g = oracle.sample_grid(1809068395, 0, 5000)
    assert g.min() >= 0.7 and g.max() <= 1.3
