"""Pins of the CPU side of the serving workload's counter-based operands
(oracle/synthetic.py): the generator against its published known-answer
vectors, the element layout against hand-derived values, and the value
distribution against its closed-form moments and bounds."""
import json
import math
import os
from fractions import Fraction

import numpy as np
import pytest

from oracle import synthetic as S

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "philox4x32_10_kat.json")


def _kat():
    return json.load(open(GOLDEN))["vectors"]


def _block(gen, counter, key):
    out = gen(*[np.array([int(x, 16)], dtype=np.uint32) for x in counter], int(key[0], 16), int(key[1], 16))
    return [f"{int(o[0]):08x}" for o in out]


@pytest.mark.parametrize("vec", _kat())
def test_philox_known_answers(vec):
    assert _block(S.philox4x32_10, vec["counter"], vec["key"]) == vec["output"]


def _planted(kind):
    """Copies of the generator with one plausible mistake each."""
    def gen(c0, c1, c2, c3, k0, k1):
        c0, c1, c2, c3 = (np.asarray(x, dtype=np.uint32) for x in (c0, c1, c2, c3))
        rounds = 9 if kind == "nine_rounds" else 10
        m0, m1 = (S.PHILOX_M1, S.PHILOX_M0) if kind == "swapped_multipliers" else (S.PHILOX_M0, S.PHILOX_M1)
        for r in range(rounds):
            if r and kind != "no_key_bump":
                k0 = (k0 + S.PHILOX_W0) & S.MASK32
                k1 = (k1 + S.PHILOX_W1) & S.MASK32
            hi0, lo0 = S._mulhilo(m0, c0)
            hi1, lo1 = S._mulhilo(m1, c2)
            if kind == "swapped_outputs":
                c0, c1, c2, c3 = hi0 ^ c1 ^ np.uint32(k0), lo0, hi1 ^ c3 ^ np.uint32(k1), lo1
            else:
                c0, c1, c2, c3 = hi1 ^ c1 ^ np.uint32(k0), lo1, hi0 ^ c3 ^ np.uint32(k1), lo0
        return c0, c1, c2, c3
    return gen


@pytest.mark.parametrize("kind", ["nine_rounds", "swapped_multipliers", "no_key_bump", "swapped_outputs"])
def test_planted_generator_mistakes_fail_the_known_answers(kind):
    gen = _planted(kind)
    assert any(_block(gen, v["counter"], v["key"]) != v["output"] for v in _kat())


def test_scale_constant_is_the_nearest_fp32_to_sqrt3_over_2_17():
    c = Fraction(float(S.SCALE))
    # sqrt(3) * 2^-17 lies within half an FP32 ulp of c: compare squares exactly
    ulp = Fraction(2) ** (math.frexp(float(S.SCALE))[1] - 24)
    lo, hi = (c - ulp / 2) * 2 ** 17, (c + ulp / 2) * 2 ** 17
    assert lo * lo < 3 < hi * hi


def test_first_elements_from_the_zero_key_block():
    # seed 0, operand A (tag 0): pair 0 is the counter-0 / key-0 block, whose
    # words are the first known-answer vector: 6627e8d5 e169c58d | bc57ac4c 9b00dbd8
    halves = [[0x6627, 0xE8D5, 0xE169, 0xC58D], [0xBC57, 0xAC4C, 0x9B00, 0xDBD8]]
    got = S.synthetic_elements([0, 1], seed=0, tag=0)
    for g, h in zip(got, halves):
        x = 2 * sum(h) - 4 * 65535
        assert float(g) == float(np.float32(np.float32(x) * S.SCALE))
        assert abs(float(g) - x * math.sqrt(3) / 2 ** 17) <= 2.0 ** -22 * abs(float(g))


def test_layout_counter_key_and_pairs():
    idx = np.array([0, 1, 2, 3, 2 ** 33 + 4, 2 ** 33 + 5], dtype=np.int64)
    seed = 0x0123456789ABCDEF
    for tag in (0, 1):
        got = S.synthetic_elements(idx, seed, tag)
        for e, g in zip(idx, got):
            q = int(e) // 2
            w = S.philox4x32_10([q & S.MASK32], [q >> 32], [tag], [0], seed & S.MASK32, seed >> 32)
            ws = (w[0][0], w[1][0]) if e % 2 == 0 else (w[2][0], w[3][0])
            s = sum(int(x) & 0xFFFF for x in ws) + sum(int(x) >> 16 for x in ws)
            assert g == np.float32(np.float32(2 * s - 4 * 65535) * S.SCALE)
    assert not np.array_equal(S.synthetic_elements(idx, seed, 0), S.synthetic_elements(idx, seed, 1))
    assert not np.array_equal(S.synthetic_elements(idx, seed, 0), S.synthetic_elements(idx, seed + 1, 0))


def test_operand_rows_are_slices_of_the_flat_stream():
    full = S.synthetic_operand(37, 53, seed=9, tag=1)
    assert full.dtype == np.float32 and full.shape == (37, 53)
    assert np.array_equal(full.ravel(), S.synthetic_elements(np.arange(37 * 53), 9, 1))
    rows = [36, 0, 17]
    assert np.array_equal(S.synthetic_operand(37, 53, seed=9, tag=1, row_index=rows), full[rows])


def test_distribution_moments_and_bounds():
    x = S.synthetic_elements(np.arange(1 << 20), seed=5, tag=0).astype(np.float64)
    n = x.size
    # 2 S - 4 * 65535 with S the sum of four independent uniform integers in
    # [0, 65535]: mean 0, variance 16 (65536^2 - 1) / 12; times c^2 = 3 / 2^34
    # that is 1 - 2^-32; excess kurtosis of a sum of four uniforms: -6/5 / 4
    assert abs(x.mean()) < 5.0 / math.sqrt(n)
    assert abs(x.var() - 1.0) < 5.0 * math.sqrt(1.7 / n)
    k = ((x - x.mean()) ** 4).mean() / x.var() ** 2 - 3.0
    assert abs(k + 0.3) < 0.03
    bound = 4 * 65535 * float(S.SCALE) * 2 / 2
    assert np.abs(x).max() <= bound * (1 + 2 ** -23)
    # symmetric about 0: the sum S and 4*65535 - S are equally likely
    assert abs((x > 0).mean() - (x < 0).mean()) < 5.0 / math.sqrt(n)
