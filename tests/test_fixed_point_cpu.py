"""The fixed-point arithmetic of the deterministic weight sums, on the host.

cf_fixed_sum runs the same limb split, int64 limb sums, 192-bit assembly and
single rounding (pc_fixed.h) as the sweep's deterministic weight sums.  Here
it is checked against two references that share nothing with it: Python's
math.fsum (the exact sum, rounded once to nearest-even) and the exact
rational sum converted by float(Fraction) -- on float32 products, full 53-bit
values, mixed signs, exact cancellation, ties to even, sums that cross the
64- and 128-bit words, and values off the grid (refused).
"""
import math
from fractions import Fraction

import numpy as np
import pytest

import synth

pc = pytest.importorskip("paper_1911_03545_amd")


def exact(values):
    return float(sum((Fraction(float(v)) for v in values), Fraction(0)))


@pytest.fixture(scope="module")
def lib():
    try:
        return pc.load_library()
    except RuntimeError as e:
        pytest.skip(str(e))


def test_float32_products(lib):
    rng = synth.rng_for(801)
    a = synth.uniform_weights(50000, 802).astype(np.float64)
    b = synth.uniform_weights(50000, 803).astype(np.float64)
    p = a * b * np.where(rng.random(50000) < 0.3, -1.0, 1.0)   # exact products
    got = pc.fixed_sum(p, -48)
    assert got == math.fsum(p)
    assert pc.fixed_sum(p[:5000], -48) == exact(p[:5000])


def test_full_precision_values(lib):
    rng = synth.rng_for(804)
    p = np.exp2(rng.uniform(-10.0, 10.0, 20000))
    e_min = math.frexp(float(p.min()))[1] - 1
    q = e_min - 52
    got = pc.fixed_sum(p, q)
    assert got == math.fsum(p) == exact(p)


def test_cancellation_and_signs(lib):
    rng = synth.rng_for(805)
    p = np.exp2(rng.uniform(-4.0, 4.0, 3000))
    both = np.concatenate([p, -p])
    rng.shuffle(both)
    q = math.frexp(float(p.min()))[1] - 1 - 52
    assert pc.fixed_sum(both, q) == 0.0
    tail = np.concatenate([both, [2.0 ** q]])
    assert pc.fixed_sum(tail, q) == 2.0 ** q
    neg = -p
    assert pc.fixed_sum(neg, q) == math.fsum(neg) < 0


def test_ties_to_even(lib):
    two53 = 2.0 ** 53
    assert pc.fixed_sum([two53, 1.0], 0) == two53            # tie, even below
    assert pc.fixed_sum([two53, 3.0], 0) == two53 + 4.0      # tie, even above
    assert pc.fixed_sum([two53, 1.0, 2.0 ** -30], -30) == two53 + 2.0   # above the tie
    assert pc.fixed_sum([-two53, -1.0], 0) == -two53
    # ties far above the first word: 2^100 + 2^47 is halfway between
    # neighbours 2^100 and 2^100 + 2^48
    big = 2.0 ** 93
    vals = [big] * 128 + [2.0 ** 47]
    assert pc.fixed_sum(vals, 0) == 2.0 ** 100
    # 2^100 + 1.5 ulp: halfway between 2^100 + 2^48 (odd) and 2^100 + 2^49
    vals3 = vals + [2.0 ** 47, 2.0 ** 47]
    assert pc.fixed_sum(vals3, 0) == 2.0 ** 100 + 2.0 ** 49 == math.fsum(vals3)


def test_sums_across_words(lib):
    rng = synth.rng_for(806)
    # values up to 2^93 (just under the limit) with low bits set: the total
    # reaches past 2^104, the limbs carry into the second and third words
    hi = (rng.integers(1, 2 ** 40, 2000).astype(np.float64)) * 2.0 ** 53
    lo = rng.integers(1, 2 ** 20, 2000).astype(np.float64)
    p = np.concatenate([hi, lo, -hi[:700]])
    rng.shuffle(p)
    assert pc.fixed_sum(p, 0) == exact(p)
    assert pc.fixed_sum(p * 2.0 ** -60, -60) == exact(p * 2.0 ** -60)


def test_empty_and_grid_checks(lib):
    assert pc.fixed_sum([], 0) == 0.0
    with pytest.raises(pc.PairCountError):
        pc.fixed_sum([0.5], 0)                 # not a multiple of 2^0
    with pytest.raises(pc.PairCountError):
        pc.fixed_sum([2.0 ** 94], 0)           # beyond the limbs
    with pytest.raises(pc.PairCountError):
        pc.fixed_sum([1.0], -1023)             # grid below the normal range
    assert pc.fixed_sum([2.0 ** 94 - 2.0 ** 41], 0) == 2.0 ** 94 - 2.0 ** 41
