"""Pins of the oracle's float ziggurat (normf, expf).

The paper gives binary32 versions of its continuous laws and says only that
the float case is analogous to the double one.  The reading taken: a float
draw consumes 32-bit items (low half first), with a 23-bit (normal) or 24-bit
(exponential) magnitude in the double ziggurat's geometry and 24-bit wedge
and tail uniforms, rounded once to binary32.  These tests pin it against the
mathematics: the exact laws (KS, moments), the tail mass and the conditional
tail laws, and the items consumed per value, which must equal the double
sampler's words per value (the same geometry; the paper's figures 1.022 and
1.034 for normal and exponential draws).
"""
import math

import numpy as np
import pytest
from scipy import stats

from oracle import Stream

R_NORM = 3.6541528853610088
R_EXP = 7.69711747013105


@pytest.mark.parametrize("eng", ["philox4x32", "x256++", "pcg64"])
def test_normf_ks_and_moments(eng):
    x = Stream.seeded(eng, 21).normf(400000)
    assert x.dtype == np.float32
    assert stats.kstest(x.astype(np.float64), "norm").pvalue > 1e-4
    n = len(x)
    xd = x.astype(np.float64)
    assert abs(xd.mean()) < 5 / math.sqrt(n)
    assert abs(xd.var() - 1) < 6 * math.sqrt(2 / n)
    assert abs(stats.skew(xd)) < 6 * math.sqrt(6 / n)
    assert abs(stats.kurtosis(xd)) < 6 * math.sqrt(24 / n)


@pytest.mark.parametrize("eng", ["philox4x32", "sfc64"])
def test_expf_ks_and_moments(eng):
    x = Stream.seeded(eng, 22).expf(400000).astype(np.float64)
    assert stats.kstest(x, "expon").pvalue > 1e-4
    assert x.min() >= 0
    n = len(x)
    assert abs(x.mean() - 1) < 5 / math.sqrt(n)
    assert abs(x.var() - 1) < 6 * math.sqrt(8 / n)


def test_float_tails():
    """Tail mass P(|Z| > r) = 2 Phi(-r) and P(E > r) = e^-r, and the tail
    values follow the laws conditioned on the tail (Marsaglia's normal tail,
    the exponential's memorylessness)."""
    n = 6_000_000
    x = Stream.seeded("philox4x32", 23).normf(n).astype(np.float64)
    t = np.abs(x[np.abs(x) > R_NORM])
    p = 2 * stats.norm.sf(R_NORM)
    assert abs(len(t) - n * p) < 5 * math.sqrt(n * p)
    cdf = lambda v: 1 - stats.norm.sf(v) / stats.norm.sf(R_NORM)
    assert stats.kstest(t, cdf).pvalue > 1e-4
    e = Stream.seeded("philox4x32", 24).expf(n).astype(np.float64)
    te = e[e > R_EXP] - R_EXP
    pe = math.exp(-R_EXP)
    assert abs(len(te) - n * pe) < 5 * math.sqrt(n * pe)
    # binary32 rounding of r + E' moves values by < 2^-20; far below the KS resolution here
    assert stats.kstest(te, "expon").pvalue > 1e-4


def _words_used(s0, s1):
    """Philox4x32-10 words between two states (counter of 2-word blocks + phase)."""
    c0 = s0.state[0] | (s0.state[1] << 64)
    c1 = s1.state[0] | (s1.state[1] << 64)
    return 2 * (c1 - c0) + s1.phase - s0.phase


def test_float_items_per_value():
    """Items per value equal the double sampler's words per value: one item
    per candidate, one per wedge test, two per normal tail pair, one for the
    exponential tail."""
    n = 4_000_000
    for meth, ref in (("normf", 1.0220), ("expf", 1.0336)):
        s = Stream.seeded("philox4x32", 25)
        s0 = s.copy()
        getattr(s, meth)(n)
        items = 2 * _words_used(s0, s)  # a dropped high half counts once at most
        assert abs(items / n - ref) < 0.001, (meth, items / n)


def test_float_symmetry_and_range():
    x = Stream.seeded("pcg64", 26).normf(1_000_000)
    pos = int((x > 0).sum())
    assert abs(pos - 500000) < 5 * math.sqrt(250000)
    assert np.isfinite(x).all() and np.abs(x).max() < 8
    e = Stream.seeded("pcg64", 27).expf(1_000_000)
    assert (e >= 0).all() and np.isfinite(e).all() and e.max() < 30


def test_float_halves_are_consumed_in_order():
    """A float draw uses the low half of a word first: after one fast-accepted
    value the stream sits in the middle of its first word, and the next call
    drops the high half (a call never keeps a half for the next one)."""
    s = Stream.seeded("philox4x32", 28)
    s0 = s.copy()
    s.normf(1)
    assert _words_used(s0, s) == 1
    a = Stream.seeded("philox4x32", 28)
    b = Stream.seeded("philox4x32", 28)
    x2 = a.normf(2)
    y1 = b.normf(1)
    assert x2[0] == y1[0]
    assert _words_used(s0, b) == 1
