"""Correctly rounded exp, log, log1p, pow and u^(1/a): the functions of the
bitexact setting (Section 4.2, exact reproducibility across platforms).

The oracle's functions (binary128 through libquadmath, rounded once to
binary64) are pinned to Python's decimal module at 60 significant digits:
decimal's exp and ln are correctly rounded at the context precision, and
float() of a decimal rounds correctly, so the reference is the correctly
rounded binary64 value unless the exact result lies within about 10^-60
relative of a rounding boundary.  The library's host build (rp_crmath_host)
must then equal the oracle bit for bit on random arguments over the whole
range and on the edges: overflow and underflow thresholds, subnormal
results, arguments next to 1 and to -1, and the special values of C99
Annex F (F.9.4.4 for pow), written out below from the standard.
"""
from decimal import Decimal, getcontext
import math

import numpy as np
import pytest

import oracle
import paper_2605_05099_amd as rp

getcontext().prec = 60
INF, NAN = math.inf, math.nan
FNS = {"exp": (rp.RP_CR_EXP, oracle.CR_EXP), "log": (rp.RP_CR_LOG, oracle.CR_LOG),
       "log1p": (rp.RP_CR_LOG1P, oracle.CR_LOG1P), "pow": (rp.RP_CR_POW, oracle.CR_POW),
       "powinv": (rp.RP_CR_POWINV, oracle.CR_POWINV)}


def _dec(fn, x, y):
    x = Decimal(float(x))
    if fn == "exp":
        return float(x.exp())
    if fn == "log":
        return float(x.ln())
    if fn == "log1p":
        if abs(x) < Decimal("1e-3"):  # the series: 1 + x would lose x's digits
            s, t, k = Decimal(0), x, 1
            while t != 0 and abs(t) > abs(x) * Decimal("1e-70"):
                s += t / k
                k += 1
                t = -t * x
            return float(s)
        return float((1 + x).ln())
    if fn == "pow":
        return float((Decimal(float(y)) * x.ln()).exp())
    return float((x.ln() / Decimal(float(y))).exp())


def _args(fn, n, seed):
    """Arguments spread over the range of fn, with its edges."""
    g = np.random.default_rng(seed)
    if fn == "exp":
        x = np.concatenate([g.uniform(-745.1, 709.78, n), g.uniform(-1, 1, n), g.uniform(-2**-20, 2**-20, n // 4),
                            g.uniform(-745.13, -708.3, n // 2),       # subnormal results
                            709.782712893384 - g.uniform(0, 1e-9, 20),  # next to the overflow threshold
                            np.array([-745.1332191019411, -745.1332191019412, -744.44007192138126,
                                      -708.39641853226408, -708.39641853226419, 2.0**-54, -2.0**-54,
                                      2.0**-53, -2.0**-53, 1e-300, -1e-300, 5e-324])])
        return x, None
    if fn == "log":
        x = np.concatenate([np.exp(g.uniform(-744, 709, n)), g.uniform(0.5, 2.0, n),
                            1 + g.integers(-2**20, 2**20, n // 4) * 2.0**-52,
                            g.uniform(0, 2.2e-308, n // 8),           # subnormal arguments
                            np.array([5e-324, 2.2250738585072014e-308, 1.7976931348623157e308,
                                      0.9999999999999999, 1.0000000000000002, 2.0, 0.5, math.e])])
        return x, None
    if fn == "log1p":
        x = np.concatenate([g.uniform(-0.999, 20, n), g.uniform(-2**-7, 2**-7, n),
                            np.exp(g.uniform(-700, 700, n // 2)), -1 + np.exp(g.uniform(-36, -1e-3, n // 2)),
                            np.array([2.0**-54, -2.0**-54, 2.0**-53, -2.0**-53, 2.0**-7, -2.0**-7,
                                      -0.9999999999999999, 1e-310, -1e-310, 1.7976931348623157e308])])
        return x, None
    if fn == "pow":
        x = np.concatenate([np.exp(g.uniform(-30, 30, n)), g.uniform(0, 1, n), g.uniform(0.9, 1.1, n // 4),
                            np.exp(g.uniform(-700, 700, n // 4))])
        y = np.concatenate([g.uniform(-40, 40, n), g.uniform(0.05, 12, n), g.uniform(-3000, 3000, n // 4),
                            g.uniform(-1.5, 1.5, n // 4)])
        return x, y
    u = np.concatenate([g.uniform(0, 1, n), np.exp(g.uniform(-700, 0, n // 2)), g.integers(1, 2**53, n // 2) * 2.0**-53])
    a = np.concatenate([g.uniform(0.005, 1, n), g.uniform(0.05, 0.999, n // 2), g.uniform(0.001, 0.2, n // 2)])
    return u, a


def _same(a, b):
    a, b = np.asarray(a, dtype=np.float64), np.asarray(b, dtype=np.float64)
    return (a.view(np.int64) == b.view(np.int64)) | (np.isnan(a) & np.isnan(b))


@pytest.mark.parametrize("fn", list(FNS))
def test_oracle_crmath_is_correctly_rounded(fn):
    x, y = _args(fn, 600, 11)
    got = oracle.crmath(FNS[fn][1], x, y)
    ref = np.array([_dec(fn, x[i], None if y is None else y[i]) for i in range(len(x))])
    bad = ~_same(got, ref)
    assert not bad.any(), (fn, x[bad][:3], got[bad][:3], ref[bad][:3])


@pytest.mark.parametrize("fn", list(FNS))
def test_library_host_functions_equal_the_oracle(fn):
    x, y = _args(fn, 60000, 12)
    got = rp.rp_crmath_host(FNS[fn][0], x, y)
    ref = oracle.crmath(FNS[fn][1], x, y)
    bad = ~_same(got, ref)
    assert not bad.any(), (fn, int(bad.sum()), x[bad][:3], got[bad][:3], ref[bad][:3])


def test_library_functions_on_decimal_references():
    """The library directly against decimal on a small set (independent of the
    oracle's libquadmath)."""
    for fn, (code, _) in FNS.items():
        x, y = _args(fn, 150, 13)
        got = rp.rp_crmath_host(code, x, y)
        ref = np.array([_dec(fn, x[i], None if y is None else y[i]) for i in range(len(x))])
        assert _same(got, ref).all(), fn


def test_special_values():
    # exp, log, log1p (C99 F.9.3)
    cases = [
        ("exp", 0.0, None, 1.0), ("exp", -0.0, None, 1.0), ("exp", INF, None, INF), ("exp", -INF, None, 0.0),
        ("exp", NAN, None, NAN), ("exp", 710.0, None, INF), ("exp", -746.0, None, 0.0),
        ("exp", 1e-320, None, 1.0),
        ("log", 1.0, None, 0.0), ("log", 0.0, None, -INF), ("log", -0.0, None, -INF), ("log", -1.0, None, NAN),
        ("log", INF, None, INF), ("log", NAN, None, NAN), ("log", -INF, None, NAN),
        ("log1p", 0.0, None, 0.0), ("log1p", -0.0, None, -0.0), ("log1p", -1.0, None, -INF),
        ("log1p", -2.0, None, NAN), ("log1p", INF, None, INF), ("log1p", NAN, None, NAN), ("log1p", 5e-324, None, 5e-324),
        # pow (F.9.4.4)
        ("pow", 0.0, -3.0, INF), ("pow", -0.0, -3.0, -INF), ("pow", 0.0, -2.0, INF), ("pow", -0.0, -0.5, INF),
        ("pow", 0.0, -INF, INF), ("pow", 0.0, 3.0, 0.0), ("pow", -0.0, 3.0, -0.0), ("pow", -0.0, 2.0, 0.0),
        ("pow", -0.0, 0.5, 0.0), ("pow", -1.0, INF, 1.0), ("pow", -1.0, -INF, 1.0), ("pow", 1.0, NAN, 1.0),
        ("pow", 1.0, INF, 1.0), ("pow", NAN, 0.0, 1.0), ("pow", NAN, -0.0, 1.0), ("pow", -2.0, 0.5, NAN),
        ("pow", 0.5, -INF, INF), ("pow", 2.0, -INF, 0.0), ("pow", 0.5, INF, 0.0), ("pow", 2.0, INF, INF),
        ("pow", -INF, -3.0, -0.0), ("pow", -INF, -2.0, 0.0), ("pow", -INF, 3.0, -INF), ("pow", -INF, 2.0, INF),
        ("pow", INF, -1.0, 0.0), ("pow", INF, 2.5, INF), ("pow", -2.0, 3.0, -8.0), ("pow", -2.0, -2.0, 0.25),
        ("pow", 2.0, 1024.0, INF), ("pow", 2.0, -1074.0, 5e-324), ("pow", 2.0, -1075.0, 0.0), ("pow", NAN, 1.0, NAN),
        ("pow", 4.0, 0.5, 2.0), ("pow", 3.0, 3.0, 27.0), ("pow", 10.0, -1.0, 0.1),
        ("powinv", 0.0, 0.3, 0.0), ("powinv", 1.0, 0.3, 1.0), ("powinv", 0.25, 0.5, 0.0625), ("powinv", -1.0, 0.5, NAN),
        ("powinv", 0.5, 0.0, NAN), ("powinv", 0.5, INF, 1.0),
    ]
    for fn, x, y, want in cases:
        got = rp.rp_crmath_host(FNS[fn][0], [x], None if y is None else [y])[0]
        assert _same(got, want), (fn, x, y, got, want)
        got = oracle.crmath(FNS[fn][1], [x], None if y is None else [y])[0]
        assert _same(got, want) or fn == "powinv", ("oracle", fn, x, y, got, want)


def test_crmath_errors():
    x = np.zeros(4)
    with pytest.raises(rp.RpError) as ei:
        rp.rp_crmath_host(7, x)
    assert ei.value.code == rp.RP_EINVAL
    with pytest.raises(rp.RpError) as ei:
        rp.rp_crmath_host(rp.RP_CR_POW, x)  # y missing
    assert ei.value.code == rp.RP_ENULL
