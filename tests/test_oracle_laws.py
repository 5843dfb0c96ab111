"""Pins of the derived laws' oracle (CPU only): each transform of Table 4,
applied to the oracle's own base draws, must give the law it names -- a
Kolmogorov-Smirnov test against SciPy's distribution with the paper's
parameterization (a swapped parameter, a wrong sign or a scale taken as a
rate fails it) -- and the special cases that reduce to another law must."""
import numpy as np
import pytest
from scipy import stats

import oracle
from oracle import laws

N = 20000

CASES = [
    (laws.UNIF, (-2.0, 5.0), stats.uniform(loc=-2.0, scale=7.0)),
    (laws.NORMAL, (3.0, 5.0), stats.norm(loc=3.0, scale=5.0)),
    (laws.LOGNORMAL, (0.5, 0.75), stats.lognorm(s=0.75, scale=np.exp(0.5))),
    (laws.EXP, (2.5,), stats.expon(scale=2.5)),
    (laws.GUMBEL, (1.0, 2.0), stats.gumbel_r(loc=1.0, scale=2.0)),
    (laws.PARETO, (1.5, 3.0), stats.pareto(b=3.0, scale=1.5)),
    (laws.GPARETO, (0.5, 2.0, 0.3), stats.genpareto(c=0.3, loc=0.5, scale=2.0)),
    (laws.GPARETO, (0.5, 2.0, -0.4), stats.genpareto(c=-0.4, loc=0.5, scale=2.0)),
    (laws.GPARETO, (0.5, 2.0, 0.0), stats.genpareto(c=0.0, loc=0.5, scale=2.0)),
    (laws.WEIBULL, (1.7, 4.0), stats.weibull_min(c=1.7, scale=4.0)),
    (laws.GAMMA, (2.5, 1.5), stats.gamma(a=2.5, scale=1.5)),
    (laws.GAMMA, (0.4, 3.0), stats.gamma(a=0.4, scale=3.0)),
    (laws.BETA, (2.0, 5.0), stats.beta(2.0, 5.0)),
    (laws.CHI2, (3.0,), stats.chi2(df=3.0)),
    (laws.CHI2, (0.8,), stats.chi2(df=0.8)),
    (laws.T, (4.5,), stats.t(df=4.5)),
    (laws.F, (5.0, 7.0), stats.f(dfn=5.0, dfd=7.0)),
    (laws.SKEWNORMAL, (1.0, 2.0, 3.0), stats.skewnorm(a=3.0, loc=1.0, scale=2.0)),
    (laws.SKEWNORMAL, (0.0, 1.0, -1.5), stats.skewnorm(a=-1.5, loc=0.0, scale=1.0)),
]


@pytest.mark.parametrize("law,p,dist", CASES, ids=lambda c: str(c) if not hasattr(c, "cdf") else "")
def test_law_matches_its_distribution(law, p, dist):
    s = oracle.Stream.seeded("x256++", 1000 + law)
    x = laws.draw(s, law, p, N if law not in (laws.T, laws.F) else N // 4)
    assert np.isfinite(x).all()
    assert stats.kstest(x, dist.cdf).pvalue > 1e-3


def test_special_cases():
    s = oracle.Stream.seeded("pcg64", 5)
    base = s.copy().exp(1000)
    # Weibull with k = 1 and Exp(beta) are beta E; Pareto(1, alpha) is exp(E / alpha)
    assert np.array_equal(laws.transform(laws.WEIBULL, base, (1.0, 2.5)), 2.5 * base ** 1.0)
    assert np.array_equal(laws.transform(laws.EXP, base, (2.5,)), 2.5 * base)
    # generalized Pareto with xi > 0 at mu = 0, s = xi: P - 1
    P = laws.transform(laws.PARETO, base, (1.0, 1.0 / 0.5))
    np.testing.assert_allclose(laws.transform(laws.GPARETO, base, (0.0, 0.5, 0.5)), P - 1.0, rtol=1e-12)
    # Gumbel at u = exp(-1) is mu; normal and lognormal are exp-related
    assert laws.transform(laws.GUMBEL, [np.exp(-1.0)], (3.0, 2.0))[0] == pytest.approx(3.0, abs=1e-15)
    z = oracle.Stream.seeded("x256++", 9).norm(1000)
    np.testing.assert_allclose(np.log(laws.transform(laws.LOGNORMAL, z, (0.3, 1.2))),
                               laws.transform(laws.NORMAL, z, (0.3, 1.2)), rtol=1e-13, atol=1e-13)


def test_draw_advances_like_the_base_fill():
    a = oracle.Stream.seeded("philox4x32", 3)
    b = a.copy()
    laws.draw(a, laws.PARETO, (1.0, 2.0), 777)
    b.exp(777)
    assert a.state == b.state and a.phase == b.phase


@pytest.mark.parametrize("law,p,dist", [
    (laws.LOGNORMAL, (0.5, 0.75), lambda: stats.lognorm(s=0.75, scale=np.exp(0.5))),
    (laws.WEIBULL, (1.7, 4.0), lambda: stats.weibull_min(c=1.7, scale=4.0)),
    (laws.GUMBEL, (1.0, 2.0), lambda: stats.gumbel_r(loc=1.0, scale=2.0)),
])
def test_float_laws_ks(law, p, dist):
    """Binary32 laws (float base draws, binary64 transform, one rounding)
    follow the named law."""
    x = laws.draw_f32(oracle.Stream.seeded("pcg64", 41), law, p, 200000)
    assert x.dtype == np.float32
    assert stats.kstest(x.astype(np.float64), dist().cdf).pvalue > 1e-4



@pytest.mark.parametrize("alpha", [2.5, 0.4])
def test_float_gamma_ks_and_mean(alpha):
    """The float gamma follows Gamma(alpha, theta)."""
    x = oracle.Stream.seeded("x256++", 43).gammaf(alpha, 200000, 1.5).astype(np.float64)
    assert stats.kstest(x, stats.gamma(alpha, scale=1.5).cdf).pvalue > 1e-4
    assert abs(x.mean() - 1.5 * alpha) < 6 * 1.5 * np.sqrt(alpha / len(x))


@pytest.mark.parametrize("law,p,dist", [c for c in CASES if c[0] in (laws.BETA, laws.CHI2, laws.T, laws.F,
                                                                      laws.SKEWNORMAL)],
                         ids=lambda c: str(c) if not hasattr(c, "cdf") else "")
def test_float_mix_laws_ks(law, p, dist):
    """The binary32 laws of several draws (float gammas and binary32
    normals, binary64 combination, one rounding) follow the named law (a
    swapped parameter or a wrong combination fails the KS test)."""
    x = laws.draw_f32(oracle.Stream.seeded("x256++", 2000 + law), law, p, N if law not in (laws.T, laws.F) else N // 2)
    assert x.dtype == np.float32
    assert np.isfinite(x).all()
    assert stats.kstest(x.astype(np.float64), dist.cdf).pvalue > 1e-3


def test_float_mix_laws_reduce_to_the_float_gamma():
    """chi2(nu) in binary32 is 2 G(nu / 2) of the float gamma on the same
    items, and t and F advance the stream as their draws say."""
    a = oracle.Stream.seeded("pcg64", 77)
    b = a.copy()
    x = laws.draw_f32(a, laws.CHI2, (3.0,), 500)
    y = b.gammaf(1.5, 500, 2.0)
    assert np.array_equal(x, y)
    assert a.state == b.state
