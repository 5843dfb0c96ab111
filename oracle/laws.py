"""Derived continuous laws by transform (Table 4 and Section 3.1) -- TEST
INFRASTRUCTURE ONLY: the oracle of rp_fill_law.

Each draw is one transform of one base draw of the oracle's streams, written
out as the paper gives it, in binary64 and in the order written:

  unif(a, b)          a + (b - a) U                      (shift-scale)
  normal(mu, sigma)   mu + sigma Z                       (shift-scale; sigma is
                                                          the standard deviation)
  lognormal(mu, s)    exp(mu + s Z)                      (exponential transform)
  exp(beta)           beta E                             (beta the scale)
  gumbel(mu, beta)    mu - beta log(-log U)              (inverse CDF)
  pareto(xm, alpha)   xm exp(E / alpha)
  gpareto(mu, s, xi)  P = Pareto(1, 1/|xi|) = exp(E / (1/|xi|));
                      xi > 0: mu + s (P - 1) / xi,  xi < 0: mu - s (1 - 1/P) / xi,
                      xi = 0: mu + s E               (a shifted Exp(s))
  weibull(k, lam)     lam E^(1/k)

U is the 53-bit uniform, Z and E the ziggurat normal and exponential of the
same stream (Stream.u01 / norm / exp).  Pinned against the laws themselves in
tests/test_oracle_laws.py.
"""
import numpy as np

UNIF, NORMAL, LOGNORMAL, EXP, GUMBEL, PARETO, GPARETO, WEIBULL = range(1, 9)
NPARAMS = {UNIF: 2, NORMAL: 2, LOGNORMAL: 2, EXP: 1, GUMBEL: 2, PARETO: 2, GPARETO: 3, WEIBULL: 2}
BASE = {UNIF: "u01", NORMAL: "norm", LOGNORMAL: "norm", EXP: "exp", GUMBEL: "u01", PARETO: "exp",
        GPARETO: "exp", WEIBULL: "exp"}


def transform(law, base, p):
    """The law's value for each base draw (a float64 array)."""
    x = np.asarray(base, dtype=np.float64)
    p = [float(v) for v in p]
    with np.errstate(divide="ignore", over="ignore", invalid="ignore"):
        if law == UNIF:
            a, b = p
            return a + (b - a) * x
        if law == NORMAL:
            mu, sigma = p
            return mu + sigma * x
        if law == LOGNORMAL:
            mu, sigma = p
            return np.exp(mu + sigma * x)
        if law == EXP:
            (beta,) = p
            return beta * x
        if law == GUMBEL:
            mu, beta = p
            return mu - beta * np.log(-np.log(x))
        if law == PARETO:
            xm, alpha = p
            return xm * np.exp(x / alpha)
        if law == GPARETO:
            mu, s, xi = p
            if xi == 0.0:
                return mu + s * x
            P = np.exp(x / (1.0 / abs(xi)))
            if xi > 0.0:
                return mu + (s * (P - 1.0)) / xi
            return mu - (s * (1.0 - 1.0 / P)) / xi
        if law == WEIBULL:
            k, lam = p
            return lam * np.power(x, 1.0 / k)
    raise ValueError(f"unknown law {law}")


def draw(stream, law, p, n):
    """n draws of the law from one oracle stream (advancing it)."""
    return transform(law, getattr(stream, BASE[law])(n), p)
