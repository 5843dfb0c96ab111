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
same stream (Stream.u01 / norm / exp).

Laws of several base draws per value, G(a) the Marsaglia-Tsang gamma draw of
the stream (Stream.gamma), drawn in the order written:

  gamma(alpha, theta)  theta G(alpha)
  beta(a, b)           X / (X + Y), X = G(a) then Y = G(b)    (Stream.beta)
  chi2(nu)             2 G(nu / 2)                (gamma, alpha = nu/2, theta = 2)
  t(nu)                Z / sqrt(V / nu), Z then V = 2 G(nu / 2)
  f(nu1, nu2)          (X / nu1) / (Y / nu2), X = G(nu1 / 2) then Y = G(nu2 / 2)
  skew_normal(mu, s, alpha)
                       mu + s (d |Z0| + c Z1), Z0 then Z1, d = alpha / sqrt(1 + alpha^2),
                       c = sqrt(1 - d^2)      (Azzalini's construction from two normals)

Pinned against the laws themselves in tests/test_oracle_laws.py.
"""
import numpy as np

UNIF, NORMAL, LOGNORMAL, EXP, GUMBEL, PARETO, GPARETO, WEIBULL = range(1, 9)
GAMMA, BETA, CHI2, T, F, SKEWNORMAL = range(9, 15)
NPARAMS = {UNIF: 2, NORMAL: 2, LOGNORMAL: 2, EXP: 1, GUMBEL: 2, PARETO: 2, GPARETO: 3, WEIBULL: 2,
           GAMMA: 2, BETA: 2, CHI2: 1, T: 1, F: 2, SKEWNORMAL: 3}
BASE = {UNIF: "u01", NORMAL: "norm", LOGNORMAL: "norm", EXP: "exp", GUMBEL: "u01", PARETO: "exp",
        GPARETO: "exp", WEIBULL: "exp"}


def transform(law, base, p, bitexact=None):
    """The law's value for each base draw (a float64 array).  bitexact (default:
    the oracle's current setting) takes exp, log and pow correctly rounded."""
    from oracle import bitexact_on, crmath, CR_EXP, CR_LOG, CR_POW
    x = np.asarray(base, dtype=np.float64)
    p = [float(v) for v in p]
    if bitexact is None:
        bitexact = bitexact_on()
    if bitexact:
        exp = lambda t: crmath(CR_EXP, t).reshape(np.shape(t))
        log = lambda t: crmath(CR_LOG, t).reshape(np.shape(t))
        power = lambda t, e: crmath(CR_POW, t, e).reshape(np.shape(t))
    else:
        exp, log, power = np.exp, np.log, np.power
    with np.errstate(divide="ignore", over="ignore", invalid="ignore"):
        if law == UNIF:
            a, b = p
            return a + (b - a) * x
        if law == NORMAL:
            mu, sigma = p
            return mu + sigma * x
        if law == LOGNORMAL:
            mu, sigma = p
            return exp(mu + sigma * x)
        if law == EXP:
            (beta,) = p
            return beta * x
        if law == GUMBEL:
            mu, beta = p
            return mu - beta * log(-log(x))
        if law == PARETO:
            xm, alpha = p
            return xm * exp(x / alpha)
        if law == GPARETO:
            mu, s, xi = p
            if xi == 0.0:
                return mu + s * x
            P = exp(x / (1.0 / abs(xi)))
            if xi > 0.0:
                return mu + (s * (P - 1.0)) / xi
            return mu - (s * (1.0 - 1.0 / P)) / xi
        if law == WEIBULL:
            k, lam = p
            return lam * power(x, 1.0 / k)
    raise ValueError(f"unknown law {law}")


def draw(stream, law, p, n):
    """n draws of the law from one oracle stream (advancing it)."""
    p = [float(v) for v in p]
    if law in BASE:
        return transform(law, getattr(stream, BASE[law])(n), p)
    if law == GAMMA:
        alpha, theta = p
        return theta * stream.gamma(alpha, n)
    if law == BETA:
        return stream.beta(p[0], p[1], n)
    if law == CHI2:
        return 2.0 * stream.gamma(p[0] / 2.0, n)
    if law == T:
        (nu,) = p
        out = np.empty(n)
        for k in range(n):
            z = stream.norm(1)[0]
            v = 2.0 * stream.gamma(nu / 2.0, 1)[0]
            out[k] = z / np.sqrt(v / nu)
        return out
    if law == F:
        nu1, nu2 = p
        out = np.empty(n)
        for k in range(n):
            x = stream.gamma(nu1 / 2.0, 1)[0]
            y = stream.gamma(nu2 / 2.0, 1)[0]
            out[k] = (x / nu1) / (y / nu2)
        return out
    if law == SKEWNORMAL:
        mu, s, alpha = p
        d = alpha / np.sqrt(1.0 + alpha * alpha)
        c = np.sqrt(1.0 - d * d)
        z = stream.norm(2 * n).reshape(n, 2)
        return mu + s * (d * np.abs(z[:, 0]) + c * z[:, 1])
    raise ValueError(f"unknown law {law}")


# binary32 base draws of the float versions (32-bit items)
BASE_F32 = {"u01": "u01f", "norm": "normf", "exp": "expf"}


def draw_f32(stream, law, p, n):
    """n binary32 draws of a law (the paper's float versions): the binary32
    base draw, the transform in binary64 on that value, one rounding to
    binary32; Gamma(alpha, theta) is the float gamma; the laws of several
    draws combine float gammas (binary64, unrounded) and binary32 normals of
    one item stream in binary64, as their binary64 forms do, with one
    rounding (oracle.c, or_mixf)."""
    if law == GAMMA:
        return stream.gammaf(p[0], n, p[1])
    if law in (BETA, CHI2, T, F, SKEWNORMAL):
        return stream.mixf(law, p, n)
    if law not in BASE:
        raise ValueError(f"law {law} has no binary32 form")
    base = getattr(stream, BASE_F32[BASE[law]])(n).astype(np.float64)
    with np.errstate(divide="ignore", over="ignore", invalid="ignore"):
        return transform(law, base, [float(v) for v in p]).astype(np.float32)
