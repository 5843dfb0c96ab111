"""Gradient oracle for the implicit-reparameterization backward (test infrastructure).

A sample z = F^{-1}(u; theta) moves with its parameter while the uniform
u = F(z; theta) is held fixed, so dz/dtheta = -(dF/dtheta)(z) / f(z; theta).
The oracle evaluates that derivative directly from its definition, as a
central finite difference of the binary64 inverse CDF at fixed u, with one
Richardson extrapolation step:

    D(h) = [F^{-1}(u; theta + h) - F^{-1}(u; theta - h)] / (2 h)
    dz/dtheta ~ (4 D(h/2) - D(h)) / 3

SciPy supplies F and F^{-1} (regularized incomplete gamma / beta and their
inverses).  In the upper tail the complementary functions are used so that u
keeps its relative precision.  Pins: closed forms (Beta(a, 1), Beta(1, b)),
the small-z asymptote of the gamma case, mpmath evaluations of the defining
ratio, and the unbiasedness identities E[dz/dalpha] = 1 for Gamma(alpha, 1)
and E[dz/da] = b/(a+b)^2, E[dz/db] = -a/(a+b)^2 for Beta(a, b).
"""
import numpy as np
from scipy import special as sp


def _richardson(fn, theta, rel_h):
    h = rel_h * theta
    d1 = (fn(theta + h) - fn(theta - h)) / (2 * h)
    d2 = (fn(theta + h / 2) - fn(theta - h / 2)) / h
    return (4 * d2 - d1) / 3


def gamma_dz_dalpha(z, alpha, rel_h=1e-4):
    """dz/dalpha for Gamma(alpha, 1) samples z (arrays, binary64)."""
    z = np.asarray(z, dtype=np.float64)
    alpha = np.asarray(alpha, dtype=np.float64)
    p = sp.gammainc(alpha, z)
    q = sp.gammaincc(alpha, z)
    lower = p <= 0.5

    def inv(a):
        return np.where(lower, sp.gammaincinv(a, p), sp.gammainccinv(a, q))

    return _richardson(inv, alpha, rel_h)


def beta_dz_dab(z, a, b, rel_h=1e-4):
    """(dz/da, dz/db) for Beta(a, b) samples z (arrays, binary64)."""
    z = np.asarray(z, dtype=np.float64)
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    u = sp.betainc(a, b, z)
    w = sp.betainc(b, a, 1 - z)   # = 1 - u, accurate when z is near 1
    lower = u <= 0.5

    # Lower half: difference z = I^{-1}(u; a, b) itself.  Upper half:
    # difference y = 1 - z = I^{-1}(1 - u; b, a), which keeps full relative
    # precision near z = 1, and negate (dz = -dy).
    def inv(aa, bb):
        return np.where(lower, sp.betaincinv(aa, bb, u), -sp.betaincinv(bb, aa, w))

    ga = _richardson(lambda t: inv(t, b), a, rel_h)
    gb = _richardson(lambda t: inv(a, t), b, rel_h)
    return ga, gb


def gamma_dz_dalpha_mp(z, alpha, dps=40):
    """Defining ratio -dP/dalpha / p at high precision (mpmath), scalar."""
    import mpmath as mp
    with mp.workdps(dps):
        z = mp.mpf(float(z))
        a = mp.mpf(float(alpha))
        dP = mp.diff(lambda t: mp.gammainc(t, 0, z, regularized=True), a)
        pdf = mp.exp((a - 1) * mp.log(z) - z - mp.loggamma(a))
        return float(-dP / pdf)


def beta_dz_da_mp(z, a, b, dps=40):
    import mpmath as mp
    with mp.workdps(dps):
        z, a, b = mp.mpf(float(z)), mp.mpf(float(a)), mp.mpf(float(b))
        dIa = mp.diff(lambda t: mp.betainc(t, b, 0, z, regularized=True), a)
        dIb = mp.diff(lambda t: mp.betainc(a, t, 0, z, regularized=True), b)
        pdf = mp.exp((a - 1) * mp.log(z) + (b - 1) * mp.log(1 - z) - mp.log(mp.beta(a, b)))
        return float(-dIa / pdf), float(-dIb / pdf)
