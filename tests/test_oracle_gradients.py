"""Pins of the gradient and multivariate-normal references (CPU only)."""
import math

import numpy as np
import pytest
from scipy import special as sp

import oracle
from oracle import Stream, gradients, mvn


def test_beta_a1_closed_form():
    """Beta(a, 1): z = u^(1/a) so dz/da = -z ln z / a."""
    rng = np.random.default_rng(1)
    a = np.exp(rng.uniform(np.log(0.05), np.log(50), 200))
    z = rng.random(200) ** (1 / a)
    z = np.clip(z, 1e-300, 1 - 1e-12)
    ga, _ = gradients.beta_dz_dab(z, a, np.ones_like(a))
    ref = -z * np.log(z) / a
    ok = np.abs(ref) > 1e-200
    assert np.allclose(ga[ok], ref[ok], rtol=1e-6, atol=0)


def test_beta_1b_closed_form():
    """Beta(1, b): z = 1 - (1-u)^(1/b) so dz/db = (1 - z) ln(1 - z) / b."""
    rng = np.random.default_rng(2)
    b = np.exp(rng.uniform(np.log(0.05), np.log(50), 200))
    z = 1 - rng.random(200) ** (1 / b)
    z = np.clip(z, 1e-12, 1 - 1e-12)
    _, gb = gradients.beta_dz_dab(z, np.ones_like(b), b)
    ref = (1 - z) * np.log1p(-z) / b
    assert np.allclose(gb, ref, rtol=1e-6, atol=0)


def test_gamma_small_z_asymptote():
    """As z -> 0, P(alpha, z) ~ z^alpha / Gamma(alpha + 1), so
    dz/dalpha ~ z (psi(alpha + 1) - ln z) / alpha (relative error O(z))."""
    alpha = np.array([0.05, 0.1, 0.5, 1.0, 3.0])
    z = np.array([1e-30, 1e-20, 1e-12, 1e-10, 1e-8])
    g = gradients.gamma_dz_dalpha(z, alpha)
    ref = z * (sp.digamma(alpha + 1) - np.log(z)) / alpha
    assert np.allclose(g, ref, rtol=1e-6)


@pytest.mark.parametrize("alpha,z", [(0.05, 1e-8), (0.05, 0.3), (0.5, 0.01), (1.0, 1.0), (2.5, 0.3),
                                     (2.5, 9.0), (20.0, 12.0), (20.0, 35.0), (50.0, 50.0), (50.0, 80.0)])
def test_gamma_fd_matches_mpmath(alpha, z):
    g = gradients.gamma_dz_dalpha(np.array([z]), np.array([alpha]))[0]
    ref = gradients.gamma_dz_dalpha_mp(z, alpha)
    assert abs(g - ref) <= 1e-7 * abs(ref)


@pytest.mark.parametrize("a,b,z", [(0.05, 0.05, 1e-6), (0.5, 3.0, 0.2), (2.0, 5.0, 0.3), (2.0, 5.0, 0.95),
                                   (40.0, 0.1, 0.999), (10.0, 10.0, 0.5), (0.3, 45.0, 1e-4)])
def test_beta_fd_matches_mpmath(a, b, z):
    ga, gb = gradients.beta_dz_dab(np.array([z]), np.array([a]), np.array([b]))
    ra, rb = gradients.beta_dz_da_mp(z, a, b)
    assert abs(ga[0] - ra) <= 1e-6 * abs(ra)
    assert abs(gb[0] - rb) <= 1e-6 * abs(rb)


@pytest.mark.parametrize("alpha", [0.3, 2.0, 15.0])
def test_gamma_gradient_unbiased(alpha):
    """d/dalpha E[z] = 1 and d/dalpha E[z^2] = 2 alpha + 1 for Gamma(alpha, 1)."""
    n = 100000
    z = Stream.seeded("philox4x32", 3).gamma(alpha, n)
    g = gradients.gamma_dz_dalpha(z, np.full(n, alpha))
    assert abs(g.mean() - 1) < 6 * g.std() / math.sqrt(n)
    h = 2 * z * g
    assert abs(h.mean() - (2 * alpha + 1)) < 6 * h.std() / math.sqrt(n)


@pytest.mark.parametrize("a,b", [(0.5, 2.0), (3.0, 3.0)])
def test_beta_gradient_unbiased(a, b):
    n = 100000
    z = Stream.seeded("philox4x32", 4).beta(a, b, n)
    z = np.clip(z, 1e-300, np.nextafter(1, 0))
    ga, gb = gradients.beta_dz_dab(z, np.full(n, a), np.full(n, b))
    assert abs(ga.mean() - b / (a + b) ** 2) < 6 * ga.std() / math.sqrt(n)
    assert abs(gb.mean() + a / (a + b) ** 2) < 6 * gb.std() / math.sqrt(n)


def test_mvn_reference_identities():
    rng = np.random.default_rng(5)
    d, n = 16, 5000
    q, r = np.linalg.qr(rng.standard_normal((d, d)))
    q = q * np.sign(np.diag(r))
    sigma = q @ np.diag(np.logspace(-2, 2, d)) @ q.T
    sigma = (sigma + sigma.T) / 2
    L = mvn.cholesky(sigma)
    assert np.allclose(L @ L.T, sigma, rtol=0, atol=1e-12 * np.abs(sigma).max())
    assert np.allclose(np.triu(L, 1), 0)
    z = Stream.seeded("philox4x32", 6).norm(n * d).reshape(n, d).astype(np.float32)
    mu = rng.standard_normal(d).astype(np.float32)
    x = mvn.forward(z, L.astype(np.float32), mu)
    # sample covariance approaches Sigma (Wishart scale)
    c = np.cov(x.T)
    assert np.abs(c - sigma).max() < 8 * np.sqrt(2 / n) * np.abs(sigma).max()
    g = rng.standard_normal((n, d)).astype(np.float32)
    gmu, gL = mvn.backward(g, z)
    # linear in mu and L: a finite difference of <G, X> is exact up to rounding
    eps = 1e-3
    Lp = L.astype(np.float64).copy()
    Lp[5, 2] += eps
    fd = (np.sum(g * (mvn.forward(z, Lp, mu) - mvn.forward(z, L.astype(np.float32), mu)))) / eps
    assert abs(fd - gL[5, 2]) < 1e-6 * np.abs(g).sum()
    assert np.allclose(gmu, g.astype(np.float64).sum(0))
