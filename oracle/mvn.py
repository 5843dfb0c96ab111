"""Multivariate-normal reference (test infrastructure).

Section 3.1 ("Multivariate normal distribution"): Sigma = L L^T by Cholesky,
then X = mu + L Z for a d x n matrix Z of standard normals; the library also
offers the n x d orientation, X = mu + Z L^T, used here (row j of Z is the
j-th d-vector of normals).  The reference evaluates it in binary64 from the
same binary32 Z, L and mu that the GPU uses, so the only difference left is
the GPU's binary32 accumulation, bounded elementwise by the standard
dot-product bound |X - X_ref| <= gamma_{d+1} (|Z| |L|^T + |mu|),
gamma_k = k u / (1 - k u), u = 2^-24.

Backward: X is linear in mu and L, so grad_mu = sum over rows of G and
grad_L = tril(G^T Z) exactly (only the lower triangle of L is a parameter).
"""
import numpy as np


def cholesky(sigma):
    """Binary64 Cholesky factor (library routine)."""
    return np.linalg.cholesky(np.asarray(sigma, dtype=np.float64))


def forward(z32, l32, mu32):
    z = np.asarray(z32, dtype=np.float64)
    L = np.asarray(l32, dtype=np.float64)
    mu = np.asarray(mu32, dtype=np.float64)
    return mu[None, :] + z @ L.T


def forward_bound(z32, l32, mu32):
    d = np.asarray(l32).shape[0]
    u = 2.0**-24
    g = (d + 1) * u / (1 - (d + 1) * u)
    return g * (np.abs(np.asarray(z32, np.float64)) @ np.abs(np.asarray(l32, np.float64)).T
                + np.abs(np.asarray(mu32, np.float64))[None, :])


def backward(g32, z32):
    g = np.asarray(g32, dtype=np.float64)
    z = np.asarray(z32, dtype=np.float64)
    return g.sum(axis=0), np.tril(g.T @ z)


def backward_bound(g32, z32):
    """Elementwise bound for a binary32 accumulation over the n rows."""
    n = np.asarray(g32).shape[0]
    u = 2.0**-24
    gam = n * u / (1 - n * u)
    g = np.abs(np.asarray(g32, np.float64))
    z = np.abs(np.asarray(z32, np.float64))
    return gam * g.sum(axis=0), gam * np.tril(g.T @ z)
