"""Multivariate-normal reference (test infrastructure).

Section 3.1 ("Multivariate normal distribution"): Sigma = L L^T by Cholesky,
then X = mu + L Z for a d x n matrix Z of standard normals; the library also
offers the n x d orientation, X = mu + Z L^T, used here (row j of Z is the
j-th d-vector of normals).  The reference evaluates it in binary64 from the
same binary32 Z, L and mu that the GPU uses, so the only difference left is
the GPU's binary32 accumulation, bounded elementwise by the standard
dot-product bound |X - X_ref| <= gamma_{d+1} (|Z| |L|^T + |mu|),
gamma_k = k u / (1 - k u), u = 2^-24.

Semidefinite covariances: when the Cholesky factorization fails, a pivoted
Cholesky factorization (LAPACK dpstrf semantics) gives Sigma = A A^T with
A = P L not triangular; the forward is the same product with A.

Backward: X is linear in mu and L, so grad_mu = sum over rows of G and
grad_L = tril(G^T Z) exactly (only the lower triangle of L is a parameter).
"""
import numpy as np


def cholesky(sigma):
    """Binary64 Cholesky factor (library routine)."""
    return np.linalg.cholesky(np.asarray(sigma, dtype=np.float64))


def pivoted_cholesky(sigma):
    """Pivoted Cholesky of a symmetric positive semidefinite matrix (the
    paper's fallback when the plain factorization fails; LAPACK's dpstrf
    semantics).  Step j takes the largest remaining diagonal entry of the
    Schur complement as the pivot and stops when it is at most
    tol = d eps max_i Sigma_ii.  Left-looking: column j of L is formed from
    the permuted Sigma and the earlier columns.  Returns (L, perm, rank,
    smallest trailing diagonal), with Sigma[perm][:, perm] = L L^T and the
    columns of L from rank on zero."""
    S = np.array(sigma, dtype=np.float64)
    d = S.shape[0]
    S = np.tril(S) + np.tril(S, -1).T          # the lower triangle is read
    perm = list(range(d))
    L = np.zeros((d, d))
    tol = d * np.finfo(np.float64).eps * max(S[i, i] for i in range(d))
    rank = d
    rest = 0.0
    for j in range(d):
        diag = [S[i, i] - sum(L[i, k] * L[i, k] for k in range(j)) for i in range(j, d)]
        p = j + int(np.argmax(diag))
        if not diag[p - j] > tol:
            rank = j
            rest = min(diag)
            break
        if p != j:
            S[[j, p], :] = S[[p, j], :]
            S[:, [j, p]] = S[:, [p, j]]
            L[[j, p], :j] = L[[p, j], :j]
            perm[j], perm[p] = perm[p], perm[j]
        ljj = np.sqrt(diag[p - j])
        L[j, j] = ljj
        for i in range(j + 1, d):
            L[i, j] = (S[i, j] - sum(L[i, k] * L[j, k] for k in range(j))) / ljj
    return L, perm, rank, rest


def factor(sigma):
    """The paper's factor A with Sigma = A A^T: the Cholesky factor when
    Sigma is positive definite, else P L from the pivoted factorization
    (row perm[k] of A is row k of L).  Raises ValueError when a trailing
    diagonal entry is below -tol (Sigma is not semidefinite)."""
    try:
        return cholesky(sigma), len(sigma)
    except np.linalg.LinAlgError:
        pass
    L, perm, rank, rest = pivoted_cholesky(sigma)
    d = L.shape[0]
    tol = d * np.finfo(np.float64).eps * max(np.diag(np.asarray(sigma, dtype=np.float64)))
    if rank < d and rest < -tol:
        raise ValueError("covariance is not positive semidefinite")
    A = np.zeros_like(L)
    A[perm, :] = L
    return A, rank


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
