"""The covariance factor for semidefinite matrices (host code, no GPU).

Pins: the oracle's pivoted Cholesky against LAPACK's dpstrf (SciPy), which
defines the pivot rule, the stopping tolerance and the factor; the library's
rp_mvn_factor against the oracle (definite, rank-deficient, indefinite and
non-finite inputs).
"""
import numpy as np
import pytest
import scipy.linalg.lapack as lapack

from oracle import mvn as omvn
import paper_2605_05099_amd as rp


def _psd(d, r, seed):
    B = np.random.default_rng(seed).standard_normal((d, r))
    return B @ B.T


@pytest.mark.parametrize("d,r", [(5, 2), (20, 11), (40, 39), (17, 17), (9, 1)])
def test_oracle_pivoted_cholesky_matches_lapack_dpstrf(d, r):
    S = _psd(d, r, d * 7 + r)
    L, perm, rank, _ = omvn.pivoted_cholesky(S)
    c, piv, rk, info = lapack.dpstrf(S, lower=1)
    assert rank == rk
    assert perm == list(piv - 1)
    Lc = np.tril(c)[:, :rk]
    assert np.abs(L[:, :rk] - Lc).max() <= 1e-12 * max(1.0, np.abs(Lc).max())
    assert np.abs(S[np.ix_(perm, perm)] - L @ L.T).max() <= 1e-12 * np.abs(S).max()


def test_oracle_factor_reduces_to_cholesky_when_definite():
    S = _psd(12, 30, 1)
    A, rank = omvn.factor(S)
    assert rank == 12
    assert np.array_equal(A, np.linalg.cholesky(S))


def test_oracle_factor_rejects_indefinite():
    with pytest.raises(ValueError):
        omvn.factor(np.diag([2.0, -1.0, 1.0]))


@pytest.mark.parametrize("d,r", [(6, 6), (6, 3), (64, 40), (100, 1), (130, 100)])
def test_library_factor_matches_oracle(d, r):
    S = _psd(d, r, 100 + d + r)
    A, rank = rp.rp_mvn_factor(S)
    Ao, rko = omvn.factor(S)
    assert rank == rko == r
    assert np.abs(A - Ao).max() <= 1e-11 * max(1.0, np.abs(Ao).max())
    assert np.abs(A @ A.T - S).max() <= 1e-11 * np.abs(S).max()
    assert not A[:, r:].any()
    if r == d:   # definite: the plain Cholesky factor, lower triangular
        assert not np.triu(A, 1).any()


def test_library_factor_errors():
    with pytest.raises(rp.RpError) as ei:
        rp.rp_mvn_factor(np.diag([1.0, -1.0, 2.0]))
    assert ei.value.code == rp.RP_ENOTSPD
    S = np.eye(3)
    S[2, 1] = np.nan
    with pytest.raises(rp.RpError) as ei:
        rp.rp_mvn_factor(S)
    assert ei.value.code == rp.RP_EINVAL
    A, rank = rp.rp_mvn_factor(np.zeros((4, 4)))   # the zero matrix: rank 0
    assert rank == 0 and not A.any()
