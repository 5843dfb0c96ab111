"""GPU multivariate normal against the binary64 oracle (MI355X).

Forward: X = mu + Z L^T with Z the binary32-rounded ziggurat normals of the
row substreams; the oracle evaluates the same product in binary64 from the
same binary32 Z, L and mu, and every element must lie within the dot-product
rounding bound gamma_{d+1} (|Z| |L|^T + |mu|).  Backward: gmu = column sums
of G, gL = tril(G^T Z); each partial is a binary32 accumulation over one row
slice (at most `slice` rows), the partials are combined in binary64, so
|error| <= (gamma_slice + u) (|G|^T |Z|) elementwise.
"""
import numpy as np
import pytest

import oracle
from oracle import mvn as omvn
import paper_2605_05099_amd as rp
from paper_2605_05099_amd import workloads
from tests.gpu_common import make_streams, oracle_stream

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

U = 2.0**-24


def _gamma(k):
    return k * U / (1 - k * U)


def _slice_rows(n, d):
    """Rows per backward slice, as the library chooses them."""
    nt = (d + 127) // 128
    ntl = nt * (nt + 1) // 2
    nsl = min((2048 + ntl - 1) // ntl, (n + 31) // 32)
    nsl = max(nsl, 1)
    sl = (n + nsl - 1) // nsl
    return max((sl + 31) // 32 * 32, 32)


def _factor(d):
    w = workloads.mvn(d)
    L = rp.rp_cholesky(w["sigma"]).astype(np.float32)
    return w["mu"].astype(np.float32), L


def _dev(a):
    return torch.as_tensor(np.ascontiguousarray(a), device="cuda")


def _z_oracle(rows, d):
    return oracle.StreamArray([oracle_stream("philox4x32", int(i)) for i in rows]).mvn_z(d)


@pytest.mark.parametrize("d", [1, 3, 64, 100, 256, 300, 520])
def test_mvn_forward_backward_small(d):
    n = 1000
    mu, L = _factor(d)
    S = make_streams("philox4x32", n + 3)
    S0 = S.duplicate()
    X = torch.empty((n, d), dtype=torch.float32, device="cuda")
    rp.rp_mvn(S, _dev(mu), _dev(L), d, n, X)
    torch.cuda.synchronize()
    z = _z_oracle(range(n), d)
    ref = omvn.forward(z, L, mu)
    err = np.abs(X.cpu().numpy().astype(np.float64) - ref)
    assert (err <= omvn.forward_bound(z, L, mu)).all(), err.max()
    # substreams advanced by d normals each; the extra ones untouched
    words, phase = S.get()
    for i in (0, 1, n // 2, n - 1, n, n + 2):
        o = oracle_stream("philox4x32", i)
        if i < n:
            o.norm(d)
        assert [int(words[k, i]) for k in range(3)] == o.state[:3] and int(phase[i]) == o.phase
    # backward from the states the forward started at
    rng = np.random.default_rng(d)
    G = rng.standard_normal((n, d)).astype(np.float32)
    gmu = torch.empty(d, dtype=torch.float32, device="cuda")
    gL = torch.empty((d, d), dtype=torch.float32, device="cuda")
    rp.rp_mvn_backward(S0, _dev(G), d, n, gmu, gL)
    torch.cuda.synchronize()
    rmu, rL = omvn.backward(G, z)
    g = _gamma(_slice_rows(n, d)) + U
    ag = np.abs(G.astype(np.float64))
    assert (np.abs(gmu.cpu().numpy() - rmu) <= g * ag.sum(axis=0)).all()
    bound = g * np.tril(ag.T @ np.abs(z.astype(np.float64)))
    gl = gL.cpu().numpy().astype(np.float64)
    assert (np.abs(gl - rL) <= bound).all()
    assert (np.triu(gl, 1) == 0).all()
    # the backward did not advance S0
    assert (S0.get()[0] == make_streams("philox4x32", n + 3).get()[0]).all()


def test_cholesky_on_device_inputs_and_errors():
    with pytest.raises(rp.RpError) as ei:
        rp.rp_cholesky(np.array([[1.0, 2.0], [2.0, 1.0]]))
    assert ei.value.code == rp.RP_ENOTSPD
    S = make_streams("philox4x32", 4)
    X = torch.empty((4, 4), dtype=torch.float32, device="cuda")
    with pytest.raises(rp.RpError) as ei:
        rp.rp_mvn(S, 0, 0, 4, 4, X)
    assert ei.value.code == rp.RP_ENULL
    with pytest.raises(rp.RpError) as ei:
        rp.rp_mvn(S, X, X, 4, 5, X)          # more rows than substreams
    assert ei.value.code == rp.RP_EINVAL
    rp.rp_mvn(S, X, X, 4, 0, X)              # n = 0 does nothing


@pytest.mark.parametrize("d", [64, 256, 512])
def test_mvn_full_size(d):
    """2^20 rows: forward checked on 2048 sampled rows; backward gmu in full
    and gL in full for its first 8 columns (which need only the first 8
    normals of every row)."""
    n = 2**20
    mu, L = _factor(d)
    S = make_streams("philox4x32", n)
    S0 = S.duplicate()
    X = torch.empty((n, d), dtype=torch.float32, device="cuda")
    rp.rp_mvn(S, _dev(mu), _dev(L), d, n, X)
    torch.cuda.synchronize()
    rows = workloads.sampled_substreams(n, k=2048)
    z = _z_oracle(rows, d)
    got = X[torch.as_tensor(rows, device="cuda")].cpu().numpy().astype(np.float64)
    del X
    err = np.abs(got - omvn.forward(z, L, mu))
    assert (err <= omvn.forward_bound(z, L, mu)).all(), err.max()
    G = torch.randn((n, d), dtype=torch.float32, device="cuda", generator=torch.Generator("cuda").manual_seed(d))
    gmu = torch.empty(d, dtype=torch.float32, device="cuda")
    gL = torch.empty((d, d), dtype=torch.float32, device="cuda")
    rp.rp_mvn_backward(S0, G, d, n, gmu, gL)
    torch.cuda.synchronize()
    Gh = G.cpu().numpy().astype(np.float64)
    del G
    g = _gamma(_slice_rows(n, d)) + U
    assert (np.abs(gmu.cpu().numpy() - Gh.sum(axis=0)) <= g * np.abs(Gh).sum(axis=0)).all()
    z8 = oracle.StreamArray.key_family("philox4x32", 42, n).mvn_z(8).astype(np.float64)
    ref = Gh.T @ z8                     # columns 0..7 of G^T Z
    bound = g * (np.abs(Gh).T @ np.abs(z8))
    gl = gL.cpu().numpy().astype(np.float64)[:, :8]
    low = np.tril(np.ones((d, 8), dtype=bool))
    assert (np.abs(gl - ref)[low] <= bound[low]).all()
    assert (gl[~low] == 0).all()


def test_mvn_autograd():
    from paper_2605_05099_amd.autograd import sample_mvn
    d, n = 64, 4096
    mu, L = _factor(d)
    mu_t = _dev(mu).requires_grad_(True)
    L_t = _dev(L).requires_grad_(True)
    S = make_streams("philox4x32", n)
    X = sample_mvn(mu_t, L_t, S, n)
    G = torch.randn_like(X)
    X.backward(G)
    gmu = torch.empty(d, dtype=torch.float32, device="cuda")
    gL = torch.empty((d, d), dtype=torch.float32, device="cuda")
    rp.rp_mvn_backward(make_streams("philox4x32", n), G, d, n, gmu, gL)
    torch.cuda.synchronize()
    assert torch.equal(mu_t.grad, gmu) and torch.equal(L_t.grad, gL)


@pytest.mark.parametrize("d,r", [(64, 40), (100, 1), (256, 200)])
def test_mvn_forward_semidefinite_pivoted_factor(d, r):
    """A rank-r covariance: rp_mvn_factor falls back to the pivoted
    factorization (A = P L, not triangular); rp_mvn reads the whole A."""
    rng = np.random.default_rng(d + r)
    B = rng.standard_normal((d, r))
    A, rank = rp.rp_mvn_factor(B @ B.T)
    assert rank == r
    A = A.astype(np.float32)
    mu = rng.standard_normal(d).astype(np.float32)
    n = 777
    S = make_streams("philox4x32", n)
    X = torch.empty((n, d), dtype=torch.float32, device="cuda")
    rp.rp_mvn(S, _dev(mu), _dev(A), d, n, X)
    torch.cuda.synchronize()
    z = _z_oracle(range(n), d)
    ref = omvn.forward(z, A, mu)
    err = np.abs(X.cpu().numpy().astype(np.float64) - ref)
    assert (err <= omvn.forward_bound(z, A, mu)).all(), err.max()
    # the sample covariance lives in the column space of B: X - mu is
    # orthogonal to the complement of range(B)
    if r < d:
        q, _ = np.linalg.qr(B, mode="complete")
        off = (X.cpu().numpy().astype(np.float64) - mu) @ q[:, r:]
        assert np.abs(off).max() < 1e-3 * max(1.0, np.abs(X.cpu().numpy()).max())
