"""GPU parity of the lane-per-substream samplers against the oracle (MI355X).

rp_norm_moments: the per-substream sums must equal, bit for bit, the
in-order binary64 sums of the normals rp_fill returns for the same
substreams, and the oracle's sums bit for bit on every substream whose
normals hold no tail value (only tail values may differ, by an ulp of
log1p); the states left behind must equal the oracle's.

rp_gamma_elem / rp_beta_elem: the Marsaglia-Tsang accept/reject decisions
must all agree (shown by equal states afterwards).  For shape >= 1 the value
d v involves no transcendental function, so the binary32 results are equal;
for shape < 1 the boost U^(1/a) is within about an ulp of the correctly
rounded binary64 power, which after rounding to binary32 leaves at most one
binary32 ulp of difference.
"""
import numpy as np
import pytest

import oracle
import paper_2605_05099_amd as rp
from paper_2605_05099_amd import workloads
from tests.gpu_common import ENGINES, make_streams, oracle_stream

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _states_equal(S, engine, ostreams):
    words, phase = S.get()
    nw = rp.STATE_WORDS[rp.ENGINES[engine]]
    for i, o in ostreams.items():
        assert [int(words[k, i]) for k in range(nw)] == o.state[:nw], (engine, i)
        assert int(phase[i]) == o.phase, (engine, i)


def _moments(S, per):
    n = len(S)
    s = torch.empty(n, dtype=torch.float64, device="cuda")
    q = torch.empty(n, dtype=torch.float64, device="cuda")
    rp.rp_norm_moments(S, per, s, q)
    torch.cuda.synchronize()
    return s.cpu().numpy(), q.cpu().numpy()


def _fill_normals(S, per):
    n = len(S)
    t = torch.empty(n * per, dtype=torch.float64, device="cuda")
    rp.rp_fill(S, rp.RP_NORM, rp.RP_F64, 0, 0, t, per)
    torch.cuda.synchronize()
    return t.cpu().numpy().reshape(n, per)


def _in_order(x):
    """s = x_0 + x_1 + ... and q = RN(x_0 x_0) + RN(x_1 x_1) + ..., each added
    in index order in binary64 (cumulative sums run strictly left to right)."""
    if x.shape[-1] == 0:
        return 0.0, 0.0
    return np.cumsum(x)[-1], np.cumsum(x * x)[-1]


def _check_moments(engine, S, per, ostreams):
    """The moments equal, bit for bit, the in-order binary64 sums of the very
    normals rp_fill returns for the same substreams; those normals equal the
    oracle's except in the tail (|x| > r, where log1p may differ by an ulp),
    so the moments of every substream without a tail value equal the
    oracle's bit for bit.  Tail substreams: the oracle's sums within a few
    ulps of the partial sums."""
    D = S.duplicate()
    s, q = _moments(S, per)
    x = _fill_normals(D, per)
    r = 3.6541528853610088
    exact = 0
    for i, o in ostreams.items():
        gs, gq = _in_order(x[i])
        assert s[i] == gs and q[i] == gq, (engine, per, i, s[i] - gs, q[i] - gq)
        ox = o.copy().norm(per)
        rs, rq = o.norm_moments(per)
        if per and np.abs(ox).max() >= r:
            assert abs(s[i] - rs) <= 1e-13 * max(1.0, rq), (engine, per, i, s[i], rs)
            assert abs(q[i] - rq) <= 1e-13 * max(1.0, rq), (engine, per, i, q[i], rq)
        else:
            assert s[i] == rs and q[i] == rq, (engine, per, i, s[i] - rs, q[i] - rq)
            exact += 1
    return exact


@pytest.mark.parametrize("engine", ENGINES)
def test_norm_moments_matches_oracle(engine):
    n = 67 if engine != "ranlux++" else 37
    S = make_streams(engine, n)
    ostreams = {i: oracle_stream(engine, i) for i in range(n)}
    exact = 0
    for per in (3000, 1, 0, 257):
        exact += _check_moments(engine, S, per, ostreams)
        _states_equal(S, engine, ostreams)
    # most substreams of 1, 257 and 3000 normals have no tail value
    assert exact >= 2 * n, exact


def test_norm_moments_continues_a_fill():
    """Moments after a fill continue the same substreams (shared state)."""
    S = make_streams("philox4x32", 64)
    t = torch.empty(64 * 5, dtype=torch.float64, device="cuda")
    rp.rp_fill(S, rp.RP_NORM, rp.RP_F64, 0, 0, t, 5)
    ostreams = {}
    for i in (0, 17, 63):
        o = oracle_stream("philox4x32", i)
        o.norm(5)
        ostreams[i] = o
    _check_moments("philox4x32", S, 100, ostreams)


@pytest.mark.parametrize("engine,jump_log2", [("ranlux++", 64), ("sfc64", 0)])
def test_norm_moments_full_size_sampled(engine, jump_log2):
    """2^18 substreams x 2^16 normals (ranlux++ substreams 2^64 steps apart,
    sfc64 substreams from spawn keys); sampled substreams checked against the
    in-order sums of the same normals and against the oracle."""
    n, per = 2**18, 2**16
    S = make_streams(engine, n, jump_log2=jump_log2)
    D = S.duplicate()
    s, q = _moments(S, per)
    assert np.isfinite(s).all() and np.isfinite(q).all()
    # sum of squares of 2^16 normals: mean 2^16, sd sqrt(2 * 2^16)
    assert abs(q.mean() / per - 1.0) < 1e-3
    assert abs(s.mean()) < 0.05 * np.sqrt(per)
    idx = workloads.sampled_substreams(n, k=24)
    # the normals of the sampled substreams, from a copy of their states
    words, phase = D.get()
    nw = rp.STATE_WORDS[rp.ENGINES[engine]]
    sub = rp.rp_streams_create(rp.rp_create(engine).seed(1), make_kind(engine), len(idx), jump_log2)
    sub.set(words[:, idx].reshape(nw, len(idx)), phase[idx])
    x = _fill_normals(sub, per)
    for k, i in enumerate(idx):
        gs, gq = _in_order(x[k])
        assert s[i] == gs and q[i] == gq, (engine, i, s[i] - gs, q[i] - gq)
        rs, rq = oracle_stream(engine, i, jump_log2=jump_log2).norm_moments(per)
        assert abs(s[i] - rs) <= 1e-12 * rq, (engine, i)
        assert abs(q[i] - rq) <= 1e-12 * rq, (engine, i)


def make_kind(engine):
    from tests.gpu_common import FAMILY
    return FAMILY[engine][0]


# ---------------------------------------------------------------------------
EDGE_ALPHA = [1e-30, 1.4e-45, 1e-3, 0.1, 0.5, 0.999, 1.0, 1.0000001, 1.5, 2.0, 10.0, 1e3, 1e6, 3e38]


def _alpha(n, seed):
    rng = np.random.default_rng(seed)
    a = np.exp(rng.uniform(np.log(0.01), np.log(100.0), n)).astype(np.float32)
    a[: len(EDGE_ALPHA)] = EDGE_ALPHA
    return a


def _f32_ulps(a, b):
    ia = np.asarray(a, dtype=np.float32).view(np.int32).astype(np.int64)
    ib = np.asarray(b, dtype=np.float32).view(np.int32).astype(np.int64)
    return np.abs(ia - ib)


def _check_values(got, ref, shape_lt_1):
    assert got.shape == ref.shape
    d = _f32_ulps(got, ref)
    assert (d[~shape_lt_1] == 0).all(), (got[~shape_lt_1][d[~shape_lt_1] > 0], ref[~shape_lt_1][d[~shape_lt_1] > 0])
    assert d.max() <= 1, d.max()


@pytest.mark.parametrize("engine", ENGINES)
def test_gamma_elem_matches_oracle(engine):
    n = 300 if engine != "ranlux++" else 100
    S = make_streams(engine, n)
    ostreams = {i: oracle_stream(engine, i) for i in range(n)}
    for call in range(2):   # a second call continues every substream
        alpha = _alpha(n, 10 + call)
        a_d = torch.as_tensor(alpha, device="cuda")
        z_d = torch.empty(n, dtype=torch.float32, device="cuda")
        rp.rp_gamma_elem(S, a_d, z_d, n)
        torch.cuda.synchronize()
        got = z_d.cpu().numpy()
        ref = oracle.StreamArray([ostreams[i] for i in range(n)])
        want = ref.gamma_elem(alpha)
        for i in range(n):
            ostreams[i] = ref.stream(i)
        _check_values(got, want, alpha < 1)
        _states_equal(S, engine, ostreams)


@pytest.mark.parametrize("engine", ENGINES)
def test_beta_elem_matches_oracle(engine):
    n = 300 if engine != "ranlux++" else 100
    S = make_streams(engine, n)
    ostreams = {i: oracle_stream(engine, i) for i in range(n)}
    a = _alpha(n, 20)
    b = _alpha(n, 21)[::-1].copy()
    a_d = torch.as_tensor(a, device="cuda")
    b_d = torch.as_tensor(b, device="cuda")
    z_d = torch.empty(n, dtype=torch.float32, device="cuda")
    rp.rp_beta_elem(S, a_d, b_d, z_d, n)
    torch.cuda.synchronize()
    got = z_d.cpu().numpy()
    ref = oracle.StreamArray([ostreams[i] for i in range(n)])
    want = ref.beta_elem(a, b)
    for i in range(n):
        ostreams[i] = ref.stream(i)
    # X / (X + Y) amplifies a one-ulp boost difference by at most a factor 2
    d = _f32_ulps(got, want)
    exact = (a >= 1) & (b >= 1)
    assert (d[exact] == 0).all()
    assert d.max() <= 2, d.max()
    assert ((got >= 0) & (got <= 1)).all()
    _states_equal(S, engine, ostreams)


def test_elem_invalid_shapes_and_sizes():
    S = make_streams("philox4x32", 8)
    before = S.get()[0].copy()
    alpha = torch.tensor([0.0, -1.0, float("nan"), 2.0, -0.0, float("-inf"), 0.5, 3.0], device="cuda")
    z = torch.empty(8, dtype=torch.float32, device="cuda")
    rp.rp_gamma_elem(S, alpha, z, 8)
    torch.cuda.synchronize()
    zc = z.cpu().numpy()
    bad = np.array([1, 1, 1, 0, 1, 1, 0, 0], dtype=bool)
    assert np.isnan(zc[bad]).all() and np.isfinite(zc[~bad]).all()
    after = S.get()[0]
    assert (after[:, bad] == before[:, bad]).all()      # invalid elements use no words
    assert (after[:, ~bad] != before[:, ~bad]).any()
    with pytest.raises(rp.RpError) as ei:
        rp.rp_gamma_elem(S, alpha, z, 9)                 # more elements than substreams
    assert ei.value.code == rp.RP_EINVAL
    with pytest.raises(rp.RpError) as ei:
        rp.rp_beta_elem(S, alpha, 0, z, 8)
    assert ei.value.code == rp.RP_ENULL
    rp.rp_gamma_elem(S, alpha, z, 0)                      # n = 0 does nothing
    z2 = torch.empty(3, dtype=torch.float32, device="cuda")
    alpha2 = torch.tensor([2.0, 0.5, 3.0], device="cuda")
    rp.rp_gamma_elem(S, alpha2, z2, 3)                    # first 3 substreams only
    torch.cuda.synchronize()
    assert np.isfinite(z2.cpu().numpy()).all()


def test_gamma_beta_elem_full_size_sampled():
    """[4096, 1024] elements, element e on Philox4x32-10 substream e."""
    w = workloads.per_element()
    shape = w["alpha"].shape
    n = int(np.prod(shape))
    S = make_streams("philox4x32", n)
    S2 = S.duplicate()
    alpha = w["alpha"].reshape(-1)
    z = torch.empty(n, dtype=torch.float32, device="cuda")
    rp.rp_gamma_elem(S, torch.as_tensor(alpha, device="cuda"), z, n)
    zb = torch.empty(n, dtype=torch.float32, device="cuda")
    a, b = w["a"].reshape(-1), w["b"].reshape(-1)
    rp.rp_beta_elem(S2, torch.as_tensor(a, device="cuda"), torch.as_tensor(b, device="cuda"), zb, n)
    torch.cuda.synchronize()
    zc, zbc = z.cpu().numpy(), zb.cpu().numpy()
    idx = workloads.sampled_substreams(n, k=512)
    ref = oracle.StreamArray([oracle_stream("philox4x32", i) for i in idx])
    _check_values(zc[idx], ref.gamma_elem(alpha[idx]), alpha[idx] < 1)
    ref = oracle.StreamArray([oracle_stream("philox4x32", i) for i in idx])
    d = _f32_ulps(zbc[idx], ref.beta_elem(a[idx], b[idx]))
    assert d.max() <= 2
    # Gamma(alpha) has mean alpha: the normalised mean over 4M elements
    assert abs(np.mean(zc / alpha) - 1.0) < 5e-3
