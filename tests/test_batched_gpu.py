"""GPU parity of batched gamma / beta against the oracle (MI355X).

Set j draws count[j] values from substream j into its slice of the output.
The Marsaglia-Tsang decisions must all agree (equal states afterwards); for
shape >= 1 the value d v uses no transcendental function and must be equal;
with the shape < 1 boost (one exp and a table log on the GPU, a correctly
rounded binary128 power in the oracle) gamma values are within 4 ulp.  A
beta value X / (X + Y) carries the relative differences of both gammas
(each within 2 ulp: the boost and the product g U^(1/a)) plus the rounding
of the sum and the quotient, so beta values are within 8 ulp.  Every
replay of the recorded graph is checked, with eager work in between.
"""
import numpy as np
import pytest

import oracle
import paper_2605_05099_amd as rp
from paper_2605_05099_amd import workloads
from tests.gpu_common import ENGINES, make_streams, oracle_stream, ulp_diff

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

EDGE = [0.01, 0.5, 0.999, 1.0, 1.5, 100.0, 1e-300, 1e300]


def _sets(n, seed, mean=16, cap=100, lo=0.01, hi=100.0):
    rng = np.random.default_rng(seed)
    alpha = np.exp(rng.uniform(np.log(lo), np.log(hi), n))
    count = np.minimum(rng.geometric(1.0 / mean, n), cap).astype(np.int64)
    count[::37] = 0
    count[5::41] = -3          # negative counts count as 0
    alpha[: len(EDGE)] = EDGE
    return alpha, count


def _dev(a):
    return torch.as_tensor(np.ascontiguousarray(a), device="cuda")


def _states_equal(S, engine, ostreams):
    words, phase = S.get()
    nw = rp.STATE_WORDS[rp.ENGINES[engine]]
    for i, o in enumerate(ostreams):
        assert [int(words[k, i]) for k in range(nw)] == o.state[:nw], (engine, i)
        assert int(phase[i]) == o.phase, (engine, i)


def _compare(got, ref, exact_mask, tol=4):
    assert got.shape == ref.shape
    d = ulp_diff(got, ref)
    worst = np.argsort(-d)[:4]
    info = [(int(i), float(got[i]), float(ref[i]), int(d[i])) for i in worst]
    assert (d[exact_mask] == 0).all(), info
    assert d.max() <= tol, info


def _run(kind, S, params, count, plan, total):
    n = len(count)
    out = torch.full((max(total, 1),), -1.0, dtype=torch.float64, device="cuda")
    dc = _dev(count)
    if kind == "gamma":
        rp.rp_gamma_batched(S, _dev(params[0]), dc, n, out, plan)
    else:
        rp.rp_beta_batched(S, _dev(params[0]), _dev(params[1]), dc, n, out, plan)
    torch.cuda.synchronize()
    return out.cpu().numpy()[:total]


def _oracle(kind, ostreams, params, count):
    arr = oracle.StreamArray(ostreams)
    c = np.maximum(count, 0)
    ref = arr.gamma_batched(params[0], c) if kind == "gamma" else arr.beta_batched(params[0], params[1], c)
    return ref, [arr.stream(i) for i in range(len(ostreams))]


def _tol(kind):
    return 4 if kind == "gamma" else 8


def _exact_mask(kind, params, count):
    c = np.maximum(count, 0)
    if kind == "gamma":
        ok = params[0] >= 1.0
    else:
        ok = (params[0] >= 1.0) & (params[1] >= 1.0)
    return np.repeat(ok, c)


@pytest.mark.parametrize("kind", ["gamma", "beta"])
def test_batched_matches_oracle_with_replays(kind):
    engine = "philox4x32"
    n = 2000
    alpha, count = _sets(n, 1)
    b = _sets(n, 2, lo=0.1, hi=10.0)[0]
    params = (alpha,) if kind == "gamma" else (np.clip(alpha, 1e-3, 1e3), b)
    total = int(np.maximum(count, 0).sum())
    S = make_streams(engine, n + 5)     # more substreams than sets
    ostreams = [oracle_stream(engine, i) for i in range(n)]
    plan = rp.rp_plan_create()
    for rep in range(3):                # first call records the graph, then replays
        got = _run(kind, S, params, count, plan, total)
        ref, ostreams = _oracle(kind, ostreams, params, count)
        _compare(got, ref, _exact_mask(kind, params, count), _tol(kind))
        _states_equal(S, engine, ostreams)
        # eager work between replays
        t = torch.empty(64 * 7, dtype=torch.float64, device="cuda")
        rp.rp_fill(make_streams("pcg64", 64), rp.RP_NORM, rp.RP_F64, 0, 0, t, 7)
        torch.cuda.synchronize()
    # substreams beyond n_sets are untouched
    words, _ = S.get()
    for i in range(n, n + 5):
        assert [int(words[k, i]) for k in range(3)] == oracle_stream(engine, i).state[:3]


@pytest.mark.parametrize("kind", ["gamma", "beta"])
@pytest.mark.parametrize("engine", ["philox4x32", "philox"])
def test_batched_long_sets(engine, kind):
    """Sets of a few thousand values among short ones (the longest sets sort
    first and run longest): values, decisions and final states must be the
    oracle's, on both sides of the shape-1 boundary; two calls in a row
    (graph replay) continue every substream."""
    n = 160
    g = np.random.default_rng(9)
    alpha = np.exp(g.uniform(np.log(0.05), np.log(30.0), n))
    alpha[:4] = [0.3, 0.999, 1.0, 7.5]
    bpar = np.exp(g.uniform(np.log(0.1), np.log(10.0), n))
    count = g.integers(0, 60, n).astype(np.int64)
    count[::16] = g.integers(1025, 3000, len(count[::16]))  # ten long sets
    count[1] = 1025
    count[2] = 1024
    params = (alpha,) if kind == "gamma" else (np.clip(alpha, 0.1, 10.0), bpar)
    total = int(count.sum())
    S = make_streams(engine, n)
    ostreams = [oracle_stream(engine, i) for i in range(n)]
    plan = rp.rp_plan_create()
    for rep in range(2):
        got = _run(kind, S, params, count, plan, total)
        ref, ostreams = _oracle(kind, ostreams, params, count)
        _compare(got, ref, _exact_mask(kind, params, count), _tol(kind))
        _states_equal(S, engine, ostreams)


@pytest.mark.parametrize("engine", ENGINES)
def test_batched_all_engines(engine):
    n = 300 if engine != "ranlux++" else 120
    alpha, count = _sets(n, 3, mean=8, cap=40)
    total = int(np.maximum(count, 0).sum())
    S = make_streams(engine, n)
    plan = rp.rp_plan_create()
    got = _run("gamma", S, (alpha,), count, plan, total)
    ref, ost = _oracle("gamma", [oracle_stream(engine, i) for i in range(n)], (alpha,), count)
    _compare(got, ref, _exact_mask("gamma", (alpha,), count))
    _states_equal(S, engine, ost)
    a, _ = _sets(n, 4, mean=8, cap=40, lo=0.1, hi=10)
    b, _ = _sets(n, 5, mean=8, cap=40, lo=0.1, hi=10)
    got = _run("beta", S, (a, b), count, plan, total)
    ref, ost = _oracle("beta", ost, (a, b), count)
    _compare(got, ref, _exact_mask("beta", (a, b), count), _tol("beta"))
    _states_equal(S, engine, ost)


def test_configurations_give_identical_results():
    n = 3000
    alpha, count = _sets(n, 6, mean=20, cap=200)
    total = int(np.maximum(count, 0).sum())
    outs = []
    for cfg in [(256, 8, 1), (64, 2, 2), (128, 16, 4), (192, 1, 16)]:
        plan = rp.rp_plan_create()
        plan.set_config(*cfg)
        outs.append(_run("gamma", make_streams("philox4x32", n), (alpha,), count, plan, total))
    for o in outs[1:]:
        assert np.array_equal(o.view(np.int64), outs[0].view(np.int64))


def test_invalid_and_degenerate():
    S = make_streams("philox4x32", 16)
    plan = rp.rp_plan_create()
    before = S.get()[0].copy()
    alpha = np.array([0.0, -1.0, np.nan, 2.0, 0.5, -0.0, np.inf * -1, 3.0] * 2)
    count = np.array([3, 2, 1, 4, 2, 1, 1, 0] * 2, dtype=np.int64)
    got = _run("gamma", S, (alpha,), count, plan, int(count.sum()))
    owner = np.repeat(np.arange(16), count)
    bad = ~(alpha > 0)
    assert np.isnan(got[bad[owner]]).all() and np.isfinite(got[~bad[owner]]).all()
    after = S.get()[0]
    assert (after[:, bad] == before[:, bad]).all()
    assert (after[:, 7] == before[:, 7]).all()       # count 0: no draws
    # all counts zero: nothing written, nothing advanced
    out = torch.full((4,), 7.0, dtype=torch.float64, device="cuda")
    rp.rp_gamma_batched(S, _dev(alpha), _dev(np.zeros(16, dtype=np.int64)), 16, out, plan)
    torch.cuda.synchronize()
    assert (out.cpu().numpy() == 7.0).all() and (S.get()[0] == after).all()
    rp.rp_gamma_batched(S, _dev(alpha), _dev(count), 0, out, plan)      # n_sets = 0
    with pytest.raises(rp.RpError) as ei:
        rp.rp_gamma_batched(S, _dev(np.ones(17)), _dev(np.ones(17, dtype=np.int64)), 17, out, plan)
    assert ei.value.code == rp.RP_EINVAL
    with pytest.raises(rp.RpError) as ei:
        plan.set_config(96, 8, 1)
    assert ei.value.code == rp.RP_EINVAL


def test_full_size_autotuned_sampled():
    """10^6 sets, alpha log-uniform in [0.01, 100], counts geometric (mean
    256, cap 4096): about 2.6e8 doubles; then beta with a, b log-uniform in
    [0.1, 10].  Sampled sets checked in full against the oracle."""
    w = workloads.batched_sets()
    n = len(w["alpha"])
    plan = rp.rp_plan_create()
    S = make_streams("philox4x32", n)
    idx = workloads.sampled_substreams(n, k=256)
    for kind, params, count in (("gamma", (w["alpha"],), w["count"]), ("beta", (w["a"], w["b"]), w["count_beta"])):
        total = int(count.sum())
        off = np.concatenate([[0], np.cumsum(count)])
        out = torch.empty(total, dtype=torch.float64, device="cuda")
        dp = [_dev(p) for p in params]
        dc = _dev(count)
        S2 = S.duplicate()
        rp.rp_plan_autotune(plan, S2, kind == "beta", dp[0], dp[1] if kind == "beta" else None, dc, n, out)
        cfg = plan.get_config()
        assert cfg["tuned"]
        if kind == "gamma":
            rp.rp_gamma_batched(S2, dp[0], dc, n, out, plan)
        else:
            rp.rp_beta_batched(S2, dp[0], dp[1], dc, n, out, plan)
        torch.cuda.synchronize()
        # the tuner ran on a copy: S2 was advanced once, by the call above
        sl = np.concatenate([np.arange(off[j], off[j + 1]) for j in idx])
        got = out[torch.as_tensor(sl, device="cuda")].cpu().numpy()
        del out
        ref, _ = _oracle(kind, [oracle_stream("philox4x32", int(j)) for j in idx],
                         tuple(p[idx] for p in params), count[idx])
        _compare(got, ref, _exact_mask(kind, tuple(p[idx] for p in params), count[idx]), _tol(kind))
