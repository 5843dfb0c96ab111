"""GPU derived laws (rp_fill_law) against the oracle's transforms (MI355X).

Each value is one transform of one base draw; the base draws are those of
rp_fill (bit-exact uniforms; ziggurat values within 4 ulp, tails only), and
the substreams must end where the oracle's do.  The transforms themselves
differ only by the rounding of exp / log / pow (an ulp or two on either
side), so each value is checked against an absolute bound of 32 eps times
the magnitudes that enter it (law by law below): far below any real
mistake, which moves values by O(1) relative amounts.  Uniform, normal and
exponential shift-scale laws use no transcendental and must be bit-exact
away from the ziggurat tails.
"""
import numpy as np
import pytest

import oracle
from oracle import laws
import paper_2605_05099_amd as rp
from paper_2605_05099_amd import workloads
from tests.gpu_common import make_streams, oracle_stream

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

EPS = np.finfo(np.float64).eps
LAWS = [
    (rp.RP_LAW_UNIF, (-2.0, 5.0)),
    (rp.RP_LAW_NORMAL, (3.0, 5.0)),
    (rp.RP_LAW_LOGNORMAL, (0.5, 0.75)),
    (rp.RP_LAW_EXP, (2.5,)),
    (rp.RP_LAW_GUMBEL, (1.0, 2.0)),
    (rp.RP_LAW_PARETO, (1.5, 3.0)),
    (rp.RP_LAW_GPARETO, (0.5, 2.0, 0.3)),
    (rp.RP_LAW_GPARETO, (0.5, 2.0, -0.4)),
    (rp.RP_LAW_GPARETO, (0.5, 2.0, 0.0)),
    (rp.RP_LAW_WEIBULL, (1.7, 4.0)),
]
IDS = [f"law{l}_{'_'.join(str(v) for v in p)}" for l, p in LAWS]


def _scale(law, p, base, ref):
    """Magnitudes entering each value (for the absolute bound)."""
    b = np.abs(base)
    with np.errstate(divide="ignore", invalid="ignore", over="ignore"):
        if law in (rp.RP_LAW_UNIF, rp.RP_LAW_NORMAL):
            return abs(p[0]) + abs(p[1]) * (b + 1.0)
        if law == rp.RP_LAW_EXP:
            return p[0] * (b + 1.0)
        if law == rp.RP_LAW_LOGNORMAL:
            return np.abs(ref) * (2.0 + abs(p[1]) * b)
        if law == rp.RP_LAW_GUMBEL:
            return abs(p[0]) + p[1] * (np.abs(np.log(-np.log(base))) + 2.0)
        if law == rp.RP_LAW_PARETO:
            return np.abs(ref) * (2.0 + b / p[1])
        if law == rp.RP_LAW_GPARETO:
            mu, s, xi = p
            if xi == 0.0:
                return abs(mu) + s * (b + 1.0)
            P = np.exp(base * abs(xi))
            return abs(mu) + s * np.maximum(P, 1.0 / P) * (2.0 + b * abs(xi)) / abs(xi)
        if law == rp.RP_LAW_WEIBULL:
            return np.abs(ref) * (2.0 + 1.0 / p[0])
    raise ValueError(law)


def _check(law, p, got, ostreams, per):
    base_name = laws.BASE[law]
    for i, o in enumerate(ostreams):
        base = getattr(o, base_name)(per)
        ref = laws.transform(law, base, p)
        g = got[i]
        tol = 32 * EPS * _scale(law, p, base, ref)
        # ziggurat tails (values the GPU forms with log1p) carry up to 4 ulp
        # of the base value through the transform
        if base_name != "u01":
            tail = np.abs(base) >= (3.6541528853610088 if base_name == "norm" else 7.69711747013105)
            tol = np.where(tail, tol * 8, tol)
        bad = ~(np.abs(g - ref) <= tol) & ~(g == ref)
        assert not bad.any(), (i, int(np.argmax(bad)), float(g[bad][0]), float(ref[bad][0]))
        if law in (rp.RP_LAW_UNIF, rp.RP_LAW_NORMAL, rp.RP_LAW_EXP) and base_name == "u01":
            assert np.array_equal(g, ref)


def _states_equal(S, engine, ostreams):
    words, phase = S.get()
    nw = rp.STATE_WORDS[rp.ENGINES[engine]]
    for i, o in enumerate(ostreams):
        assert [int(words[k, i]) for k in range(nw)] == o.state[:nw], (engine, i)
        assert int(phase[i]) == o.phase, (engine, i)


@pytest.mark.parametrize("law,p", LAWS, ids=IDS)
@pytest.mark.parametrize("engine", ["philox4x32", "pcg64", "x256++", "philox"])
def test_law_matches_oracle(engine, law, p):
    n, per = 48, 1500 + 13      # several 512-word chunks and a ragged tail
    S = make_streams(engine, n)
    out = torch.empty(n * per, dtype=torch.float64, device="cuda")
    rp.rp_fill_law(S, law, p, out, per)
    torch.cuda.synchronize()
    got = out.cpu().numpy().reshape(n, per)
    ost = [oracle_stream(engine, i) for i in range(n)]
    _check(law, p, got, ost, per)
    _states_equal(S, engine, ost)


def test_law_ranlux_and_sfc64_lanes():
    for engine in ("ranlux++", "sfc64"):
        n, per = 64, 300
        S = make_streams(engine, n)
        for law, p in ((rp.RP_LAW_LOGNORMAL, (0.5, 0.75)), (rp.RP_LAW_GUMBEL, (1.0, 2.0))):
            out = torch.empty(n * per, dtype=torch.float64, device="cuda")
            rp.rp_fill_law(S, law, p, out, per)
            torch.cuda.synchronize()
            ost = [oracle_stream(engine, i) for i in range(n)]
            # second law continues the streams where the first left them
            if law == rp.RP_LAW_GUMBEL:
                for o in ost:
                    o.norm(per)
            _check(law, p, out.cpu().numpy().reshape(n, per), ost, per)


def test_law_full_size_sampled():
    """The substream workload's size (2^16 x 2^14 values): sampled
    substreams in full."""
    n, per = workloads.SUB_N, workloads.SUB_PER
    S = make_streams("philox4x32", n)
    out = torch.empty(n * per, dtype=torch.float64, device="cuda")
    idx = workloads.sampled_substreams(n, k=64)
    for law, p in ((rp.RP_LAW_LOGNORMAL, (0.5, 0.75)), (rp.RP_LAW_WEIBULL, (1.7, 4.0))):
        rp.rp_fill_law(S, law, p, out, per)
        torch.cuda.synchronize()
        got = out.view(n, per)[torch.as_tensor(idx, device="cuda")].cpu().numpy()
        ost = [oracle_stream("philox4x32", int(i)) for i in idx]
        if law == rp.RP_LAW_WEIBULL:
            for o in ost:
                o.norm(per)
        _check(law, p, got, ost, per)
    del out


def test_law_errors():
    S = make_streams("philox4x32", 4)
    out = torch.empty(16, dtype=torch.float64, device="cuda")
    bad = [(rp.RP_LAW_UNIF, (1.0, 1.0)), (rp.RP_LAW_NORMAL, (0.0, -1.0)), (rp.RP_LAW_EXP, (0.0,)),
           (rp.RP_LAW_PARETO, (1.0, 0.0)), (rp.RP_LAW_GPARETO, (0.0, 0.0, 1.0)), (rp.RP_LAW_WEIBULL, (-1.0, 1.0)),
           (rp.RP_LAW_GUMBEL, (float("nan"), 1.0)), (rp.RP_LAW_NORMAL, (0.0,)), (99, (1.0, 2.0))]
    before = S.get()[0].copy()
    for law, p in bad:
        with pytest.raises(rp.RpError) as ei:
            rp.rp_fill_law(S, law, p, out, 4)
        assert ei.value.code == rp.RP_EINVAL, (law, p)
    assert (S.get()[0] == before).all()
    rp.rp_fill_law(S, rp.RP_LAW_EXP, (1.0,), out, 0)     # per_stream = 0 does nothing
    assert (S.get()[0] == before).all()


MIX = [
    (rp.RP_LAW_GAMMA, (2.5, 1.5)),
    (rp.RP_LAW_GAMMA, (0.4, 3.0)),
    (rp.RP_LAW_BETA, (2.0, 5.0)),
    (rp.RP_LAW_BETA, (0.5, 0.7)),
    (rp.RP_LAW_CHI2, (3.0,)),
    (rp.RP_LAW_CHI2, (0.8,)),
    (rp.RP_LAW_T, (4.5,)),
    (rp.RP_LAW_F, (5.0, 7.0)),
    (rp.RP_LAW_SKEWNORMAL, (1.0, 2.0, 3.0)),
]
MIX_IDS = [f"law{l}_{'_'.join(str(v) for v in p)}" for l, p in MIX]


@pytest.mark.parametrize("law,p", MIX, ids=MIX_IDS)
@pytest.mark.parametrize("engine", ["philox4x32", "pcg64", "x256++", "sfc64"])
def test_mix_law_matches_oracle(engine, law, p):
    """Laws of several draws per value: every decision (so every state) is
    the oracle's; values differ by the boost's power (4 ulp per gamma draw,
    shape < 1), the ziggurat tails and a division or square root: within 64
    eps of the value (skew-normal: of its terms)."""
    n = 64
    per = 150 if law in (rp.RP_LAW_T, rp.RP_LAW_F) else 300
    S = make_streams(engine, n)
    out = torch.empty(n * per, dtype=torch.float64, device="cuda")
    rp.rp_fill_law(S, law, p, out, per)
    torch.cuda.synchronize()
    got = out.cpu().numpy().reshape(n, per)
    ost = [oracle_stream(engine, i) for i in range(n)]
    for i, o in enumerate(ost):
        ref = laws.draw(o, law, p, per)
        scale = np.abs(ref)
        if law == rp.RP_LAW_SKEWNORMAL:
            scale = scale + abs(p[0]) + p[1] * (np.abs(ref - p[0]) / p[1] + 10.0)
        bad = ~(np.abs(got[i] - ref) <= 64 * EPS * scale) & ~(got[i] == ref)
        assert not bad.any(), (engine, i, int(np.argmax(bad)), float(got[i][bad][0]), float(ref[bad][0]))
    _states_equal(S, engine, ost)


def test_mix_law_errors():
    S = make_streams("philox4x32", 4)
    out = torch.empty(16, dtype=torch.float64, device="cuda")
    for law, p in ((rp.RP_LAW_GAMMA, (0.0, 1.0)), (rp.RP_LAW_BETA, (1.0, -1.0)), (rp.RP_LAW_CHI2, (0.0,)),
                   (rp.RP_LAW_T, (-2.0,)), (rp.RP_LAW_F, (1.0, 0.0)), (rp.RP_LAW_SKEWNORMAL, (0.0, -1.0, 1.0)),
                   (rp.RP_LAW_T, (1.0, 2.0)), (rp.RP_LAW_SKEWNORMAL, (0.0, 1.0, float("inf")))):
        with pytest.raises(rp.RpError) as ei:
            rp.rp_fill_law(S, law, p, out, 4)
        assert ei.value.code == rp.RP_EINVAL, (law, p)


def test_mix_law_ranlux_lanes_and_continuation():
    """ranlux++ (block engine with the table step): two mixture laws in a row
    continue the substreams where the first left them."""
    n, per = 64, 200
    S = make_streams("ranlux++", n)
    ost = [oracle_stream("ranlux++", i) for i in range(n)]
    for law, p in ((rp.RP_LAW_GAMMA, (0.7, 1.0)), (rp.RP_LAW_SKEWNORMAL, (0.0, 1.0, -1.5))):
        out = torch.empty(n * per, dtype=torch.float64, device="cuda")
        rp.rp_fill_law(S, law, p, out, per)
        torch.cuda.synchronize()
        got = out.cpu().numpy().reshape(n, per)
        for i, o in enumerate(ost):
            ref = laws.draw(o, law, p, per)
            tol = 64 * EPS * (np.abs(ref) + (10.0 if law == rp.RP_LAW_SKEWNORMAL else 0.0))
            assert (np.abs(got[i] - ref) <= tol).all(), (law, i)
    _states_equal(S, "ranlux++", ost)


def test_mix_law_full_size_sampled():
    """Gamma and t at the substream workload's size (2^16 x 2^14 values):
    sampled substreams in full."""
    n, per = workloads.SUB_N, workloads.SUB_PER
    S = make_streams("philox4x32", n)
    out = torch.empty(n * per, dtype=torch.float64, device="cuda")
    idx = workloads.sampled_substreams(n, k=32)
    ost = [oracle_stream("philox4x32", int(i)) for i in idx]
    for law, p in ((rp.RP_LAW_GAMMA, (2.5, 1.5)), (rp.RP_LAW_T, (4.5,))):
        rp.rp_fill_law(S, law, p, out, per)
        torch.cuda.synchronize()
        got = out.view(n, per)[torch.as_tensor(idx, device="cuda")].cpu().numpy()
        for k, o in enumerate(ost):
            ref = laws.draw(o, law, p, per)
            assert (np.abs(got[k] - ref) <= 64 * EPS * np.abs(ref)).all(), (law, int(idx[k]))
    del out


@pytest.mark.parametrize("law,p", LAWS, ids=IDS)
@pytest.mark.parametrize("engine", ["philox4x32", "pcg64", "x256++", "squares", "chacha20"])
def test_float_law_matches_oracle(engine, law, p):
    """rp_fill_lawf: the binary32 base draw, the transform in binary64, one
    rounding.  Both sides transform the same binary32 value, so results are
    equal unless an ulp difference of exp / log / pow (or of log1p in a
    ziggurat tail) straddles a binary32 rounding boundary: at most 2
    binary32 ulp, and rare."""
    from tests.gpu_common import ulp_diff
    n, per = 48, 1500 + 13
    S = make_streams(engine, n)
    out = torch.empty(n * per, dtype=torch.float32, device="cuda")
    rp.rp_fill_lawf(S, law, p, out, per)
    torch.cuda.synchronize()
    got = out.cpu().numpy().reshape(n, per)
    ost = [oracle_stream(engine, i) for i in range(n)]
    nz = 0
    for i, o in enumerate(ost):
        ref = laws.draw_f32(o, law, p, per)
        same = (got[i] == ref) | (np.isnan(got[i]) & np.isnan(ref))
        if not same.all():
            d = ulp_diff(got[i][~same], ref[~same])
            assert (np.sign(got[i][~same]) == np.sign(ref[~same])).all()
            assert d.max() <= 2, (engine, i, int(d.max()))
            nz += int((~same).sum())
    assert nz <= max(8, n * per // 2000), nz
    _states_equal(S, engine, ost)


def test_float_law_errors():
    S = make_streams("philox4x32", 4)
    out = torch.empty(16, dtype=torch.float32, device="cuda")
    with pytest.raises(rp.RpError) as ei:
        rp.rp_fill_lawf(S, rp.RP_LAW_BETA, (2.0, -1.0), out, 4)
    assert ei.value.code == rp.RP_EINVAL
    with pytest.raises(rp.RpError) as ei:
        rp.rp_fill_lawf(S, rp.RP_LAW_UNIF, (1.0, 1.0), out, 4)
    assert ei.value.code == rp.RP_EINVAL


@pytest.mark.parametrize("engine", ["ranlux++", "sfc64", "xoro++"])
def test_float_law_lane_bodies(engine):
    """The binary32 laws through the per-lane kernel body (ranlux++) and the
    staged one (sfc64, xoroshiro128++), ziggurat and uniform bases."""
    from tests.gpu_common import ulp_diff
    n, per = 64, 300
    S = make_streams(engine, n)
    ost = [oracle_stream(engine, i) for i in range(n)]
    for law, p in ((rp.RP_LAW_LOGNORMAL, (0.5, 0.75)), (rp.RP_LAW_GUMBEL, (1.0, 2.0)),
                   (rp.RP_LAW_WEIBULL, (1.7, 4.0))):
        out = torch.empty(n * per, dtype=torch.float32, device="cuda")
        rp.rp_fill_lawf(S, law, p, out, per)
        torch.cuda.synchronize()
        got = out.cpu().numpy().reshape(n, per)
        for i, o in enumerate(ost):
            ref = laws.draw_f32(o, law, p, per)
            same = got[i] == ref
            if not same.all():
                assert ulp_diff(got[i][~same], ref[~same]).max() <= 2, (engine, law, i)
    _states_equal(S, engine, ost)



@pytest.mark.parametrize("alpha", [2.5, 0.4])
@pytest.mark.parametrize("engine", ["philox4x32", "pcg64", "x256++", "ranlux++", "chacha20"])
def test_float_gamma_matches_oracle(engine, alpha):
    """The float gamma (rp_fill_lawf, RP_LAW_GAMMA): identical decisions on
    the 32-bit items, binary64 arithmetic on both sides; values equal unless
    the boost's power (about an ulp of binary64 apart) straddles a binary32
    rounding boundary: at most 2 binary32 ulp, and rare."""
    from tests.gpu_common import ulp_diff
    n, per = 64, 400
    S = make_streams(engine, n)
    out = torch.empty(n * per, dtype=torch.float32, device="cuda")
    rp.rp_fill_lawf(S, rp.RP_LAW_GAMMA, (alpha, 1.5), out, per)
    torch.cuda.synchronize()
    got = out.cpu().numpy().reshape(n, per)
    ost = [oracle_stream(engine, i) for i in range(n)]
    nz = 0
    for i, o in enumerate(ost):
        ref = laws.draw_f32(o, rp.RP_LAW_GAMMA, (alpha, 1.5), per)
        same = got[i] == ref
        if not same.all():
            assert ulp_diff(got[i][~same], ref[~same]).max() <= 2, (engine, i)
            nz += int((~same).sum())
    assert nz <= max(8, n * per // 1000), nz
    _states_equal(S, engine, ost)


MIXF = [m for m in MIX if m[0] != rp.RP_LAW_GAMMA]


@pytest.mark.parametrize("law,p", MIXF, ids=[f"law{l}_{'_'.join(str(v) for v in p)}" for l, p in MIXF])
@pytest.mark.parametrize("engine", ["philox4x32", "pcg64", "x256++", "ranlux++"])
def test_float_mix_law_matches_oracle(engine, law, p):
    """rp_fill_lawf for the laws of several draws: float gammas and binary32
    normals on one item stream, the combination in binary64, one rounding.
    Every decision (so every state) is the oracle's; the binary64 values
    differ only through the boost's power and the ziggurat tails (a few
    binary64 ulp), so the binary32 results are equal except where that
    straddles a rounding boundary: at most 2 binary32 ulp, and rare."""
    from tests.gpu_common import ulp_diff
    n = 64
    per = 150 if law in (rp.RP_LAW_T, rp.RP_LAW_F) else 300
    S = make_streams(engine, n)
    out = torch.empty(n * per, dtype=torch.float32, device="cuda")
    rp.rp_fill_lawf(S, law, p, out, per)
    torch.cuda.synchronize()
    got = out.cpu().numpy().reshape(n, per)
    ost = [oracle_stream(engine, i) for i in range(n)]
    nz = 0
    for i, o in enumerate(ost):
        ref = laws.draw_f32(o, law, p, per)
        same = got[i] == ref
        if not same.all():
            assert (np.sign(got[i][~same]) == np.sign(ref[~same])).all()
            assert ulp_diff(got[i][~same], ref[~same]).max() <= 2, (engine, law, i)
            nz += int((~same).sum())
    assert nz <= max(8, n * per // 1000), nz
    _states_equal(S, engine, ost)
