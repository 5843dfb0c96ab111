"""GPU parity of rp_fill against the oracle (needs an MI355X).

Bit-exact for raw words, uniforms and bounded integers.  For the ziggurat the
accept/reject decisions must all agree, which shows as the two sequences
staying aligned; values are then equal except in the tail, where log1p may
differ by an ulp (tolerance: 4 ulp; for the float draws 4 binary32 ulp, and
a tail value rounds to binary32 identically unless log1p's last-bit
difference straddles a binary32 rounding boundary).  The substream states
left behind must equal the oracle's after the same draws, so a second call
continues exactly.
"""
import numpy as np
import pytest

import oracle
import paper_2605_05099_amd as rp
from paper_2605_05099_amd import workloads
from tests.gpu_common import ENGINES, FAMILY, NP_VIEW, TORCH_DTYPE, make_streams, oracle_fill, oracle_stream, ulp_diff

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

CASES = [
    (rp.RP_RAW, rp.RP_U64, 0, 0),
    (rp.RP_RAW, rp.RP_U32, 0, 0),
    (rp.RP_U01, rp.RP_F64, 0, 0),
    (rp.RP_U01, rp.RP_F64, 0, rp.RP_FLAG_52BIT),
    (rp.RP_U01, rp.RP_F32, 0, 0),
    (rp.RP_U01, rp.RP_F32, 0, rp.RP_FLAG_52BIT),
    (rp.RP_BOUNDED, rp.RP_U64, 6, 0),
    (rp.RP_BOUNDED, rp.RP_U64, 6 * 10**18, 0),
    (rp.RP_BOUNDED, rp.RP_U64, 0, 0),
    (rp.RP_BOUNDED, rp.RP_U32, 3 * 10**9, 0),
    (rp.RP_BOUNDED, rp.RP_U32, 2**31, 0),
    (rp.RP_NORM, rp.RP_F64, 0, 0),
    (rp.RP_EXP, rp.RP_F64, 0, 0),
    (rp.RP_NORM, rp.RP_F32, 0, 0),
    (rp.RP_EXP, rp.RP_F32, 0, 0),
]


def _gpu_fill(S, dist, dtype, per, bound, flags):
    t = torch.empty(len(S) * per, dtype=getattr(torch, TORCH_DTYPE[dtype]), device="cuda")
    rp.rp_fill(S, dist, dtype, bound, flags, t, per)
    torch.cuda.synchronize()
    return t.cpu().numpy().view(NP_VIEW[dtype]).reshape(len(S), per)


def _compare(got, ref, dist):
    if dist in (rp.RP_NORM, rp.RP_EXP):
        assert got.shape == ref.shape
        d = ulp_diff(got, ref)
        assert (np.sign(got) == np.sign(ref)).all()
        assert d.max() <= 4, d.max()
        # only tail values (|x| beyond the ziggurat radius) may differ at all
        r = 3.6541528853610088 if dist == rp.RP_NORM else 7.69711747013105
        assert (np.abs(ref[d > 0]) >= r).all()
    else:
        assert np.array_equal(got, ref)


def _states_equal(S, engine, ostreams):
    words, phase = S.get()
    nw = rp.STATE_WORDS[rp.ENGINES[engine]]
    for i, o in ostreams.items():
        assert [int(words[k, i]) for k in range(nw)] == o.state[:nw], (engine, i)
        assert int(phase[i]) == o.phase, (engine, i)


@pytest.mark.parametrize("engine", ENGINES)
@pytest.mark.parametrize("case", CASES, ids=lambda c: f"d{c[0]}t{c[1]}b{c[2]}f{c[3]}")
def test_fill_matches_oracle(engine, case):
    dist, dtype, bound, flags = case
    n = 67 if engine not in ("ranlux++",) else 37   # ragged: not a multiple of 4 or 64
    S = make_streams(engine, n)
    ostreams = {i: oracle_stream(engine, i) for i in range(n)}
    for per in (129, 1, 333):   # successive calls continue each substream
        got = _gpu_fill(S, dist, dtype, per, bound, flags)
        for i in range(n):
            ref = oracle_fill(ostreams[i], dist, dtype, per, bound, flags)
            _compare(got[i], ref, dist)
        _states_equal(S, engine, ostreams)


@pytest.mark.parametrize("engine", ["philox4x32", "pcg64", "philox"])
@pytest.mark.parametrize("dtype", [rp.RP_F64, rp.RP_F32])
def test_ziggurat_long_run_with_tails(engine, dtype):
    """Enough normals to cross many chunks and hit the tail path in the
    wavefront kernel (tail probability 2.6e-4 per sample)."""
    n, per = 20, 20000
    S = make_streams(engine, n)
    got = _gpu_fill(S, rp.RP_NORM, dtype, per, 0, 0)
    tails = 0
    for i in range(n):
        o = oracle_stream(engine, i)
        ref = o.norm(per) if dtype == rp.RP_F64 else o.normf(per)
        _compare(got[i], ref, rp.RP_NORM)
        tails += int((np.abs(ref) > 3.6541528853610088).sum())
    assert tails > 30


@pytest.mark.parametrize("dist", [rp.RP_NORM, rp.RP_EXP])
@pytest.mark.parametrize("engine", ["philox4x32", "pcg64", "philox", "squares"])
def test_ziggurat_tails_across_ragged_calls(engine, dist):
    """The store-order ziggurat over successive calls of ragged lengths (a
    call ending inside a group of 128 positions, samples carried across
    chunks and calls) with a few hundred tail draws among them: a tail's
    value written after the walk, the walk taken only by groups where a
    normal tail starts.  Values, decisions and states equal the oracle's."""
    n = 400
    S = make_streams(engine, n)
    ost = {i: oracle_stream(engine, i) for i in range(n)}
    r = 3.6541528853610088 if dist == rp.RP_NORM else 7.69711747013105
    tails = 0
    for per in (1, 2, 7, 64, 130, 511, 512, 513, 1000):
        got = _gpu_fill(S, dist, rp.RP_F64, per, 0, 0)
        for i in range(n):
            ref = oracle_fill(ost[i], dist, rp.RP_F64, per)
            _compare(got[i], ref, dist)
            tails += int((np.abs(ref) > r).sum())
        _states_equal(S, engine, ost)
    assert tails > 100


@pytest.mark.parametrize("engine", ["philox4x32", "pcg64", "philox", "x256++", "sfc64"])
def test_float_exponential_long_run_with_tails(engine):
    """Float exponentials over many chunks; the tail (P = 4.5e-4) included."""
    n, per = 16, 20000
    S = make_streams(engine, n)
    got = _gpu_fill(S, rp.RP_EXP, rp.RP_F32, per, 0, 0)
    tails = 0
    ost = {}
    for i in range(n):
        ost[i] = oracle_stream(engine, i)
        ref = ost[i].expf(per)
        _compare(got[i], ref, rp.RP_EXP)
        tails += int((ref > 7.69711747013105).sum())
    assert tails > 50
    _states_equal(S, engine, ost)


def test_zero_and_invalid():
    S = make_streams("philox4x32", 8)
    before = S.get()[0].copy()
    t = torch.empty(0, dtype=torch.float64, device="cuda")
    rp.rp_fill(S, rp.RP_NORM, rp.RP_F64, 0, 0, t, 0)    # per_stream = 0 is a no-op
    assert (S.get()[0] == before).all()
    with pytest.raises(rp.RpError) as ei:
        rp.rp_fill(S, rp.RP_NORM, rp.RP_U64, 0, 0, torch.empty(8, dtype=torch.int64, device="cuda"), 1)
    assert ei.value.code == rp.RP_EUNSUPPORTED
    with pytest.raises(rp.RpError) as ei:
        rp.rp_fill(S, rp.RP_NORM, rp.RP_F64, 0, 0, 0, 4)
    assert ei.value.code == rp.RP_ENULL
    with pytest.raises(rp.RpError) as ei:
        rp.rp_fill(S, rp.RP_BOUNDED, rp.RP_U32, 2**40, 0, torch.empty(8, dtype=torch.int32, device="cuda"), 1)
    assert ei.value.code == rp.RP_EUNSUPPORTED


@pytest.mark.parametrize("engine,kind", [("philox4x32", "key"), ("pcg64", "inc")])
@pytest.mark.parametrize("dist,dtype", [(rp.RP_RAW, rp.RP_U64), (rp.RP_U01, rp.RP_F32), (rp.RP_U01, rp.RP_F64),
                                        (rp.RP_NORM, rp.RP_F64), (rp.RP_EXP, rp.RP_F64),
                                        (rp.RP_NORM, rp.RP_F32), (rp.RP_EXP, rp.RP_F32)])
def test_full_size_substreams_sampled(engine, kind, dist, dtype):
    """2^16 substreams x 2^14 values (the benchmark's launch); 258 substreams
    checked in full against the oracle."""
    n, per = workloads.SUB_N, workloads.SUB_PER
    S = make_streams(engine, n)
    t = torch.empty(n * per, dtype=getattr(torch, TORCH_DTYPE[dtype]), device="cuda")
    rp.rp_fill(S, dist, dtype, 0, 0, t, per)
    idx = workloads.sampled_substreams(n)
    rows = t.view(n, per).index_select(0, torch.as_tensor(idx, device="cuda")).cpu().numpy().view(NP_VIEW[dtype])
    del t
    for r, i in zip(rows, idx):
        ref = oracle_fill(oracle_stream(engine, i), dist, dtype, per)
        _compare(r, ref, dist)


@pytest.mark.parametrize("engine", ["philox4x32", "pcg64", "x256++", "sfc64"])
@pytest.mark.parametrize("dtype", [rp.RP_F64, rp.RP_F32])
def test_full_mantissa_off_selects_method_2(engine, dtype):
    """A stream with the full-mantissa setting off gives method-2 uniforms
    (as RP_FLAG_52BIT does) from its substream sets, which keep the setting
    they were created with, and from the one-stream split."""
    kind, _ = FAMILY[engine]
    base = rp.rp_create(engine).seed(42)
    base.full_mantissa = False
    S = rp.rp_streams_create(base, kind, 300, 64)
    base.full_mantissa = True
    got = _gpu_fill(S, rp.RP_U01, dtype, 777, 0, 0)
    for i in (0, 1, 150, 299):
        ref = oracle_fill(oracle_stream(engine, i), rp.RP_U01, dtype, 777, 0, rp.RP_FLAG_52BIT)
        assert np.array_equal(got[i], ref)
    rng = rp.rp_create(engine).seed(7)
    rng.full_mantissa = False
    o = oracle.Stream.seeded(engine, 7)
    t = torch.empty(40001, dtype=getattr(torch, TORCH_DTYPE[dtype]), device="cuda")
    rp.rp_fill_serial(rng, rp.RP_U01, dtype, 0, 0, t, 40001)
    torch.cuda.synchronize()
    ref = oracle_fill(o, rp.RP_U01, dtype, 40001, 0, rp.RP_FLAG_52BIT)
    assert np.array_equal(t.cpu().numpy().view(NP_VIEW[dtype]), ref)


@pytest.mark.parametrize("engine", ["philox4x32", "pcg64", "ranlux++", "chacha20", "x256++"])
def test_streams_serialize_resumes_exactly(engine):
    """A substream set restored from its byte image continues exactly as the
    original does, partly used blocks and the full-mantissa setting included."""
    kind, _ = FAMILY[engine]
    base = rp.rp_create(engine).seed(42)
    base.full_mantissa = False
    S = rp.rp_streams_create(base, kind, 1000, 64)
    _gpu_fill(S, rp.RP_NORM, rp.RP_F64, 333, 0, 0)
    img = S.serialize()
    assert len(img) == 24 + 8 * rp.STATE_WORDS[S.engine] * 1000 + 4 * 1000
    a = _gpu_fill(S, rp.RP_U01, rp.RP_F64, 777, 0, 0)
    T = rp.rp_streams_deserialize(img)
    assert T.engine == S.engine and len(T) == len(S)
    b = _gpu_fill(T, rp.RP_U01, rp.RP_F64, 777, 0, 0)
    assert np.array_equal(a, b)
    ws, ps = S.get()
    wt, pt = T.get()
    assert (ws == wt).all() and (ps == pt).all()
    for i in (0, 999):
        o = oracle_stream(engine, i)
        o.norm(333)
        assert np.array_equal(b[i], oracle_fill(o, rp.RP_U01, rp.RP_F64, 777, 0, rp.RP_FLAG_52BIT))
    with pytest.raises(rp.RpError) as ei:
        rp.rp_streams_deserialize(img[:-4])
    assert ei.value.code == rp.RP_EINVAL
