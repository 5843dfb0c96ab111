"""GPU split of one stream over many lanes against the serial oracle (MI355X).

rp_fill_serial must return exactly what n serial calls on the stream return
(bit-exact for raw bits, uniforms and bounded integers; ziggurat values
within 4 ulp, tails only) and leave the stream where those calls leave it.
The x256++ case at 10^6 values per output is the one-stream workload of the
plain method (seed 12345, each output from a freshly seeded stream).
"""
import numpy as np
import pytest

import oracle
import paper_2605_05099_amd as rp
from tests.gpu_common import NP_VIEW, TORCH_DTYPE, oracle_fill, ulp_diff

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

ENGINES = ["x256++", "pcg64", "philox4x32", "philox", "ranlux++", "sfc64", "x256**", "squares", "chacha20",
           "xoro++", "x128+", "cwg128", "x256++simd", "x256**simd", "sfc64simd"]
CASES = [
    (rp.RP_RAW, rp.RP_U64, 0, 0),
    (rp.RP_RAW, rp.RP_U32, 0, 0),
    (rp.RP_U01, rp.RP_F64, 0, 0),
    (rp.RP_U01, rp.RP_F32, 0, rp.RP_FLAG_52BIT),
    (rp.RP_BOUNDED, rp.RP_U64, 6, 0),
    (rp.RP_BOUNDED, rp.RP_U64, 6 * 10**18, 0),
    (rp.RP_BOUNDED, rp.RP_U32, 3 * 10**9, 0),
    (rp.RP_BOUNDED, rp.RP_U64, 0, 0),
    (rp.RP_NORM, rp.RP_F64, 0, 0),
    (rp.RP_EXP, rp.RP_F64, 0, 0),
    (rp.RP_NORM, rp.RP_F32, 0, 0),
    (rp.RP_EXP, rp.RP_F32, 0, 0),
]


def _gpu(rng, dist, dtype, bound, flags, n):
    t = torch.empty(max(n, 1), dtype=getattr(torch, TORCH_DTYPE[dtype]), device="cuda")
    rp.rp_fill_serial(rng, dist, dtype, bound, flags, t, n)
    torch.cuda.synchronize()
    return t.cpu().numpy().view(NP_VIEW[dtype])[:n]


def _compare(got, ref, dist):
    assert got.shape == ref.shape
    if dist in (rp.RP_NORM, rp.RP_EXP):
        d = ulp_diff(got, ref)
        assert d.max() <= 4, int(d.max())
        r = 3.6541528853610088 if dist == rp.RP_NORM else 7.69711747013105
        assert (np.abs(ref[d > 0]) >= r).all()
    else:
        assert np.array_equal(got, ref)


def _same_state(rng, o):
    words, phase = rng.get_state()
    assert words == o.state[: len(words)] and phase == o.phase


@pytest.mark.parametrize("engine", ENGINES)
@pytest.mark.parametrize("case", CASES, ids=lambda c: f"d{c[0]}t{c[1]}b{c[2]}f{c[3]}")
def test_serial_matches_oracle(engine, case):
    dist, dtype, bound, flags = case
    rng = rp.rp_create(engine).seed(7)
    o = oracle.Stream.seeded(engine, 7)
    if engine in ("sfc64", "cwg128", "sfc64simd"):   # no jump: move on by drawing
        rng.raw_host(3)
        o.raw(3)
    else:
        rng.advance(3)
        o.advance(3)
    if engine in ("philox4x32", "philox", "ranlux++", "chacha20", "x256++simd", "x256**simd", "sfc64simd"):
        rng.raw_host(1)                 # and with a partly used block
        o.raw(1)
    for n in (1, 777, 40001):           # successive calls continue the stream
        got = _gpu(rng, dist, dtype, bound, flags, n)
        _compare(got, oracle_fill(o, dist, dtype, n, bound, flags), dist)
        _same_state(rng, o)


@pytest.mark.parametrize("what", ["raw", "u01", "norm", "exp", "normf", "expf"])
def test_one_stream_workload(what):
    """x256++ from seed 12345, 10^6 values; each output from a fresh stream."""
    n = 10**6
    dist, dtype = {"raw": (rp.RP_RAW, rp.RP_U64), "u01": (rp.RP_U01, rp.RP_F64),
                   "norm": (rp.RP_NORM, rp.RP_F64), "exp": (rp.RP_EXP, rp.RP_F64),
                   "normf": (rp.RP_NORM, rp.RP_F32), "expf": (rp.RP_EXP, rp.RP_F32)}[what]
    rng = rp.rp_create("x256++").seed(12345)
    got = _gpu(rng, dist, dtype, 0, 0, n)
    o = oracle.Stream.seeded("x256++", 12345)
    _compare(got, oracle_fill(o, dist, dtype, n), dist)
    _same_state(rng, o)


def test_serial_errors():
    rng = rp.rp_create("x256++").seed(1)
    t = torch.empty(4, dtype=torch.float64, device="cuda")
    with pytest.raises(rp.RpError) as ei:
        rp.rp_fill_serial(rng, rp.RP_NORM, rp.RP_U64, 0, 0, t, 4)
    assert ei.value.code == rp.RP_EUNSUPPORTED
    with pytest.raises(rp.RpError) as ei:
        rp.rp_fill_serial(rng, rp.RP_RAW, rp.RP_U64, 0, 0, 0, 4)
    assert ei.value.code == rp.RP_ENULL
    before = rng.get_state()
    rp.rp_fill_serial(rng, rp.RP_RAW, rp.RP_U64, 0, 0, t, 0)
    assert rng.get_state() == before


@pytest.mark.parametrize("engine", ["x256++", "pcg64", "ranlux++"])
def test_serial_many_lanes(engine):
    """2^27 raw words (2^16 lanes, 1024 wavefronts of jump levels) and 2^24
    normals (about 2^15 chunks of stitching) against the serial stream."""
    rng = rp.rp_create(engine).seed(5)
    o = oracle.Stream.seeded(engine, 5)
    n = 2**27 if engine != "ranlux++" else 2**24
    got = _gpu(rng, rp.RP_RAW, rp.RP_U64, 0, 0, n)
    assert np.array_equal(got, o.raw(n))
    del got
    _same_state(rng, o)
    m = 2**24 if engine != "ranlux++" else 2**21
    got = _gpu(rng, rp.RP_NORM, rp.RP_F64, 0, 0, m)
    _compare(got, o.norm(m), rp.RP_NORM)
    _same_state(rng, o)


@pytest.mark.parametrize("dist,dtype", [(rp.RP_RAW, rp.RP_U64), (rp.RP_U01, rp.RP_F64)])
def test_serial_wavefront_runs_ragged(dist, dtype):
    """2^16 lanes of 1001 words (not a multiple of the 16-value runs the
    wavefront writes together) with a partial last wavefront: the staged runs,
    the per-lane remainders and the per-lane path must all land in place."""
    n = 2**16 * 1000 + 12345
    rng = rp.rp_create("x256++").seed(77)
    o = oracle.Stream.seeded("x256++", 77)
    got = _gpu(rng, dist, dtype, 0, 0, n)
    ref = o.raw(n) if dist == rp.RP_RAW else o.u01(n)
    assert np.array_equal(got, ref)
    del got, ref
    _same_state(rng, o)


@pytest.mark.parametrize("engine", ["x256++", "philox4x32"])
def test_serial_float_ziggurat_many_lanes(engine):
    """2^24 binary32 normals, then 2^24 binary32 exponentials, from one
    stream split over lanes: about 2^15 stitched chunks of 32-bit items."""
    rng = rp.rp_create(engine).seed(11)
    o = oracle.Stream.seeded(engine, 11)
    m = 2**24
    got = _gpu(rng, rp.RP_NORM, rp.RP_F32, 0, 0, m)
    _compare(got, o.normf(m), rp.RP_NORM)
    _same_state(rng, o)
    got = _gpu(rng, rp.RP_EXP, rp.RP_F32, 0, 0, m)
    _compare(got, o.expf(m), rp.RP_EXP)
    _same_state(rng, o)
