"""C ABI checks that need no GPU: the library loads, exports every function
include/rp.h declares, and its host-side stream control (seeding, setters,
jumps, advance, state get/set, serialization, errors) matches the oracle."""
import ctypes
import os
import re

import numpy as np
import pytest

import oracle
import paper_2605_05099_amd as rp

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ENGINES = ["x256++", "pcg64", "philox4x32", "philox", "sfc64", "ranlux++", "cwg128", "x256++simd", "x256**simd",
           "sfc64simd"]


def declared_functions():
    text = open(os.path.join(ROOT, "include", "rp.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(rp_[a-z0-9_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    names = declared_functions()
    assert len(names) >= 25
    lib = ctypes.CDLL(rp.LIB_PATH)
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_covers_every_declared_symbol():
    assert set(declared_functions()) <= set(rp._SIGS)


def test_engine_query_and_ids():
    txt = rp.rp_engines()
    for e in ENGINES:
        assert e + ":" in txt
    assert rp.rp_engine_id("X256++") == rp.RP_X256PP
    assert rp.rp_engine_id("RANLUX++") == rp.RP_RANLUX
    with pytest.raises(rp.RpError) as ei:
        rp.rp_engine_id("x256")
    assert ei.value.code == rp.RP_EINVAL
    with pytest.raises(rp.RpError):
        rp.rp_create("mt19937")
    # a new stream is randomized: two of them differ; seeding makes them equal
    a, b = rp.rp_create(""), rp.rp_create("x256++")
    assert a.state_words() == b.state_words() == 4
    assert a.get_state()[0] != b.get_state()[0]
    assert a.seed(7).get_state()[0] == b.seed(7).get_state()[0]


def test_randomize_gives_valid_distinct_states():
    for eng in ENGINES:
        r1 = rp.rp_create(eng).randomize()
        r2 = rp.rp_create(eng).randomize()
        assert r1.get_state()[0] != r2.get_state()[0], eng
    # a randomized stream is an ordinary seeded one: re-seeding makes it reproducible
    r = rp.rp_create("pcg64").randomize().seed(99)
    assert r.get_state()[0] == rp.rp_create("pcg64").seed(99).get_state()[0]


def test_full_mantissa_setting():
    """The stream's U(0,1) resolution switch: on by default, kept across
    seeding and randomizing, copied by duplicate, 0 or 1 only."""
    r = rp.rp_create("pcg64")
    assert r.full_mantissa is True
    r.full_mantissa = False
    assert r.full_mantissa is False
    r.seed(3).randomize()
    assert r.full_mantissa is False
    assert r.duplicate().full_mantissa is False
    r.full_mantissa = True
    assert r.full_mantissa is True
    assert rp.lib().rp_set_full_mantissa(r.h, 2) == rp.RP_EINVAL
    assert r.full_mantissa is True
    assert rp.lib().rp_set_full_mantissa(None, 0) == rp.RP_ENULL
    assert rp.lib().rp_get_full_mantissa(None) == rp.RP_ENULL


def test_streams_deserialize_rejects_bad_images():
    """Images that are not a serialized substream set fail before any device
    work: wrong magic, engine, word count, settings, n, phase or length."""
    import struct
    out = ctypes.c_void_p()

    def image(magic=0x31535052, engine=rp.ENGINES["pcg64"], nw=4, fm=1, n=2, words=None, phase=(0, 0)):
        words = [1] * (nw * n) if words is None else words
        return (struct.pack("<4IQ", magic, engine, nw, fm, n) + struct.pack(f"<{len(words)}Q", *words)
                + struct.pack(f"<{len(phase)}I", *phase))

    L = rp.lib()
    for bad in (image(magic=0), image(engine=len(rp.ENGINES)), image(nw=3), image(fm=8),
                image(n=0, words=[], phase=()), image(phase=(0, 1)), image()[:-1], image()[:23]):
        assert L.rp_streams_deserialize(bad, len(bad), ctypes.byref(out)) == rp.RP_EINVAL
        assert not out.value
    assert L.rp_streams_deserialize(None, 64, ctypes.byref(out)) == rp.RP_ENULL
    assert L.rp_streams_serialize(None, None, 0, None) == rp.RP_ENULL


@pytest.mark.parametrize("engine", ENGINES)
@pytest.mark.parametrize("seed,key", [(42, ()), (12345, ()), (42, (0,)), (42, (7, 8, 9)), (2**64 - 1, (1,))])
def test_seeding_matches_oracle(engine, seed, key):
    r = rp.rp_create(engine).seed(seed, key)
    o = oracle.Stream.seeded(engine, seed, key)
    w, ph = r.get_state()
    assert w == o.state[:len(w)] and ph == o.phase
    assert (r.raw_host(40) == o.raw(40)).all()


@pytest.mark.parametrize("engine", ["x256++", "pcg64", "philox4x32", "philox", "ranlux++"])
@pytest.mark.parametrize("n", [1, 5, 1000, 2**64 + 17, 3 * 2**70 + 1])
def test_advance_matches_oracle(engine, n):
    r = rp.rp_create(engine).seed(7).advance(n)
    o = oracle.Stream.seeded(engine, 7).advance(n)
    assert r.get_state()[0] == o.state[:rp.STATE_WORDS[rp.ENGINES[engine]]]


@pytest.mark.parametrize("engine", ["x256++", "philox", "ranlux++"])
@pytest.mark.parametrize("k", [32, 64, 96, 128, 192])
def test_jump_matches_oracle(engine, k):
    r = rp.rp_create(engine).seed(9).jump(k)
    o = oracle.Stream.seeded(engine, 9).advance(2**k)
    assert r.get_state()[0] == o.state[:rp.STATE_WORDS[rp.ENGINES[engine]]]


def test_jump_errors():
    with pytest.raises(rp.RpError) as ei:
        rp.rp_create("x256++").jump(5)
    assert ei.value.code == rp.RP_EINVAL
    with pytest.raises(rp.RpError) as ei:
        rp.rp_create("sfc64").jump(64)
    assert ei.value.code == rp.RP_EUNSUPPORTED
    with pytest.raises(rp.RpError) as ei:
        rp.rp_create("pcg64").jump(128)
    assert ei.value.code == rp.RP_EINVAL
    with pytest.raises(rp.RpError) as ei:
        rp.rp_create("sfc64").advance(3)
    assert ei.value.code == rp.RP_EUNSUPPORTED


def test_setters_match_oracle():
    r = rp.rp_create("pcg64").seed(1).pcg64_set_inc(2**70 + 4)
    o = oracle.Stream.seeded("pcg64", 1).pcg64_set_inc(2**70 + 4)
    assert r.get_state()[0] == o.state[:4]
    r = rp.rp_create("philox").seed(1).philox_set_key(5, 6)
    o = oracle.Stream.seeded("philox", 1).philox_set_key(5, 6)
    assert r.get_state()[0] == o.state[:6]
    r = rp.rp_create("philox4x32").seed(1).philox_set_key(2**40 + 3)
    o = oracle.Stream.seeded("philox4x32", 1).philox_set_key(2**40 + 3)
    assert r.get_state()[0] == o.state[:3]
    r = rp.rp_create("sfc64").sfc64_set_abc(1, 2, 3)
    o = oracle.Stream("sfc64").sfc64_set_abc(1, 2, 3)
    assert r.get_state()[0] == o.state[:4]
    r = rp.rp_create("cwg128").seed(1).cwg128_set_weyl(2**90 + 6)
    o = oracle.Stream.seeded("cwg128", 1).cwg128_set_weyl(2**90 + 6)
    assert r.get_state()[0] == o.state[:8]
    assert r.get_state()[0][6:] == [7, 2**26]   # made odd
    assert (r.raw_host(50) == o.raw(50)).all()
    with pytest.raises(rp.RpError) as ei:
        rp.rp_create("pcg64").cwg128_set_weyl(3)
    assert ei.value.code == rp.RP_EUNSUPPORTED
    with pytest.raises(rp.RpError) as ei:
        rp.rp_create("x256++").pcg64_set_inc(3)
    assert ei.value.code == rp.RP_EUNSUPPORTED


@pytest.mark.parametrize("engine", ENGINES)
def test_state_roundtrip_phase_and_duplicate(engine):
    r = rp.rp_create(engine).seed(3)
    r.raw_host(7)  # leaves a phase for block engines
    w, ph = r.get_state()
    o = oracle.Stream.seeded(engine, 3)
    o.raw(7)
    assert ph == o.phase and w == o.state[:len(w)]
    d = r.duplicate()
    s = rp.rp_create(engine).set_state(w, ph)
    blob = r.serialize()
    t = rp.rp_create("x256++").deserialize(blob)
    ref = r.raw_host(50)
    assert (d.raw_host(50) == ref).all()
    assert (s.raw_host(50) == ref).all()
    assert (t.raw_host(50) == ref).all()


def test_set_state_errors():
    r = rp.rp_create("philox4x32")
    with pytest.raises(rp.RpError):
        r.set_state([1, 2, 3], phase=2)
    with pytest.raises(rp.RpError):
        r.set_state([1, 2])
    with pytest.raises(rp.RpError):
        rp.rp_create("x256++").deserialize(b"\0" * 200)


@pytest.mark.parametrize("d", [1, 5, 64, 200])
def test_cholesky_matches_library(d):
    """rp_cholesky (host, binary64) against LAPACK via numpy; only the lower
    triangle of Sigma is read."""
    from paper_2605_05099_amd import workloads
    sigma = workloads.mvn(d)["sigma"] if d > 1 else np.array([[2.5]])
    L = rp.rp_cholesky(sigma)
    ref = np.linalg.cholesky(sigma)
    np.testing.assert_allclose(L, ref, rtol=1e-10, atol=1e-12 * np.abs(ref).max())
    assert (np.triu(L, 1) == 0).all()
    garbage = sigma + np.triu(np.full_like(sigma, 7.0), 1)
    assert np.array_equal(rp.rp_cholesky(garbage), L)


def test_cholesky_errors():
    for bad in (np.array([[1.0, 0.0], [3.0, 1.0]]), np.array([[0.0]]), np.array([[np.nan]]),
                -np.eye(3)):
        with pytest.raises(rp.RpError) as ei:
            rp.rp_cholesky(bad)
        assert ei.value.code == rp.RP_ENOTSPD


RL_M = 2**576 - 2**240 + 1


def _rl_words(x):
    return [(x >> (64 * k)) & (2**64 - 1) for k in range(9)]


def _rl_value(words):
    return sum(int(w) << (64 * k) for k, w in enumerate(words))


@pytest.mark.parametrize("x", [1, 2, RL_M - 1, RL_M - 2, 2**575, 2**551 - 1, 2**551, 2**240 - 1, 2**240,
                               (RL_M - 1) // 3, 2**576 - 2**241])
def test_ranlux_step_edge_states(x):
    """The folded-table step (29-bit limbs) against the oracle on states that
    stress the folds: near m, powers of two at limb and fold boundaries."""
    r = rp.rp_create("ranlux++").set_state(_rl_words(x))
    o = oracle.Stream.from_state("ranlux++", _rl_words(x))
    assert (r.raw_host(9 * 30) == o.raw(9 * 30)).all()


def test_ranlux_step_is_power_of_the_lcg_multiplier():
    """From state 1 block k is A^k mod m with A = a^2048, a = m - (m - 1)/2^24
    (ranlux++ as the LCG equivalent of RANLUX, b = 2^24, r = 24)."""
    a = RL_M - (RL_M - 1) // 2**24
    A = pow(a, 2048, RL_M)
    w = rp.rp_create("ranlux++").set_state(_rl_words(1)).raw_host(9 * 50)
    for k in range(50):
        assert _rl_value(w[9 * k: 9 * k + 9]) == pow(A, k + 1, RL_M)


def test_ranlux_long_host_draw_matches_oracle():
    r = rp.rp_create("ranlux++").seed(2024)
    o = oracle.Stream.seeded("ranlux++", 2024)
    assert (r.raw_host(9 * 3000 + 5) == o.raw(9 * 3000 + 5)).all()


ALL_ENGINES = list(rp.ENGINES)
# exclusive bound on k for jumps by 2^k steps (the period of one stream)
JUMP_LIMIT = {"x256++": 256, "x256**": 256, "philox": 256, "ranlux++": 256, "pcg64": 128, "philox4x32": 128,
              "xoro++": 128, "x128+": 128, "squares": 64, "chacha20": 32, "sfc64": 0, "cwg128": 0,
              "x256++simd": 253, "x256**simd": 253, "sfc64simd": 0}


@pytest.mark.parametrize("engine", ALL_ENGINES)
def test_jump_bounds_follow_the_period(engine):
    """rp_jump accepts 2^k only below the period of one stream, and
    rp_streams_create's JUMP family the same k (checked before any device
    work), so that no accepted jump can make substreams coincide."""
    lim = JUMP_LIMIT[engine]
    for k in (32, 64, 96, 128, 192):
        r = rp.rp_create(engine).seed(5)
        if lim == 0:
            assert rp.lib().rp_jump(r.h, k) == rp.RP_EUNSUPPORTED
        elif k >= lim:
            assert rp.lib().rp_jump(r.h, k) == rp.RP_EINVAL
            assert r.get_state()[0] == rp.rp_create(engine).seed(5).get_state()[0]
        else:
            r.jump(k)
            o = oracle.Stream.seeded(engine, 5).advance(2**k)
            assert r.get_state()[0] == o.state[:rp.STATE_WORDS[rp.ENGINES[engine]]], k
            assert r.get_state()[0] != rp.rp_create(engine).seed(5).get_state()[0]
    base = rp.rp_create(engine).seed(5)
    out = ctypes.c_void_p()
    bad = [-1, max(lim, 1), 256, 1000]
    for k in bad:
        rc = rp.lib().rp_streams_create(base.h, rp.RP_SUB_JUMP, 4, k, ctypes.byref(out))
        assert rc == (rp.RP_EUNSUPPORTED if lim == 0 else rp.RP_EINVAL), (engine, k, rc)
        assert not out.value


def test_set_state_rejects_states_seeding_never_makes():
    cases = [("x256++", [0, 0, 0, 0]), ("x256**", [0, 0, 0, 0]), ("xoro++", [0, 0]), ("x128+", [0, 0]),
             ("pcg64", [1, 2, 4, 0]), ("squares", [7, 10]), ("cwg128", [1, 2, 3, 4, 5, 6, 8, 0]),
             ("x256++simd", [k + 1 for k in range(12)] + [0, 0, 0, 0] + [5] * 16),
             ("ranlux++", _rl_words(0)),
             ("ranlux++", _rl_words(RL_M)), ("ranlux++", _rl_words(2**576 - 1))]
    for engine, words in cases:
        r = rp.rp_create(engine).seed(1)
        before = r.get_state()
        w = np.asarray(words, dtype=np.uint64)
        assert rp.lib().rp_set_state(r.h, w.ctypes.data_as(ctypes.c_void_p), len(w), 0) == rp.RP_EINVAL, engine
        assert "not a state" in r.last_error()
        assert r.get_state() == before
        # the same words in a stream image are refused as well
        img = bytearray(rp.rp_create(engine).seed(1).serialize())
        img[16:16 + 8 * len(words)] = w.tobytes()
        assert rp.lib().rp_deserialize(r.h, bytes(img), len(img)) == rp.RP_EINVAL
    # the nearest valid states are accepted
    rp.rp_create("x256++").set_state([0, 0, 0, 1])
    rp.rp_create("pcg64").set_state([1, 2, 3, 0])
    rp.rp_create("squares").set_state([7, 11])
    rp.rp_create("cwg128").set_state([1, 2, 3, 4, 5, 6, 9, 0])
    rp.rp_create("ranlux++").set_state(_rl_words(RL_M - 1))


def test_deserialize_rejects_long_keys_and_stray_words():
    import struct
    r = rp.rp_create("pcg64").seed(3, (1, 2))
    img = bytearray(r.serialize())
    ok = rp.rp_create("pcg64").deserialize(bytes(img))
    assert ok.get_state() == r.get_state()
    long_key = bytearray(img)
    long_key[12:16] = struct.pack("<I", 1025)
    long_key += b"\0" * (1025 * 4)
    assert rp.lib().rp_deserialize(ok.h, bytes(long_key), len(long_key)) == rp.RP_EINVAL
    stray = bytearray(img)
    stray[16 + 8 * 5: 16 + 8 * 6] = struct.pack("<Q", 9)  # word 5 of a 4-word engine
    assert rp.lib().rp_deserialize(ok.h, bytes(stray), len(stray)) == rp.RP_EINVAL


def test_streams_deserialize_rejects_invalid_states():
    import struct
    out = ctypes.c_void_p()
    for engine, words in (("x256++", [0, 1, 0, 2, 0, 3, 0, 4]), ("pcg64", [1, 1, 2, 2, 3, 2, 0, 0])):
        img = (struct.pack("<4IQ", 0x31535052, rp.ENGINES[engine], 4, 1, 2) + struct.pack("<8Q", *words)
               + struct.pack("<2I", 0, 0))
        # x256++: substream 0 is all zero (words 0, 2, 4, 6 of the SoA image);
        # pcg64: substream 1 has the even increment 2
        assert rp.lib().rp_streams_deserialize(img, len(img), ctypes.byref(out)) == rp.RP_EINVAL, engine
        assert not out.value
        assert "not a state" in rp.rp_errmsg()


def test_settings_flags():
    """rp_set_flag / rp_get_flag: the full-mantissa setting and the squeeze,
    both on by default, and bitexact, off by default; 0 or 1 only, copied by
    duplicate, kept by seeding."""
    r = rp.rp_create("philox4x32")
    assert r.get_flag(rp.RP_FULL_MANTISSA) and r.get_flag(rp.RP_SQUEEZE)
    assert r.get_flag(rp.RP_BITEXACT) == 0
    r.set_flag(rp.RP_BITEXACT, 1).seed(5)
    assert r.get_flag(rp.RP_BITEXACT) == 1 and r.duplicate().get_flag(rp.RP_BITEXACT) == 1
    r.set_flag(rp.RP_BITEXACT, 0)
    r.set_flag(rp.RP_SQUEEZE, 0).seed(4)
    assert not r.get_flag(rp.RP_SQUEEZE) and r.get_flag(rp.RP_FULL_MANTISSA)
    assert not r.duplicate().get_flag(rp.RP_SQUEEZE)
    r.set_flag(rp.RP_FULL_MANTISSA, 0)
    assert r.full_mantissa is False
    L = rp.lib()
    assert L.rp_set_flag(r.h, 4, 1) == rp.RP_EINVAL
    assert L.rp_set_flag(r.h, rp.RP_BITEXACT, 2) == rp.RP_EINVAL
    assert L.rp_set_flag(r.h, rp.RP_SQUEEZE, 2) == rp.RP_EINVAL
    assert L.rp_get_flag(r.h, 0) == rp.RP_EINVAL
    assert L.rp_set_flag(None, rp.RP_SQUEEZE, 1) == rp.RP_ENULL
    assert L.rp_streams_set_flag(None, rp.RP_SQUEEZE, 1) == rp.RP_ENULL
    assert L.rp_streams_get_flag(None, rp.RP_SQUEEZE) == rp.RP_ENULL
