"""Reference oracle for the Randompack hot path -- TEST INFRASTRUCTURE ONLY.

Plain, slow CPU implementations of what the GPU library computes, written from
the paper (Randompack, arXiv 2605.05099) and pinned in tests/test_oracle_*.py.
Only the test suite, ``__graft_entry__.smoke`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package; the product path never does.

The C core is ``oracle/oracle.c`` (built into ``liboracle.so`` by
``oracle/build.py``); this module wraps it with ctypes and adds the stream
construction recipes (seeding, stream setters, jumps) used by the workloads.
"""
import ctypes
import functools
import os

import numpy as np

from . import build as _build
from . import jumppoly

(X256PP, PCG64, PHILOX4X32, PHILOX4X64, SFC64, RANLUX, X256SS, SQUARES, XORO128PP, XS128P, CHACHA20, CWG128,
 X256PPS, X256SSS, SFC64S) = range(15)
ENGINE_IDS = {"x256++": X256PP, "x256**": X256SS, "squares": SQUARES, "xoro++": XORO128PP, "x128+": XS128P,
              "chacha20": CHACHA20, "cwg128": CWG128,
              "x256++simd": X256PPS, "x256**simd": X256SSS, "sfc64simd": SFC64S,
              "pcg64": PCG64, "philox4x32": PHILOX4X32,
              "philox": PHILOX4X64, "sfc64": SFC64, "ranlux++": RANLUX}

_lib = None


def lib():
    global _lib
    if _lib is None:
        path = _build.build()
        _lib = ctypes.CDLL(path)
        vp, sz, u64 = ctypes.c_void_p, ctypes.c_size_t, ctypes.c_uint64
        sig = {
            "or_stream_words": ([], sz), "or_counts_words": ([], sz),
            "or_seed": ([vp, u64, u64, vp, sz], ctypes.c_int),
            "or_set_state": ([vp, u64, vp, sz, u64], ctypes.c_int),
            "or_pcg64_set_inc": ([vp, u64, u64], ctypes.c_int),
            "or_philox_set_key": ([vp, u64, u64], ctypes.c_int),
            "or_sfc64_set_abc": ([vp, u64, u64, u64], None),
            "or_squares_set_key": ([vp, u64], ctypes.c_int),
            "or_chacha20_set_nonce": ([vp, u64, u64], ctypes.c_int),
            "or_cwg128_set_weyl": ([vp, u64, u64], ctypes.c_int),
            "or_chacha_qr": ([vp], None),
            "or_x256_apply_poly": ([vp, vp], ctypes.c_int),
            "or_x256_linear_steps": ([vp, vp, sz], None),
            "or_x128_linear_steps": ([u64, vp, vp, sz], ctypes.c_int),
            "or_x128_apply_poly": ([vp, vp], ctypes.c_int),
            "or_pcg64_advance": ([vp, u64, u64], ctypes.c_int),
            "or_philox_advance": ([vp, vp], ctypes.c_int),
            "or_ranlux_advance": ([vp, vp], ctypes.c_int),
            "or_raw64": ([vp, vp, sz], None), "or_raw32": ([vp, vp, sz], None),
            "or_u01": ([vp, vp, sz, ctypes.c_int], None),
            "or_u01f": ([vp, vp, sz, ctypes.c_int], None),
            "or_bounded64": ([vp, u64, vp, sz], None),
            "or_bounded32": ([vp, ctypes.c_uint32, vp, sz], None),
            "or_norm": ([vp, vp, sz, vp], None), "or_exp": ([vp, vp, sz, vp], None),
            "or_normf": ([vp, vp, sz], None), "or_expf": ([vp, vp, sz], None),
            "or_permutation": ([vp, ctypes.c_uint32, vp], None),
            "or_gammaf": ([vp, ctypes.c_double, ctypes.c_double, vp, sz], None),
            "or_mixf": ([vp, ctypes.c_int, vp, vp, sz], None),
            "or_sample": ([vp, ctypes.c_uint32, ctypes.c_uint32, vp], None),
            "or_norm_moments": ([vp, sz, vp, vp], None),
            "or_gamma": ([vp, ctypes.c_double, vp, sz, vp], None),
            "or_beta": ([vp, ctypes.c_double, ctypes.c_double, vp, sz], None),
            "or_gamma_batched": ([vp, vp, vp, sz, vp], None),
            "or_beta_batched": ([vp, vp, vp, vp, sz, vp], None),
            "or_gamma_elem": ([vp, vp, vp, sz], None),
            "or_beta_elem": ([vp, vp, vp, vp, sz], None),
            "or_mvn_z": ([vp, ctypes.c_int, sz, vp], None),
            "or_boost_pow": ([ctypes.c_double, ctypes.c_double], ctypes.c_double),
            "or_set_bitexact": ([ctypes.c_int], None),
            "or_get_bitexact": ([], ctypes.c_int),
            "or_crmath": ([ctypes.c_int, vp, vp, vp, sz], None),
            "or_seed_seq": ([vp, sz, vp, sz], None),
            "or_philox4x32_block": ([vp, vp, vp], None),
            "or_philox4x64_block": ([vp, vp, vp], None),
            "or_philox_constants": ([vp], None),
            "or_ranlux_constants": ([vp, vp, vp], None),
            "or_ranlux_mulmod": ([vp, vp, vp], None),
            "or_time_fills": ([vp, sz, ctypes.c_int, sz, ctypes.c_int], ctypes.c_double),
        }
        for name, (args, res) in sig.items():
            fn = getattr(_lib, name)
            fn.argtypes = args
            fn.restype = res
    return _lib


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def _split(n):
    n = int(n)
    return ctypes.c_uint64(n & (2**64 - 1)), ctypes.c_uint64(n >> 64)


class Counts:
    FIELDS = ("words", "candidates", "pdf_evals", "tail_entries", "tail_logs", "rejections",
              "mt_attempts", "mt_logtests")

    def __init__(self):
        self.buf = np.zeros(lib().or_counts_words(), dtype=np.uint64)

    def __getattr__(self, k):
        if k in Counts.FIELDS:
            return int(self.buf[Counts.FIELDS.index(k)])
        raise AttributeError(k)


# SIMD engines (Section 4.1): eight disjoint scalar sub-streams of the named
# scalar engine, xoshiro256 sub-stream k jumped by k 2^253 steps, sfc64
# sub-stream k with k 2^61 added to the counter (modulo 2^64).
SIMD_BASE = {X256PPS: "x256++", X256SSS: "x256**", SFC64S: "sfc64"}
SIMD_LANES = 8


@functools.lru_cache(maxsize=4096)
def x256_xpow(n):
    """x^n mod P for the xoshiro256 characteristic polynomial P (cached)."""
    return jumppoly.xpow_mod(int(n), jumppoly.x256_char_poly(lib()))


def simd_lanes_from_base(engine, base_words):
    """The 32 state words (sub-stream k at words 4k .. 4k+3) of a SIMD engine
    whose sub-stream 0 has the scalar state base_words."""
    words = []
    if engine == SFC64S:
        a, b, c, ctr = [int(x) for x in base_words[:4]]
        for k in range(SIMD_LANES):
            words += [a, b, c, (ctr + k * 2**61) % 2**64]
        return words
    jpoly = x256_xpow(2**253)
    cur = Stream.from_state(SIMD_BASE[engine], list(base_words[:4]))
    for k in range(SIMD_LANES):
        words += cur.state[:4]
        cur.x256_apply_poly(jpoly)
    return words


class Stream:
    """One serial stream of the oracle (a copy of the C struct)."""

    def __init__(self, engine):
        self.engine = ENGINE_IDS[engine] if isinstance(engine, str) else int(engine)
        self.buf = np.zeros(lib().or_stream_words(), dtype=np.uint64)
        self.buf[0] = self.engine

    # ---- construction ------------------------------------------------------
    @classmethod
    def seeded(cls, engine, seed, spawn_key=()):
        s = cls(engine)
        if s.engine in SIMD_BASE:
            # seeded as the scalar engine, then the eight sub-streams
            base = Stream.seeded(SIMD_BASE[s.engine], seed, spawn_key)
            return Stream.from_state(s.engine, simd_lanes_from_base(s.engine, base.state[:4]))
        key = np.array(list(spawn_key), dtype=np.uint32)
        rc = lib().or_seed(_p(s.buf), s.engine, ctypes.c_uint64(seed), _p(key) if len(key) else None,
                           len(key))
        assert rc == 0
        return s

    @classmethod
    def from_state(cls, engine, words, phase=0):
        s = cls(engine)
        w = np.array([int(x) for x in words], dtype=np.uint64)
        assert lib().or_set_state(_p(s.buf), s.engine, _p(w), len(w), phase) == 0
        return s

    def copy(self):
        s = Stream(self.engine)
        s.buf[:] = self.buf
        return s

    @property
    def state(self):
        return [int(x) for x in self.buf[2:34]]

    @property
    def phase(self):
        return int(self.buf[1])

    # ---- stream control ----------------------------------------------------
    def pcg64_set_inc(self, inc):
        lo, hi = _split(inc)
        assert lib().or_pcg64_set_inc(_p(self.buf), lo, hi) == 0
        return self

    def philox_set_key(self, k0, k1=0):
        assert lib().or_philox_set_key(_p(self.buf), ctypes.c_uint64(k0), ctypes.c_uint64(k1)) == 0
        return self

    def chacha20_set_nonce(self, nonce):
        """The 96-bit nonce (key and block counter kept)."""
        nonce = int(nonce)
        assert lib().or_chacha20_set_nonce(_p(self.buf), ctypes.c_uint64(nonce & (2**64 - 1)),
                                           ctypes.c_uint64(nonce >> 64)) == 0
        return self

    def cwg128_set_weyl(self, inc):
        """The Weyl increment (made odd), then 96 warm-up steps."""
        inc = int(inc)
        assert lib().or_cwg128_set_weyl(_p(self.buf), ctypes.c_uint64(inc & (2**64 - 1)),
                                        ctypes.c_uint64((inc >> 64) & (2**64 - 1))) == 0
        return self

    def squares_set_key(self, key):
        assert lib().or_squares_set_key(_p(self.buf), ctypes.c_uint64(key)) == 0
        return self

    def sfc64_set_abc(self, a, b, c):
        if self.engine == SFC64S:
            base = Stream("sfc64").sfc64_set_abc(a, b, c)
            self.buf[:] = Stream.from_state(SFC64S, simd_lanes_from_base(SFC64S, base.state[:4])).buf
            return self
        lib().or_sfc64_set_abc(_p(self.buf), a, b, c)
        return self

    def x256_apply_poly(self, poly):
        w = jumppoly.poly_words(poly)
        assert lib().or_x256_apply_poly(_p(self.buf), _p(w)) == 0
        return self

    def advance(self, n):
        """Move forward by n engine steps (blocks for block engines)."""
        n = int(n)
        if self.engine in (X256PPS, X256SSS):
            # every sub-stream moves n steps; the phase in the block is kept
            poly = x256_xpow(n)
            words = self.state[:32]
            for k in range(SIMD_LANES):
                lane = Stream.from_state(SIMD_BASE[self.engine], words[4 * k:4 * k + 4]).x256_apply_poly(poly)
                words[4 * k:4 * k + 4] = lane.state[:4]
            ph = self.phase
            self.buf[:] = Stream.from_state(self.engine, words, ph).buf
            return self
        if self.engine in (X256PP, X256SS):
            p = jumppoly.x256_char_poly(lib())
            return self.x256_apply_poly(jumppoly.xpow_mod(n, p))
        if self.engine in (XORO128PP, XS128P):
            p = jumppoly.x128_char_poly(lib(), self.engine)
            w = jumppoly.poly_words(jumppoly.xpow_mod(n, p), 2)
            assert lib().or_x128_apply_poly(_p(self.buf), _p(w)) == 0
            return self
        if self.engine == CHACHA20:
            # n blocks: the 32-bit counter in the high half of state word 5
            # (mod 2^32); the buffered block is recomputed on the next draw
            w5 = int(self.buf[2 + 5])
            c = ((w5 >> 32) + n) % 2**32
            self.buf[2 + 5] = np.uint64((w5 & (2**32 - 1)) | (c << 32))
            self.buf[2 + 32 + 9] = np.uint64(0)     # blk_ok
            return self
        if self.engine == SQUARES:
            # counter engine with period 2^64: the counter word moves by n
            self.buf[2] = np.uint64((int(self.buf[2]) + n) % 2**64)
            return self
        if self.engine == PCG64:
            lo, hi = _split(n % 2**128)
            assert lib().or_pcg64_advance(_p(self.buf), lo, hi) == 0
            return self
        limbs = np.array([(n >> (64 * i)) & (2**64 - 1) for i in range(4)], dtype=np.uint64)
        assert n < 2**256
        fn = {PHILOX4X32: lib().or_philox_advance, PHILOX4X64: lib().or_philox_advance,
              RANLUX: lib().or_ranlux_advance}[self.engine]
        assert fn(_p(self.buf), _p(limbs)) == 0
        return self

    # ---- samplers ----------------------------------------------------------
    def raw(self, n):
        out = np.empty(n, dtype=np.uint64)
        lib().or_raw64(_p(self.buf), _p(out), n)
        return out

    def raw32(self, n):
        out = np.empty(n, dtype=np.uint32)
        lib().or_raw32(_p(self.buf), _p(out), n)
        return out

    def u01(self, n, full_mantissa=True):
        out = np.empty(n, dtype=np.float64)
        lib().or_u01(_p(self.buf), _p(out), n, int(full_mantissa))
        return out

    def u01f(self, n, full_mantissa=True):
        out = np.empty(n, dtype=np.float32)
        lib().or_u01f(_p(self.buf), _p(out), n, int(full_mantissa))
        return out

    def bounded64(self, b, n):
        out = np.empty(n, dtype=np.uint64)
        lib().or_bounded64(_p(self.buf), ctypes.c_uint64(b), _p(out), n)
        return out

    def bounded32(self, b, n):
        out = np.empty(n, dtype=np.uint32)
        lib().or_bounded32(_p(self.buf), ctypes.c_uint32(b), _p(out), n)
        return out

    def norm(self, n, counts=None):
        out = np.empty(n, dtype=np.float64)
        lib().or_norm(_p(self.buf), _p(out), n, _p(counts.buf) if counts else None)
        return out

    def exp(self, n, counts=None):
        out = np.empty(n, dtype=np.float64)
        lib().or_exp(_p(self.buf), _p(out), n, _p(counts.buf) if counts else None)
        return out

    def normf(self, n):
        """n binary32 standard normals from 32-bit items (float ziggurat)."""
        out = np.empty(n, dtype=np.float32)
        lib().or_normf(_p(self.buf), _p(out), n)
        return out

    def expf(self, n):
        """n binary32 standard exponentials from 32-bit items (float ziggurat)."""
        out = np.empty(n, dtype=np.float32)
        lib().or_expf(_p(self.buf), _p(out), n)
        return out

    def gammaf(self, alpha, n, theta=1.0):
        """n binary32 Gamma(alpha, theta) draws (float gamma)."""
        out = np.empty(n, dtype=np.float32)
        lib().or_gammaf(_p(self.buf), float(alpha), float(theta), _p(out), n)
        return out

    def mixf(self, law, params, n):
        """n binary32 draws of a law of several draws (10 beta, 11 chi2, 12 t,
        13 F, 14 skew-normal): float base draws, binary64 combination, one
        rounding."""
        out = np.empty(n, dtype=np.float32)
        p = np.ascontiguousarray(np.asarray(params, dtype=np.float64))
        lib().or_mixf(_p(self.buf), int(law), _p(p), _p(out), n)
        return out

    def permutation(self, n):
        """Fisher-Yates permutation of 0..n-1 (32-bit Lemire draws)."""
        out = np.empty(n, dtype=np.uint32)
        lib().or_permutation(_p(self.buf), n, _p(out))
        return out

    def sample(self, n, k):
        """k distinct elements of 0..n-1: Floyd (k <= n/2) or reservoir."""
        out = np.empty(k, dtype=np.uint32)
        lib().or_sample(_p(self.buf), n, k, _p(out))
        return out

    def norm_moments(self, n):
        s = np.zeros(1)
        q = np.zeros(1)
        lib().or_norm_moments(_p(self.buf), n, _p(s), _p(q))
        return float(s[0]), float(q[0])

    def gamma(self, alpha, n, counts=None):
        out = np.empty(n, dtype=np.float64)
        lib().or_gamma(_p(self.buf), float(alpha), _p(out), n, _p(counts.buf) if counts else None)
        return out

    def beta(self, a, b, n):
        out = np.empty(n, dtype=np.float64)
        lib().or_beta(_p(self.buf), float(a), float(b), _p(out), n)
        return out


class StreamArray:
    """Contiguous array of C stream structs (one per substream)."""

    def __init__(self, streams):
        self.n = len(streams)
        w = lib().or_stream_words()
        self.buf = np.zeros((self.n, w), dtype=np.uint64)
        for i, s in enumerate(streams):
            self.buf[i] = s.buf

    @classmethod
    def key_family(cls, engine, seed, n):
        """Substreams 0..n-1 of the Philox key family (key := i over the
        seeded counter), built as one array; equal to substream(engine, seed,
        "key", i) for every i (spot-checked here)."""
        base = substream(engine, seed, "key", 0)
        arr = cls.__new__(cls)
        arr.n = n
        arr.buf = np.tile(base.buf, (n, 1))
        key_word = {"philox4x32": 2, "philox": 4}[engine]
        arr.buf[:, 2 + key_word] = np.arange(n, dtype=np.uint64)
        for i in {0, 1, n // 2, n - 1}:
            assert (arr.buf[i] == substream(engine, seed, "key", i).buf).all()
        return arr

    def stream(self, i):
        s = Stream(int(self.buf[i, 0]))
        s.buf[:] = self.buf[i]
        return s

    def gamma_batched(self, alpha, count):
        alpha = np.ascontiguousarray(alpha, dtype=np.float64)
        count = np.ascontiguousarray(count, dtype=np.int64)
        out = np.empty(int(count.sum()), dtype=np.float64)
        lib().or_gamma_batched(_p(self.buf), _p(alpha), _p(count), self.n, _p(out))
        return out

    def beta_batched(self, a, b, count):
        a = np.ascontiguousarray(a, dtype=np.float64)
        b = np.ascontiguousarray(b, dtype=np.float64)
        count = np.ascontiguousarray(count, dtype=np.int64)
        out = np.empty(int(count.sum()), dtype=np.float64)
        lib().or_beta_batched(_p(self.buf), _p(a), _p(b), _p(count), self.n, _p(out))
        return out

    def gamma_elem(self, alpha):
        alpha = np.ascontiguousarray(alpha, dtype=np.float32)
        z = np.empty(self.n, dtype=np.float32)
        lib().or_gamma_elem(_p(self.buf), _p(alpha), _p(z), self.n)
        return z

    def beta_elem(self, a, b):
        a = np.ascontiguousarray(a, dtype=np.float32)
        b = np.ascontiguousarray(b, dtype=np.float32)
        z = np.empty(self.n, dtype=np.float32)
        lib().or_beta_elem(_p(self.buf), _p(a), _p(b), _p(z), self.n)
        return z

    def mvn_z(self, d):
        z = np.empty((self.n, d), dtype=np.float32)
        lib().or_mvn_z(_p(self.buf), d, self.n, _p(z))
        return z


# ---- substream recipes (Section 2.3: duplicate, then set the stream or jump) --

def substream(engine, seed, kind, i, jump_log2=64):
    """Stream i of a substream family built from a base seeded with `seed`.

    kind: "key"   philox: key := i (counter from the seeded base)
          "inc"   pcg64: increment := 2 i + 1
          "spawn" seed mixer with spawn key [i]
          "jump"  base advanced by i * 2^jump_log2 engine steps
    """
    if kind == "spawn":
        return Stream.seeded(engine, seed, [i])
    s = Stream.seeded(engine, seed)
    if kind == "key":
        return s.philox_set_key(i, 0)
    if kind == "nonce":
        return s.chacha20_set_nonce(i)
    if kind == "inc":
        if engine == "cwg128":
            return s.cwg128_set_weyl(2 * i + 1)
        return s.pcg64_set_inc(2 * i + 1)
    if kind == "jump":
        return s.advance(i << jump_log2)
    raise ValueError(kind)


def boost_pow(u, a):
    return lib().or_boost_pow(float(u), float(a))


CR_EXP, CR_LOG, CR_LOG1P, CR_POW, CR_POWINV = range(5)


def crmath(fn, x, y=None):
    """Correctly rounded f(x, y) elementwise (binary128 rounded once to
    binary64): 0 exp, 1 log, 2 log1p, 3 pow, 4 x^(1/y)."""
    x = np.ascontiguousarray(np.asarray(x, dtype=np.float64).reshape(-1))
    yy = np.ascontiguousarray(np.broadcast_to(np.asarray(0.0 if y is None else y, dtype=np.float64), x.shape))
    out = np.empty_like(x)
    lib().or_crmath(fn, _p(x), _p(yy), _p(out), len(x))
    return out


class bitexact:
    """Context manager: the oracle's samplers use correctly rounded exp, log
    and log1p (the bitexact setting) inside the block."""

    def __init__(self, on=True):
        self.on = bool(on)

    def __enter__(self):
        self.prev = lib().or_get_bitexact()
        lib().or_set_bitexact(1 if self.on else 0)
        return self

    def __exit__(self, *exc):
        lib().or_set_bitexact(self.prev)
        return False


def bitexact_on():
    return lib().or_get_bitexact() != 0


def time_fills(streams, what, per, threads):
    """Wall seconds for `per` values of fill `what` (0 raw, 1 U(0,1)
    binary32, 2 U(0,1) binary64, 3 normal, 4 exponential) from each stream,
    on `threads` POSIX threads inside the C oracle (the streams advance)."""
    w = lib().or_stream_words()
    buf = np.concatenate([s.buf for s in streams]).astype(np.uint64)
    t = lib().or_time_fills(_p(buf), len(streams), int(what), int(per), int(threads))
    if t < 0:
        raise RuntimeError("or_time_fills: could not start threads")
    for k, s in enumerate(streams):
        s.buf[:] = buf[k * w:(k + 1) * w]
    return t
