"""MI355X (gfx950) implementation of the Randompack hot path (arXiv 2605.05099).

A thin ctypes binding over the C ABI in include/rp.h (library: librp.so next to
this file).  Functions keep the C names (``rp_create``, ``rp_fill``, ...) and
only marshal arguments: every step of generation runs in the HIP kernels.
PyTorch supplies device memory (tensors) and the current HIP stream.

There is no fallback: importing works without a GPU (host-side calls such as
seeding and jumps run anywhere), but if librp.so is missing the import fails
with an error telling how to build it.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "librp.so")

# status codes, engines, distributions, dtypes (include/rp.h)
RP_OK, RP_EINVAL, RP_ENOMEM, RP_EUNSUPPORTED, RP_EDEVICE, RP_ENOTSPD, RP_ENULL = 0, -1, -2, -3, -4, -5, -6
(RP_X256PP, RP_PCG64, RP_PHILOX4X32, RP_PHILOX, RP_SFC64, RP_RANLUX, RP_X256SS, RP_SQUARES, RP_XORO128, RP_XS128,
 RP_CHACHA20, RP_CWG128, RP_X256PPS, RP_X256SSS, RP_SFC64S) = range(15)
RP_SUB_KEY, RP_SUB_INC, RP_SUB_SPAWN, RP_SUB_JUMP = range(4)
RP_RAW, RP_U01, RP_BOUNDED, RP_NORM, RP_EXP = range(5)
RP_U64, RP_U32, RP_F64, RP_F32 = range(4)
RP_FLAG_52BIT = 1
RP_FULL_MANTISSA, RP_SQUEEZE, RP_BITEXACT = 1, 2, 3  # settings (rp_set_flag)
RP_CR_EXP, RP_CR_LOG, RP_CR_LOG1P, RP_CR_POW, RP_CR_POWINV = range(5)
(RP_LAW_UNIF, RP_LAW_NORMAL, RP_LAW_LOGNORMAL, RP_LAW_EXP, RP_LAW_GUMBEL, RP_LAW_PARETO, RP_LAW_GPARETO,
 RP_LAW_WEIBULL, RP_LAW_GAMMA, RP_LAW_BETA, RP_LAW_CHI2, RP_LAW_T, RP_LAW_F, RP_LAW_SKEWNORMAL) = range(1, 15)

ENGINES = {"x256++": RP_X256PP, "x256**": RP_X256SS, "pcg64": RP_PCG64, "philox4x32": RP_PHILOX4X32, "philox": RP_PHILOX,
           "sfc64": RP_SFC64, "ranlux++": RP_RANLUX, "squares": RP_SQUARES, "xoro++": RP_XORO128, "x128+": RP_XS128,
           "chacha20": RP_CHACHA20, "cwg128": RP_CWG128, "x256++simd": RP_X256PPS, "x256**simd": RP_X256SSS,
           "sfc64simd": RP_SFC64S}
STATE_WORDS = {RP_X256PP: 4, RP_PCG64: 4, RP_PHILOX4X32: 3, RP_PHILOX: 6, RP_SFC64: 4, RP_RANLUX: 9, RP_X256SS: 4, RP_SQUARES: 2, RP_XORO128: 2, RP_XS128: 2, RP_CHACHA20: 6,
               RP_CWG128: 8, RP_X256PPS: 32, RP_X256SSS: 32, RP_SFC64S: 32}

_vp, _sz, _u64, _u32, _int = ctypes.c_void_p, ctypes.c_size_t, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_int
_SIGS = {
    "rp_errmsg": ([], ctypes.c_char_p),
    "rp_last_error": ([_vp], ctypes.c_char_p),
    "rp_engines": ([ctypes.c_char_p, _sz], _int),
    "rp_engine_id": ([ctypes.c_char_p], _int),
    "rp_create": ([ctypes.c_char_p], _vp),
    "rp_free": ([_vp], None),
    "rp_duplicate": ([_vp], _vp),
    "rp_seed": ([_vp, _u64, _vp, _sz], _int),
    "rp_state_words": ([_vp], _int),
    "rp_get_state": ([_vp, _vp, _sz, _vp], _int),
    "rp_set_state": ([_vp, _vp, _sz, _u32], _int),
    "rp_jump": ([_vp, _int], _int),
    "rp_advance": ([_vp, _u64, _u64], _int),
    "rp_pcg64_set_inc": ([_vp, _u64, _u64], _int),
    "rp_philox_set_key": ([_vp, _u64, _u64], _int),
    "rp_sfc64_set_abc": ([_vp, _u64, _u64, _u64], _int),
    "rp_squares_set_key": ([_vp, _u64], _int),
    "rp_randomize": ([_vp], _int),
    "rp_set_full_mantissa": ([_vp, _int], _int),
    "rp_get_full_mantissa": ([_vp], _int),
    "rp_set_flag": ([_vp, _int, _int], _int),
    "rp_get_flag": ([_vp, _int], _int),
    "rp_streams_set_flag": ([_vp, _int, _int], _int),
    "rp_streams_get_flag": ([_vp, _int], _int),
    "rp_chacha20_set_nonce": ([_vp, _u64, _u64], _int),
    "rp_cwg128_set_weyl": ([_vp, _u64, _u64], _int),
    "rp_serialize": ([_vp, _vp, _sz, _vp], _int),
    "rp_deserialize": ([_vp, _vp, _sz], _int),
    "rp_raw_host": ([_vp, _vp, _sz], _int),
    "rp_streams_create": ([_vp, _int, _u64, _int, _vp], _int),
    "rp_streams_free": ([_vp], None),
    "rp_streams_count": ([_vp], _u64),
    "rp_streams_engine": ([_vp], _int),
    "rp_streams_get": ([_vp, _vp, _vp], _int),
    "rp_streams_set": ([_vp, _vp, _vp], _int),
    "rp_streams_duplicate": ([_vp, _vp], _int),
    "rp_streams_serialize": ([_vp, _vp, _sz, _vp], _int),
    "rp_streams_deserialize": ([_vp, _sz, _vp], _int),
    "rp_fill": ([_vp, _int, _int, _u64, _int, _vp, _u64, _vp], _int),
    "rp_fill_law": ([_vp, _int, _vp, _int, _vp, _u64, _vp], _int),
    "rp_fill_lawf": ([_vp, _int, _vp, _int, _vp, _u64, _vp], _int),
    "rp_fill_serial": ([_vp, _int, _int, _u64, _int, _vp, _u64, _vp], _int),
    "rp_norm_moments": ([_vp, _u64, _vp, _vp, _vp], _int),
    "rp_gamma_elem": ([_vp, _vp, _vp, _u64, _vp], _int),
    "rp_beta_elem": ([_vp, _vp, _vp, _vp, _u64, _vp], _int),
    "rp_plan_create": ([_vp], _int),
    "rp_plan_free": ([_vp], None),
    "rp_plan_set_config": ([_vp, _int, _int, _int], _int),
    "rp_plan_get_config": ([_vp, _vp, _vp, _vp], _int),
    "rp_plan_autotune": ([_vp, _vp, _int, _vp, _vp, _vp, _u64, _vp], _int),
    "rp_gamma_batched": ([_vp, _vp, _vp, _u64, _vp, _vp, _vp], _int),
    "rp_beta_batched": ([_vp, _vp, _vp, _vp, _u64, _vp, _vp, _vp], _int),
    "rp_cholesky": ([_vp, _int, _vp], _int),
    "rp_mvn_factor": ([_vp, _int, _vp, _vp], _int),
    "rp_permutations": ([_vp, _u32, _vp, _vp], _int),
    "rp_sample": ([_vp, _u32, _u32, _vp, _vp], _int),
    "rp_sample_noalloc": ([_vp, _u32, _u32, _vp, _vp], _int),
    "rp_crmath_host": ([_int, _vp, _vp, _vp, _u64], _int),
    "rp_gamma_grad_host": ([_vp, _vp, _vp, _vp, _u64], _int),
    "rp_beta_grad_host": ([_vp, _vp, _vp, _vp, _vp, _vp, _u64], _int),
    "rp_crmath": ([_int, _vp, _vp, _vp, _u64, _vp], _int),
    "rp_mvn": ([_vp, _vp, _vp, _int, _u64, _vp, _vp], _int),
    "rp_mvn_backward": ([_vp, _vp, _int, _u64, _vp, _vp, _vp], _int),
    "rp_gamma_grad": ([_vp, _vp, _vp, _vp, _u64, _vp], _int),
    "rp_beta_grad": ([_vp, _vp, _vp, _vp, _vp, _vp, _u64, _vp], _int),
}


class RpError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{msg} (status {code})")
        self.code = code


_lib = None


def lib():
    """The loaded librp.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              "`python -m paper_2605_05099_amd.build` (hipcc, gfx950)")
        l = ctypes.CDLL(LIB_PATH)
        for name, (args, res) in _SIGS.items():
            fn = getattr(l, name)
            fn.argtypes = args
            fn.restype = res
        _lib = l
    return _lib


def _check(rc, handle=None):
    if rc < 0:
        msg = lib().rp_last_error(handle) if handle else lib().rp_errmsg()
        raise RpError(rc, (msg or b"").decode())
    return rc


def _ptr(a):
    return ctypes.c_void_p(a.ctypes.data) if isinstance(a, np.ndarray) else ctypes.c_void_p(int(a))


def _dev_ptr(t):
    """Device pointer of a torch tensor (or an integer address)."""
    return ctypes.c_void_p(t if isinstance(t, int) else t.data_ptr())


def _stream_ptr(stream):
    if stream is None:
        import torch
        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, int):
        return ctypes.c_void_p(stream)
    return ctypes.c_void_p(stream.cuda_stream)


# ---- the C names ----------------------------------------------------------------
def rp_errmsg():
    return lib().rp_errmsg().decode()


def rp_engines():
    n = lib().rp_engines(None, 0)
    buf = ctypes.create_string_buffer(n + 1)
    lib().rp_engines(buf, n + 1)
    return buf.value.decode()


def rp_engine_id(name):
    return _check(lib().rp_engine_id(name.encode()))


def rp_create(engine="x256++"):
    h = lib().rp_create(engine.encode() if engine is not None else None)
    if not h:
        raise RpError(RP_EINVAL, rp_errmsg())
    return Rng(h)


def rp_streams_deserialize(image):
    out = ctypes.c_void_p()
    _check(lib().rp_streams_deserialize(image, len(image), ctypes.byref(out)))
    return Streams(out.value)


def rp_streams_create(base, kind, n, jump_log2=0):
    out = ctypes.c_void_p()
    _check(lib().rp_streams_create(base.h, kind, n, jump_log2, ctypes.byref(out)))
    return Streams(out.value)


def rp_fill(streams, dist, dtype, bound, flags, out, per_stream, stream=None):
    _check(lib().rp_fill(streams.h, dist, dtype, bound, flags, _dev_ptr(out), per_stream, _stream_ptr(stream)))


def rp_fill_lawf(streams, law, params, out, per_stream, stream=None):
    p = np.ascontiguousarray(np.asarray(params, dtype=np.float64).reshape(-1))
    _check(lib().rp_fill_lawf(streams.h, law, _ptr(p) if len(p) else None, len(p), _dev_ptr(out), per_stream,
                              _stream_ptr(stream)))


def rp_permutations(streams, n, out, stream=None):
    _check(lib().rp_permutations(streams.h, n, _dev_ptr(out), _stream_ptr(stream)))


def rp_sample(streams, n, k, out, stream=None):
    _check(lib().rp_sample(streams.h, n, k, _dev_ptr(out), _stream_ptr(stream)))


def rp_sample_noalloc(streams, n, k, out, stream=None):
    _check(lib().rp_sample_noalloc(streams.h, n, k, _dev_ptr(out), _stream_ptr(stream)))


def rp_crmath_host(fn, x, y=None):
    """Correctly rounded f(x[i], y[i]) on the host (numpy arrays)."""
    x = np.ascontiguousarray(np.asarray(x, dtype=np.float64).reshape(-1))
    yy = None if y is None else np.ascontiguousarray(np.broadcast_to(np.asarray(y, dtype=np.float64), x.shape))
    out = np.empty_like(x)
    _check(lib().rp_crmath_host(fn, _ptr(x), _ptr(yy) if yy is not None else None, _ptr(out), len(x)))
    return out


def rp_gamma_grad_host(z, alpha, gz):
    """Binary64 gradient evaluation on the host (numpy float32 arrays)."""
    z, alpha, gz = (np.ascontiguousarray(np.asarray(v, dtype=np.float32).reshape(-1)) for v in (z, alpha, gz))
    out = np.empty_like(z)
    _check(lib().rp_gamma_grad_host(_ptr(z), _ptr(alpha), _ptr(gz), _ptr(out), len(z)))
    return out


def rp_beta_grad_host(z, a, b, gz):
    """Binary64 gradient evaluation on the host (numpy float32 arrays)."""
    z, a, b, gz = (np.ascontiguousarray(np.asarray(v, dtype=np.float32).reshape(-1)) for v in (z, a, b, gz))
    ga, gb = np.empty_like(z), np.empty_like(z)
    _check(lib().rp_beta_grad_host(_ptr(z), _ptr(a), _ptr(b), _ptr(gz), _ptr(ga), _ptr(gb), len(z)))
    return ga, gb


def rp_crmath(fn, x, y, out, stream=None):
    """Correctly rounded f(x[i], y[i]) on the device (float64 tensors; y may be None)."""
    _check(lib().rp_crmath(fn, _dev_ptr(x), _dev_ptr(y) if y is not None else None, _dev_ptr(out), out.numel(),
                           _stream_ptr(stream)))


def rp_fill_law(streams, law, params, out, per_stream, stream=None):
    p = np.ascontiguousarray(np.asarray(params, dtype=np.float64).reshape(-1))
    _check(lib().rp_fill_law(streams.h, law, _ptr(p) if len(p) else None, len(p), _dev_ptr(out), per_stream,
                             _stream_ptr(stream)))


def rp_fill_serial(rng, dist, dtype, bound, flags, out, n, stream=None):
    _check(lib().rp_fill_serial(rng.h, dist, dtype, bound, flags, _dev_ptr(out), n, _stream_ptr(stream)))


def rp_norm_moments(streams, per_stream, d_sum, d_sumsq, stream=None):
    _check(lib().rp_norm_moments(streams.h, per_stream, _dev_ptr(d_sum), _dev_ptr(d_sumsq), _stream_ptr(stream)))


def rp_gamma_elem(streams, alpha, z, n, stream=None):
    _check(lib().rp_gamma_elem(streams.h, _dev_ptr(alpha), _dev_ptr(z), n, _stream_ptr(stream)))


def rp_beta_elem(streams, a, b, z, n, stream=None):
    _check(lib().rp_beta_elem(streams.h, _dev_ptr(a), _dev_ptr(b), _dev_ptr(z), n, _stream_ptr(stream)))


class Plan:
    """rp_plan*: scratch, launch configuration and recorded graph of the
    batched gamma / beta sequence."""

    def __init__(self):
        out = ctypes.c_void_p()
        _check(lib().rp_plan_create(ctypes.byref(out)))
        self.h = ctypes.c_void_p(out.value)

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.rp_plan_free(self.h)
            self.h = None

    def set_config(self, block, blocks_per_cu, sets_per_lane):
        _check(lib().rp_plan_set_config(self.h, block, blocks_per_cu, sets_per_lane))

    def get_config(self):
        b, p, s = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
        tuned = _check(lib().rp_plan_get_config(self.h, ctypes.byref(b), ctypes.byref(p), ctypes.byref(s)))
        return {"block": b.value, "blocks_per_cu": p.value, "sets_per_lane": s.value, "tuned": bool(tuned)}


def rp_plan_create():
    return Plan()


def rp_plan_autotune(plan, streams, beta, pa, pb, count, n_sets, out):
    _check(lib().rp_plan_autotune(plan.h, streams.h, int(beta), _dev_ptr(pa), _dev_ptr(pb) if pb is not None else None,
                                  _dev_ptr(count), n_sets, _dev_ptr(out)))


def rp_gamma_batched(streams, alpha, count, n_sets, out, plan, stream=None):
    _check(lib().rp_gamma_batched(streams.h, _dev_ptr(alpha), _dev_ptr(count), n_sets, _dev_ptr(out), plan.h,
                                  _stream_ptr(stream)))


def rp_beta_batched(streams, a, b, count, n_sets, out, plan, stream=None):
    _check(lib().rp_beta_batched(streams.h, _dev_ptr(a), _dev_ptr(b), _dev_ptr(count), n_sets, _dev_ptr(out), plan.h,
                                 _stream_ptr(stream)))


def rp_cholesky(sigma):
    """Binary64 Cholesky factor on the host (numpy in, numpy out)."""
    a = np.ascontiguousarray(sigma, dtype=np.float64)
    d = a.shape[0]
    if a.shape != (d, d):
        raise ValueError("sigma must be square")
    out = np.zeros((d, d), dtype=np.float64)
    _check(lib().rp_cholesky(_ptr(a), d, _ptr(out)))
    return out


def rp_mvn_factor(sigma):
    """(A, rank) with sigma = A A^T on the host: Cholesky, else pivoted
    Cholesky for a semidefinite sigma (numpy in, numpy out)."""
    a = np.ascontiguousarray(sigma, dtype=np.float64)
    d = a.shape[0]
    if a.shape != (d, d):
        raise ValueError("sigma must be square")
    out = np.zeros((d, d), dtype=np.float64)
    rank = ctypes.c_int(0)
    _check(lib().rp_mvn_factor(_ptr(a), d, _ptr(out), ctypes.byref(rank)))
    return out, rank.value


def rp_mvn(streams, mu, L, d, n, X, stream=None):
    _check(lib().rp_mvn(streams.h, _dev_ptr(mu), _dev_ptr(L), d, n, _dev_ptr(X), _stream_ptr(stream)))


def rp_mvn_backward(streams, G, d, n, gmu, gL, stream=None):
    _check(lib().rp_mvn_backward(streams.h, _dev_ptr(G), d, n, _dev_ptr(gmu), _dev_ptr(gL), _stream_ptr(stream)))


def rp_gamma_grad(z, alpha, gz, galpha, n, stream=None):
    _check(lib().rp_gamma_grad(_dev_ptr(z), _dev_ptr(alpha), _dev_ptr(gz), _dev_ptr(galpha), n,
                               _stream_ptr(stream)))


def rp_beta_grad(z, a, b, gz, ga, gb, n, stream=None):
    _check(lib().rp_beta_grad(_dev_ptr(z), _dev_ptr(a), _dev_ptr(b), _dev_ptr(gz), _dev_ptr(ga), _dev_ptr(gb), n,
                              _stream_ptr(stream)))


# ---- object wrappers ----------------------------------------------------------------
class Rng:
    """rp_rng*: one serial stream (host resident)."""

    def __init__(self, h):
        self.h = ctypes.c_void_p(h)

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.rp_free(self.h)
            self.h = None

    @property
    def engine(self):
        return self._engine if hasattr(self, "_engine") else None

    def seed(self, seed, spawn_key=()):
        key = np.asarray(list(spawn_key), dtype=np.uint32)
        _check(lib().rp_seed(self.h, seed, _ptr(key) if len(key) else None, len(key)), self.h)
        return self

    def state_words(self):
        return _check(lib().rp_state_words(self.h))

    def get_state(self):
        n = self.state_words()
        w = np.zeros(n, dtype=np.uint64)
        ph = np.zeros(1, dtype=np.uint32)
        _check(lib().rp_get_state(self.h, _ptr(w), n, _ptr(ph)), self.h)
        return [int(x) for x in w], int(ph[0])

    def set_state(self, words, phase=0):
        w = np.asarray([int(x) for x in words], dtype=np.uint64)
        _check(lib().rp_set_state(self.h, _ptr(w), len(w), phase), self.h)
        return self

    def jump(self, k):
        _check(lib().rp_jump(self.h, k), self.h)
        return self

    def advance(self, n):
        n = int(n)
        _check(lib().rp_advance(self.h, n & (2**64 - 1), n >> 64), self.h)
        return self

    def pcg64_set_inc(self, inc):
        _check(lib().rp_pcg64_set_inc(self.h, inc & (2**64 - 1), inc >> 64), self.h)
        return self

    def philox_set_key(self, k0, k1=0):
        _check(lib().rp_philox_set_key(self.h, k0, k1), self.h)
        return self

    def sfc64_set_abc(self, a, b, c):
        _check(lib().rp_sfc64_set_abc(self.h, a, b, c), self.h)
        return self

    def randomize(self):
        _check(lib().rp_randomize(self.h), self.h)
        return self

    @property
    def full_mantissa(self):
        return bool(_check(lib().rp_get_full_mantissa(self.h), self.h))

    @full_mantissa.setter
    def full_mantissa(self, on):
        _check(lib().rp_set_full_mantissa(self.h, int(bool(on))), self.h)

    def set_flag(self, flag, value):
        _check(lib().rp_set_flag(self.h, flag, int(value)), self.h)
        return self

    def get_flag(self, flag):
        return bool(_check(lib().rp_get_flag(self.h, flag), self.h))

    def squares_set_key(self, key):
        _check(lib().rp_squares_set_key(self.h, key), self.h)
        return self

    def chacha20_set_nonce(self, nonce):
        _check(lib().rp_chacha20_set_nonce(self.h, nonce & (2**64 - 1), nonce >> 64), self.h)
        return self

    def cwg128_set_weyl(self, inc):
        _check(lib().rp_cwg128_set_weyl(self.h, inc & (2**64 - 1), (inc >> 64) & (2**64 - 1)), self.h)
        return self

    def duplicate(self):
        h = lib().rp_duplicate(self.h)
        if not h:
            raise RpError(RP_ENOMEM, rp_errmsg())
        return Rng(h)

    def serialize(self):
        need = ctypes.c_size_t()
        _check(lib().rp_serialize(self.h, None, 0, ctypes.byref(need)), self.h)
        buf = ctypes.create_string_buffer(need.value)
        _check(lib().rp_serialize(self.h, buf, need.value, None), self.h)
        return buf.raw

    def deserialize(self, data):
        buf = ctypes.create_string_buffer(bytes(data), len(data))
        _check(lib().rp_deserialize(self.h, buf, len(data)), self.h)
        return self

    def raw_host(self, n):
        out = np.zeros(n, dtype=np.uint64)
        _check(lib().rp_raw_host(self.h, _ptr(out), n), self.h)
        return out

    def last_error(self):
        return lib().rp_last_error(self.h).decode()


class Streams:
    """rp_streams*: n substreams resident in device memory."""

    def __init__(self, h):
        self.h = ctypes.c_void_p(h)

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.rp_streams_free(self.h)
            self.h = None

    def __len__(self):
        return int(lib().rp_streams_count(self.h))

    @property
    def engine(self):
        return _check(lib().rp_streams_engine(self.h))

    def get(self):
        n = len(self)
        w = np.zeros(STATE_WORDS[self.engine] * n, dtype=np.uint64)
        ph = np.zeros(n, dtype=np.uint32)
        _check(lib().rp_streams_get(self.h, _ptr(w), _ptr(ph)))
        return w.reshape(STATE_WORDS[self.engine], n), ph

    def set(self, words, phase):
        w = np.ascontiguousarray(words, dtype=np.uint64).reshape(-1)
        ph = np.ascontiguousarray(phase, dtype=np.uint32)
        _check(lib().rp_streams_set(self.h, _ptr(w), _ptr(ph)))

    def duplicate(self):
        out = ctypes.c_void_p()
        _check(lib().rp_streams_duplicate(self.h, ctypes.byref(out)))
        return Streams(out.value)

    def set_flag(self, flag, value):
        _check(lib().rp_streams_set_flag(self.h, flag, int(value)))
        return self

    def get_flag(self, flag):
        return bool(_check(lib().rp_streams_get_flag(self.h, flag)))

    def serialize(self):
        need = ctypes.c_size_t()
        _check(lib().rp_streams_serialize(self.h, None, 0, ctypes.byref(need)))
        buf = ctypes.create_string_buffer(need.value)
        _check(lib().rp_streams_serialize(self.h, buf, need.value, None))
        return buf.raw

    def fill(self, dist, out, per_stream, bound=0, flags=0, stream=None):
        """Fill a device tensor of n * per_stream elements (dtype decides the form)."""
        import torch
        dt = {torch.uint64: RP_U64, torch.int64: RP_U64, torch.uint32: RP_U32, torch.int32: RP_U32,
              torch.float64: RP_F64, torch.float32: RP_F32}[out.dtype]
        if out.numel() != len(self) * per_stream or not out.is_contiguous() or not out.is_cuda:
            raise ValueError("out must be a contiguous device tensor of n * per_stream elements")
        rp_fill(self, dist, dt, bound, flags, out, per_stream, stream)
        return out
