"""Helpers shared by the GPU tests: build matching substreams on both sides."""
import numpy as np

import oracle
import paper_2605_05099_amd as rp

# how each engine's substream family is built (Section 2.3 and Table 3)
FAMILY = {
    "philox4x32": (rp.RP_SUB_KEY, "key"),
    "philox": (rp.RP_SUB_KEY, "key"),
    "pcg64": (rp.RP_SUB_INC, "inc"),
    "x256++": (rp.RP_SUB_JUMP, "jump"),
    "x256**": (rp.RP_SUB_JUMP, "jump"),
    "ranlux++": (rp.RP_SUB_JUMP, "jump"),
    "sfc64": (rp.RP_SUB_SPAWN, "spawn"),
    "squares": (rp.RP_SUB_SPAWN, "spawn"),
    "xoro++": (rp.RP_SUB_JUMP, "jump"),
    "x128+": (rp.RP_SUB_JUMP, "jump"),
    "chacha20": (rp.RP_SUB_KEY, "nonce"),
    "cwg128": (rp.RP_SUB_INC, "inc"),
    "x256++simd": (rp.RP_SUB_JUMP, "jump"),
    "x256**simd": (rp.RP_SUB_JUMP, "jump"),
    "sfc64simd": (rp.RP_SUB_SPAWN, "spawn"),
}
ENGINES = list(FAMILY)


def make_streams(engine, n, seed=42, jump_log2=64):
    kind, _ = FAMILY[engine]
    base = rp.rp_create(engine).seed(seed)
    return rp.rp_streams_create(base, kind, n, jump_log2)


def oracle_stream(engine, i, seed=42, jump_log2=64):
    _, okind = FAMILY[engine]
    return oracle.substream(engine, seed, okind, int(i), jump_log2)


def ulp_diff(a, b):
    """Distance in units of the last place between float arrays of equal sign
    (binary32 arrays in binary32 ulps, anything else in binary64 ulps)."""
    if np.asarray(a).dtype == np.float32 and np.asarray(b).dtype == np.float32:
        ia = np.asarray(a).view(np.int32).astype(np.int64)
        ib = np.asarray(b).view(np.int32).astype(np.int64)
        return np.abs(ia - ib)
    ia = np.asarray(a, dtype=np.float64).view(np.int64)
    ib = np.asarray(b, dtype=np.float64).view(np.int64)
    return np.abs(ia - ib)


def oracle_fill(s, dist, dtype, n, bound=0, flags=0):
    """The serial definition of one rp_fill call on one oracle stream."""
    full = not (flags & rp.RP_FLAG_52BIT)
    if dist == rp.RP_RAW:
        return s.raw(n) if dtype == rp.RP_U64 else s.raw32(n)
    if dist == rp.RP_U01:
        return s.u01(n, full) if dtype == rp.RP_F64 else s.u01f(n, full)
    if dist == rp.RP_BOUNDED:
        return s.bounded64(bound, n) if dtype == rp.RP_U64 else s.bounded32(bound, n)
    if dist == rp.RP_NORM:
        return s.norm(n) if dtype == rp.RP_F64 else s.normf(n)
    if dist == rp.RP_EXP:
        return s.exp(n) if dtype == rp.RP_F64 else s.expf(n)
    raise ValueError(dist)


# torch has full support for signed integers only; the bits are reinterpreted
TORCH_DTYPE = {rp.RP_U64: "int64", rp.RP_U32: "int32", rp.RP_F64: "float64", rp.RP_F32: "float32"}
NP_VIEW = {rp.RP_U64: np.uint64, rp.RP_U32: np.uint32, rp.RP_F64: np.float64, rp.RP_F32: np.float32}
