#!/usr/bin/env python3
"""Benchmark of the bulk substream-generation hot path on one MI355X.

Step (the figure in `value`): Philox4x32-10 substreams (key = substream index)
and PCG64 substreams (increment 2 i + 1), base seed 42, 2^16 substreams x 2^14
values each (2^30 values per fill), filled as raw uint64, uniform float32,
uniform float64, standard normal float64 and standard exponential float64:
ten fills, 10 x 2^30 values per step.  The substream states are resident in
HBM before timing; the fills run back to back on one HIP stream.

The same run also times the other parts of the path, each on its own
workload (`parts`): one x256++ stream split over lanes (10^6 values), batched
gamma and beta (10^6 sets, about 2.6e8 values, recorded graph, tuned plan),
per-element gamma / beta forward and backward ([4096, 1024]), multivariate
normal forward and backward (2^20 rows, d = 64, 256, 512), and the fused
per-substream moments (2^18 substreams x 2^16 normals, ranlux++ and sfc64).

Prints one JSON line: the step's throughput in Gsamples/s, the roofline of
its dominant kernel (average duration from HIP events on the launch stream;
HBM traffic from the committed counter summary when it still matches the
kernel sources), per-fill and per-part figures, and the CPU oracle timed on a
bounded sample of the step's workload on the host cores.
"""
import argparse
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FP32_MFMA_PEAK_TFLOPS = 157.3
# vector ALU: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz, one 32-bit (or binary64)
# lane operation per lane per cycle
ALU_PEAK_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12
# Algorithmic vector-ALU lane operations per value of each fill: engine
# operations per 64-bit word times words per value, plus the conversion or
# sampler's own operations (derivation in the design doc, section 6).
ENGINE_OPS_PER_WORD = {"philox4x32": 21.0, "pcg64": 26.0}
WORDS_PER_VALUE = {"u64": 1.0, "u01_f32": 0.5, "u01_f64": 1.0, "normal_f64": 1.0220, "exp_f64": 1.0336}
SAMPLER_OPS_PER_VALUE = {"u64": 0.0, "u01_f32": 3.0, "u01_f64": 4.0, "normal_f64": 11.0, "exp_f64": 11.0}


def alu_ops_per_value(fill):
    eng, out = fill.split("/")
    return ENGINE_OPS_PER_WORD[eng] * WORDS_PER_VALUE[out] + SAMPLER_OPS_PER_VALUE[out]


METRIC = "Gsamples/s per engine x distribution, % HBM-write roofline; gamma grad/s"
# counter summaries: profiles/pmc_fill_<engine>_<output>.md
TRAFFIC_SUMMARY = os.path.join(ROOT, "profiles", "pmc_fill_{}.md")
KERNEL_SOURCES = ["fill.hip", "engines.h", "rp_internal.h", "zig_tables.inc", "k_zig.h", "crmath.h", "crmath_tables.inc"]


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=5)
    p.add_argument("--warmup", type=int, default=2)
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--no-parts", action="store_true", help="time only the ten-fill step")
    p.add_argument("--parts", default=None,
                   help="comma-separated parts to time after the step: serial, batched, elem, mvn, "
                        "moments, laws, float, bitexact, engines, discrete, setup (default all; none with --only)")
    p.add_argument("--only", default="", help="comma-separated fill names to run (profiling)")
    p.add_argument("--calibrate-copy", action="store_true",
                   help="run only plain fill/copy kernels of known size (counter calibration)")
    return p.parse_args()


def kernel_source_hash():
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2605_05099_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(fill):
    """HBM bytes per launch of a fill kernel from its counter summary, or
    None when that summary is missing or was taken on other sources."""
    try:
        text = open(TRAFFIC_SUMMARY.format(fill.replace("/", "_").replace("+", "p"))).read()
    except OSError:
        return None
    src = re.search(r"^source_sha256_16:\s*([0-9a-f]+)", text, re.M)
    tot = re.search(r"^hbm_bytes_per_launch:\s*([0-9.eE+]+)", text, re.M)
    if not src or not tot or src.group(1) != kernel_source_hash():
        return None
    return float(tot.group(1))


def calibrate_copy(steps):
    """Known-size reference traffic for the HBM counters: a fill writing
    8 GiB and a copy reading 2 GiB and writing 2 GiB, per step."""
    import torch
    a = torch.empty(2**30, dtype=torch.float64, device="cuda")
    b = torch.empty(2**28, dtype=torch.float64, device="cuda")
    c = torch.empty(2**28, dtype=torch.float64, device="cuda")
    b.fill_(2.0)
    for _ in range(steps):
        a.fill_(1.0)
        c.copy_(b)
    torch.cuda.synchronize()
    print(json.dumps({"calibration": "fill 8 GiB write + copy 2 GiB read / 2 GiB write", "steps": steps}))


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.lower().startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(t1_s=1.6, tn_s=2.0):
    """The oracle on the host cores, on a bounded sample of the step's
    workload: whole substreams of 2^14 values, both engines, all five fills,
    the substreams continuing from fill to fill as on the GPU.  Threads run
    inside the C oracle (POSIX threads over contiguous substream ranges);
    timed once on one thread and once on every core this process may use."""
    import oracle
    from paper_2605_05099_amd import workloads

    per = workloads.SUB_PER
    threads = len(os.sched_getaffinity(0))
    kinds = [("philox4x32", "key"), ("pcg64", "inc")]
    # one substream per fill on one thread: seconds per 2^14 values
    cal = {}
    for eng, kind in kinds:
        s = [oracle.substream(eng, workloads.BASE_SEED, kind, 0)]
        for what in range(5):
            cal[eng, what] = max(oracle.time_fills(s, what, per, 1), 1e-6)
    res = {}
    for label, nthr, budget in (("t1", 1, t1_s), ("tn", threads, tn_s)):
        values = wall = 0.0
        subs = 0
        for eng, kind in kinds:
            k = max(nthr, int(budget * nthr / max(cal[eng, w] for w in range(5))))
            k -= k % nthr
            streams = [oracle.substream(eng, workloads.BASE_SEED, kind, i) for i in range(1, k + 1)]
            for what in range(5):
                wall += oracle.time_fills(streams, what, per, nthr)
                values += k * per
            subs += k
        res[label] = {"value": round(values / wall / 1e9, 4), "unit": "Gsamples/s", "threads": nthr,
                      "values": int(values), "wall_s": round(wall, 2), "substreams": subs}
    return {"value": res["tn"]["value"], "unit": "Gsamples/s", "cores": threads, "kind": "oracle",
            "threads": threads, "cpu": cpu_model(), "t1": res["t1"], "tn": res["tn"],
            "sample": f"the step's ten fills (philox4x32 key = i, pcg64 inc = 2i+1, seed 42; u64, u01 f32, "
                      f"u01 f64, normal f64, exponential f64) on whole substreams of 2^14 values continuing "
                      f"from fill to fill: {res['t1']['substreams']} substreams on 1 thread "
                      f"({res['t1']['wall_s']} s), {res['tn']['substreams']} substreams on {threads} threads "
                      f"({res['tn']['wall_s']} s wall); threads inside the C oracle"}


class Timer:
    """HIP events on one stream; ms per repetition of fn."""

    def __init__(self, torch, stream):
        self.torch, self.stream = torch, stream

    def __call__(self, fn, reps=3, warmup=1):
        t = self.torch
        for _ in range(warmup):
            fn()
        t.cuda.synchronize()
        a, b = t.cuda.Event(enable_timing=True), t.cuda.Event(enable_timing=True)
        a.record(self.stream)
        for _ in range(reps):
            fn()
        b.record(self.stream)
        t.cuda.synchronize()
        return a.elapsed_time(b) / reps


def parts(torch, rp, workloads, stream, only):
    """Every other row of the path on its own workload (see module doc)."""
    import numpy as np
    tm = Timer(torch, stream)
    sp = stream.cuda_stream
    out = {}
    if "serial" in only:
        out.update(part_serial(torch, rp, workloads, tm, sp))
    if "batched" in only:
        out.update(part_batched(torch, rp, workloads, tm, sp))
    if "elem" in only:
        out.update(part_elem(torch, rp, workloads, tm, sp, np))
    if "mvn" in only:
        out.update(part_mvn(torch, rp, workloads, tm, sp, np))
    if "moments" in only:
        out.update(part_moments(torch, rp, workloads, tm, sp))
    if "laws" in only:
        out.update(part_laws(torch, rp, workloads, tm, sp))
    if "float" in only:
        out.update(part_float(torch, rp, workloads, tm, sp))
    if "bitexact" in only:
        out.update(part_bitexact(torch, rp, workloads, tm, sp))
    if "engines" in only:
        out.update(part_engines(torch, rp, workloads, tm, sp))
    if "discrete" in only:
        out.update(part_discrete(torch, rp, workloads, tm, sp))
    if "setup" in only:
        out.update(part_setup(torch, rp, workloads))
    return out


def part_serial(torch, rp, workloads, tm, sp):
    out = {}

    # one stream split over lanes: x256++ seed 12345, 10^6 values each
    n = workloads.SERIAL_N
    buf = torch.empty(n, dtype=torch.float64, device="cuda")
    ser = {}
    for name, dist, dtype in (("raw_u64", rp.RP_RAW, rp.RP_U64), ("u01_f64", rp.RP_U01, rp.RP_F64),
                              ("normal_f64", rp.RP_NORM, rp.RP_F64), ("exp_f64", rp.RP_EXP, rp.RP_F64),
                              ("normal_f32", rp.RP_NORM, rp.RP_F32), ("exp_f32", rp.RP_EXP, rp.RP_F32)):
        rng = rp.rp_create("x256++").seed(workloads.SERIAL_SEED)
        ms = tm(lambda: rp.rp_fill_serial(rng, dist, dtype, 0, 0, buf, n, sp), reps=5)
        ser[name] = {"ms": round(ms, 4), "gsamples_s": round(n / ms / 1e6, 3)}
    out["serial_x256pp_1e6"] = ser
    # throughput form: the same stream, 2^30 raw words over 2^16 lanes
    n30 = 2**30
    big = torch.empty(n30, dtype=torch.int64, device="cuda")
    rng = rp.rp_create("x256++").seed(workloads.SERIAL_SEED)
    ms = tm(lambda: rp.rp_fill_serial(rng, rp.RP_RAW, rp.RP_U64, 0, 0, big, n30, sp), reps=3)
    out["serial_x256pp_2p30_raw"] = {"ms": round(ms, 4), "gsamples_s": round(n30 / ms / 1e6, 2),
                                     "write_gb_s": round(n30 * 8 / ms / 1e6, 1),
                                     "hbm_frac": round(n30 * 8 / ms / 1e6 / HBM_PEAK_GBS, 4)}
    del big
    return out


def part_batched(torch, rp, workloads, tm, sp):
    out = {}
    w = workloads.batched_sets()
    nsets = len(w["alpha"])
    bat = {}
    for kind, params, count in (("gamma", (w["alpha"],), w["count"]), ("beta", (w["a"], w["b"]), w["count_beta"])):
        total = int(count.sum())
        o = torch.empty(total, dtype=torch.float64, device="cuda")
        dp = [torch.as_tensor(p, device="cuda") for p in params]
        dc = torch.as_tensor(count, device="cuda")
        S = rp.rp_streams_create(rp.rp_create("philox4x32").seed(workloads.BASE_SEED), rp.RP_SUB_KEY, nsets)
        plan = rp.rp_plan_create()
        rp.rp_plan_autotune(plan, S, kind == "beta", dp[0], dp[1] if kind == "beta" else None, dc, nsets, o)
        if kind == "gamma":
            fn = lambda: rp.rp_gamma_batched(S, dp[0], dc, nsets, o, plan, sp)  # noqa: E731
        else:
            fn = lambda: rp.rp_beta_batched(S, dp[0], dp[1], dc, nsets, o, plan, sp)  # noqa: E731
        ms = tm(fn, reps=5)
        bat[kind] = {"ms": round(ms, 4), "samples": total, "gsamples_s": round(total / ms / 1e6, 3),
                     "write_gb_s": round(total * 8 / ms / 1e6, 1),
                     "hbm_write_frac": round(total * 8 / ms / 1e6 / HBM_PEAK_GBS, 4), "plan": plan.get_config()}
        del o, S, plan
    out["batched_1e6_sets"] = bat
    return out


def part_elem(torch, rp, workloads, tm, sp, np):
    out = {}
    pe = workloads.per_element()
    ne = int(np.prod(workloads.PER_ELEMENT_SHAPE))
    S = rp.rp_streams_create(rp.rp_create("philox4x32").seed(workloads.BASE_SEED), rp.RP_SUB_KEY, ne)
    al = torch.as_tensor(pe["alpha"].reshape(-1), device="cuda")
    a = torch.as_tensor(pe["a"].reshape(-1), device="cuda")
    b = torch.as_tensor(pe["b"].reshape(-1), device="cuda")
    gz = torch.as_tensor(pe["gz"].reshape(-1), device="cuda")
    z = torch.empty(ne, dtype=torch.float32, device="cuda")
    zb = torch.empty(ne, dtype=torch.float32, device="cuda")
    g1 = torch.empty(ne, dtype=torch.float32, device="cuda")
    g2 = torch.empty(ne, dtype=torch.float32, device="cuda")
    el = {}
    ms = tm(lambda: rp.rp_gamma_elem(S, al, z, ne, sp))
    el["gamma_fwd"] = {"ms": round(ms, 4), "gsamples_s": round(ne / ms / 1e6, 3)}
    ms = tm(lambda: rp.rp_gamma_grad(z, al, gz, g1, ne, sp))
    el["gamma_bwd"] = {"ms": round(ms, 4), "ggrad_s": round(ne / ms / 1e6, 3),
                       "hbm_gb_s": round(ne * 16 / ms / 1e6, 1)}
    ms = tm(lambda: rp.rp_beta_elem(S, a, b, zb, ne, sp))
    el["beta_fwd"] = {"ms": round(ms, 4), "gsamples_s": round(ne / ms / 1e6, 3)}
    ms = tm(lambda: rp.rp_beta_grad(zb, a, b, gz, g1, g2, ne, sp))
    el["beta_bwd"] = {"ms": round(ms, 4), "ggrad_s": round(ne / ms / 1e6, 3),
                      "hbm_gb_s": round(ne * 24 / ms / 1e6, 1)}
    out["per_element_4096x1024"] = el
    return out


def part_mvn(torch, rp, workloads, tm, sp, np):
    out = {}
    mv = {}
    nr = workloads.MVN_N
    for d in workloads.MVN_DIMS:
        wm = workloads.mvn(d)
        L = torch.as_tensor(rp.rp_cholesky(wm["sigma"]).astype(np.float32), device="cuda")
        mu = torch.as_tensor(wm["mu"].astype(np.float32), device="cuda")
        S = rp.rp_streams_create(rp.rp_create("philox4x32").seed(workloads.BASE_SEED), rp.RP_SUB_KEY, nr)
        X = torch.empty((nr, d), dtype=torch.float32, device="cuda")
        ms_f = tm(lambda: rp.rp_mvn(S, mu, L, d, nr, X, sp))
        G = torch.ones((nr, d), dtype=torch.float32, device="cuda")
        gm = torch.empty(d, dtype=torch.float32, device="cuda")
        gL = torch.empty((d, d), dtype=torch.float32, device="cuda")
        ms_b = tm(lambda: rp.rp_mvn_backward(S, G, d, nr, gm, gL, sp))
        # the method's own flops: row i needs sum_c (c + 1) multiply-adds with
        # a lower-triangular L, i.e. d (d + 1) flops (2 d^2 for a full matrix)
        fl = 1.0 * nr * d * (d + 1)
        mv[f"d{d}"] = {"fwd_ms": round(ms_f, 4), "fwd_tflops": round(fl / ms_f / 1e9, 2),
                       "fwd_mfma_frac": round(fl / ms_f / 1e9 / FP32_MFMA_PEAK_TFLOPS, 4),
                       "flops_per_row": d * (d + 1),
                       "bwd_ms": round(ms_b, 4), "bwd_tflops": round(fl / ms_b / 1e9, 2),
                       "rows_per_s_g": round(nr / ms_f / 1e6, 3)}
        del S, X, G
    out["mvn_2p20_rows"] = mv
    return out


def part_moments(torch, rp, workloads, tm, sp):
    out = {}
    mo = {}
    nm, pm = workloads.MOM_N, workloads.MOM_PER
    s1 = torch.empty(nm, dtype=torch.float64, device="cuda")
    s2 = torch.empty(nm, dtype=torch.float64, device="cuda")
    for eng, kind in (("ranlux++", rp.RP_SUB_JUMP), ("sfc64", rp.RP_SUB_SPAWN)):
        S = rp.rp_streams_create(rp.rp_create(eng).seed(workloads.BASE_SEED), kind, nm, 64)
        ms = tm(lambda: rp.rp_norm_moments(S, pm, s1, s2, sp), reps=2)
        mo[eng] = {"ms": round(ms, 3), "gsamples_s": round(nm * pm / ms / 1e6, 3)}
        del S
    out["moments_2p18x2p16"] = mo
    return out


def part_laws(torch, rp, workloads, tm, sp):
    """Derived laws on the substream workload: Philox4x32-10, 2^16 substreams
    x 2^14 values.  Transform laws fuse one transform into the base fill's
    store; the laws of several draws per value (gamma, beta, chi-square, t,
    F, skew-normal) run one lane per substream."""
    n, per = workloads.SUB_N, workloads.SUB_PER
    S = rp.rp_streams_create(rp.rp_create("philox4x32").seed(workloads.BASE_SEED), rp.RP_SUB_KEY, n)
    buf = torch.empty(n * per, dtype=torch.float64, device="cuda")
    res = {}
    for name, law, p in (("unif", rp.RP_LAW_UNIF, (-2.0, 5.0)), ("normal", rp.RP_LAW_NORMAL, (3.0, 5.0)),
                         ("lognormal", rp.RP_LAW_LOGNORMAL, (0.5, 0.75)), ("exp", rp.RP_LAW_EXP, (2.5,)),
                         ("gumbel", rp.RP_LAW_GUMBEL, (1.0, 2.0)), ("pareto", rp.RP_LAW_PARETO, (1.5, 3.0)),
                         ("gpareto", rp.RP_LAW_GPARETO, (0.5, 2.0, 0.3)), ("weibull", rp.RP_LAW_WEIBULL, (1.7, 4.0)),
                         ("gamma", rp.RP_LAW_GAMMA, (2.5, 1.5)), ("gamma_0.4", rp.RP_LAW_GAMMA, (0.4, 1.0)),
                         ("beta", rp.RP_LAW_BETA, (2.0, 5.0)), ("chi2", rp.RP_LAW_CHI2, (3.0,)),
                         ("t", rp.RP_LAW_T, (4.5,)), ("F", rp.RP_LAW_F, (5.0, 7.0)),
                         ("skewnormal", rp.RP_LAW_SKEWNORMAL, (1.0, 2.0, 3.0))):
        ms = tm(lambda: rp.rp_fill_law(S, law, p, buf, per, sp), reps=3)
        res[name] = {"ms": round(ms, 4), "gsamples_s": round(n * per / ms / 1e6, 2),
                     "hbm_frac": round(8.0 * n * per / ms / 1e6 / HBM_PEAK_GBS, 4)}
    del buf, S
    return {"laws_philox4x32_2p16x2p14": res}


def part_bitexact(torch, rp, workloads, tm, sp):
    """The bitexact setting (correctly rounded exp / log / log1p / pow) on
    the substream workload, Philox4x32-10: time with the setting on, and the
    ratio to the same call with it off."""
    n, per = workloads.SUB_N, workloads.SUB_PER
    buf = torch.empty(n * per, dtype=torch.float64, device="cuda")
    res = {}
    cases = (("normal", None, rp.RP_NORM, ()), ("exp", None, rp.RP_EXP, ()),
             ("lognormal", rp.RP_LAW_LOGNORMAL, None, (0.5, 0.75)), ("gumbel", rp.RP_LAW_GUMBEL, None, (1.0, 2.0)),
             ("pareto", rp.RP_LAW_PARETO, None, (1.5, 3.0)), ("weibull", rp.RP_LAW_WEIBULL, None, (1.7, 4.0)),
             ("gamma", rp.RP_LAW_GAMMA, None, (2.5, 1.5)), ("gamma_0.4", rp.RP_LAW_GAMMA, None, (0.4, 1.0)),
             ("beta", rp.RP_LAW_BETA, None, (2.0, 5.0)))
    for name, law, dist, p in cases:
        ms = {}
        for on in (0, 1):
            S = rp.rp_streams_create(rp.rp_create("philox4x32").seed(workloads.BASE_SEED), rp.RP_SUB_KEY, n)
            S.set_flag(rp.RP_BITEXACT, on)
            if law is None:
                ms[on] = tm(lambda: rp.rp_fill(S, dist, rp.RP_F64, 0, 0, buf, per, sp), reps=3)
            else:
                ms[on] = tm(lambda: rp.rp_fill_law(S, law, p, buf, per, sp), reps=3)
            del S
        res[name] = {"ms": round(ms[1], 4), "gsamples_s": round(n * per / ms[1] / 1e6, 2),
                     "slowdown": round(ms[1] / ms[0], 3)}
    del buf
    return {"bitexact_philox4x32_2p16x2p14": res}


def part_float(torch, rp, workloads, tm, sp):
    """Float ziggurat normal and exponential (binary32 draws from 32-bit
    items) on the substream workload, both wavefront engines; binary32 laws
    (transforms and the float gamma) on Philox4x32-10."""
    n, per = workloads.SUB_N, workloads.SUB_PER
    buf = torch.empty(n * per, dtype=torch.float32, device="cuda")
    res = {}
    for eng, kind in (("philox4x32", rp.RP_SUB_KEY), ("pcg64", rp.RP_SUB_INC)):
        S = rp.rp_streams_create(rp.rp_create(eng).seed(workloads.BASE_SEED), kind, n)
        for name, dist in (("normal_f32", rp.RP_NORM), ("exp_f32", rp.RP_EXP)):
            ms = tm(lambda: rp.rp_fill(S, dist, rp.RP_F32, 0, 0, buf, per, sp), reps=3)
            res[f"{eng}/{name}"] = {"ms": round(ms, 4), "gsamples_s": round(n * per / ms / 1e6, 2),
                                    "hbm_frac": round(4.0 * n * per / ms / 1e6 / HBM_PEAK_GBS, 4)}
        if eng == "philox4x32":
            for name, law, p in (("lawf_unif", rp.RP_LAW_UNIF, (-2.0, 5.0)),
                                 ("lawf_lognormal", rp.RP_LAW_LOGNORMAL, (0.5, 0.75)),
                                 ("lawf_weibull", rp.RP_LAW_WEIBULL, (1.7, 4.0)),
                                 ("lawf_gamma", rp.RP_LAW_GAMMA, (2.5, 1.5))):
                ms = tm(lambda: rp.rp_fill_lawf(S, law, p, buf, per, sp), reps=3)
                res[f"{eng}/{name}"] = {"ms": round(ms, 4), "gsamples_s": round(n * per / ms / 1e6, 2)}
        del S
    del buf
    return {"float_zig_2p16x2p14": res}


def part_engines(torch, rp, workloads, tm, sp):
    """Raw u64 and normal f64 fills of every engine on the substream
    workload's shape (2^16 substreams x 2^14 values): wavefront engines
    (philox4x32, philox, pcg64, squares, chacha20) and lane engines (x256++, x256**,
    sfc64, ranlux++, xoro++, x128+)."""
    n, per = workloads.SUB_N, workloads.SUB_PER
    buf = torch.empty(n * per, dtype=torch.float64, device="cuda")
    kinds = {"philox4x32": rp.RP_SUB_KEY, "philox": rp.RP_SUB_KEY, "pcg64": rp.RP_SUB_INC,
             "squares": rp.RP_SUB_SPAWN, "x256++": rp.RP_SUB_JUMP, "x256**": rp.RP_SUB_JUMP,
             "sfc64": rp.RP_SUB_SPAWN, "ranlux++": rp.RP_SUB_JUMP, "xoro++": rp.RP_SUB_JUMP,
             "x128+": rp.RP_SUB_JUMP, "chacha20": rp.RP_SUB_KEY}
    res = {}
    for eng, kind in kinds.items():
        S = rp.rp_streams_create(rp.rp_create(eng).seed(workloads.BASE_SEED), kind, n, 64)
        for name, dist, dtype in (("u64", rp.RP_RAW, rp.RP_U64), ("normal_f64", rp.RP_NORM, rp.RP_F64)):
            ms = tm(lambda: rp.rp_fill(S, dist, dtype, 0, 0, buf, per, sp), reps=2)
            res[f"{eng}/{name}"] = {"ms": round(ms, 4), "gsamples_s": round(n * per / ms / 1e6, 2),
                                    "hbm_frac": round(8.0 * n * per / ms / 1e6 / HBM_PEAK_GBS, 4)}
        del S
    del buf
    return {"engines_2p16x2p14": res}


def part_discrete(torch, rp, workloads, tm, sp):
    """Batched permutations and samples, one instance per substream
    (Philox4x32-10, 2^16 substreams): permutations of 1024 (rows in HBM) and
    512 (rows in LDS), Floyd samples of 64 from 10^6, reservoir samples of
    900 from 1000."""
    m = workloads.SUB_N
    S = rp.rp_streams_create(rp.rp_create("philox4x32").seed(workloads.BASE_SEED), rp.RP_SUB_KEY, m)
    res = {}
    buf = torch.empty(m * 1024, dtype=torch.int32, device="cuda")
    for pn in (1024, 512):
        ms = tm(lambda: rp.rp_permutations(S, pn, buf, sp), reps=3)
        res[f"permutation_{pn}"] = {"ms": round(ms, 4), "instances_per_s_m": round(m / ms / 1e3, 3),
                                    "gelem_s": round(m * pn / ms / 1e6, 3)}
    for name, n, k in (("floyd_64_of_1e6", 10**6, 64), ("reservoir_900_of_1000", 1000, 900)):
        ms = tm(lambda: rp.rp_sample(S, n, k, buf, sp), reps=3)
        res[name] = {"ms": round(ms, 4), "instances_per_s_m": round(m / ms / 1e3, 3)}
    del buf, S
    return {"discrete_2p16": res}


def part_setup(torch, rp, workloads):
    """Substream construction (host seeding and per-substream keys, increments,
    spawn keys or jumps, then the copy to device), timed on its own: it is
    outside every timed region above."""
    import time
    cases = (("philox4x32_key_2p16", "philox4x32", rp.RP_SUB_KEY, workloads.SUB_N, 0),
             ("pcg64_inc_2p16", "pcg64", rp.RP_SUB_INC, workloads.SUB_N, 0),
             ("philox4x32_key_1e6", "philox4x32", rp.RP_SUB_KEY, 10**6, 0),
             ("ranlux_jump64_2p18", "ranlux++", rp.RP_SUB_JUMP, workloads.MOM_N, 64),
             ("sfc64_spawn_2p18", "sfc64", rp.RP_SUB_SPAWN, workloads.MOM_N, 0))
    res = {}
    for name, eng, kind, n, stride in cases:
        base = rp.rp_create(eng).seed(workloads.BASE_SEED)
        best = None
        for _ in range(2):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            S = rp.rp_streams_create(base, kind, n, stride)
            torch.cuda.synchronize()
            dt = (time.perf_counter() - t0) * 1e3
            best = dt if best is None else min(best, dt)
            del S
        res[name] = {"ms": round(best, 3), "substreams": n}
    return {"substream_setup": res}


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py: only single-GPU runs are supported (every workload runs on one GPU; "
              "the multi-GPU split is described, not built); run with --gpus 1", file=sys.stderr)
        sys.exit(2)
    import torch

    import paper_2605_05099_amd as rp
    from paper_2605_05099_amd import workloads

    torch.cuda.set_device(0)
    if args.calibrate_copy:
        calibrate_copy(args.steps)
        return
    n, per = workloads.SUB_N, workloads.SUB_PER
    total = n * per
    streams = {
        "philox4x32": rp.rp_streams_create(rp.rp_create("philox4x32").seed(workloads.BASE_SEED), rp.RP_SUB_KEY, n),
        "pcg64": rp.rp_streams_create(rp.rp_create("pcg64").seed(workloads.BASE_SEED), rp.RP_SUB_INC, n),
    }
    buf = torch.empty(total, dtype=torch.float64, device="cuda")
    fills = []
    for eng in ("philox4x32", "pcg64"):
        for name, dist, dtype, nbytes in (("u64", rp.RP_RAW, rp.RP_U64, 8), ("u01_f32", rp.RP_U01, rp.RP_F32, 4),
                                          ("u01_f64", rp.RP_U01, rp.RP_F64, 8), ("normal_f64", rp.RP_NORM, rp.RP_F64, 8),
                                          ("exp_f64", rp.RP_EXP, rp.RP_F64, 8)):
            fills.append((f"{eng}/{name}", eng, dist, dtype, nbytes))
    if args.only:
        keep = set(args.only.split(","))
        fills = [f for f in fills if f[0] in keep]
    stream = torch.cuda.current_stream()

    def step(events=None):
        for k, (name, eng, dist, dtype, _) in enumerate(fills):
            if events is not None:
                events[k][0].record(stream)
            rp.rp_fill(streams[eng], dist, dtype, 0, 0, buf.data_ptr(), per, stream.cuda_stream)
            if events is not None:
                events[k][1].record(stream)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    # timed region: K steps, no per-kernel events (whole-job time on the GPU)
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0.record(stream)
    for _ in range(args.steps):
        step()
    t1.record(stream)
    torch.cuda.synchronize()
    ms_step = t0.elapsed_time(t1) / args.steps
    # per-kernel durations: a separate pass of K steps with events around each launch
    per_kernel = {f[0]: 0.0 for f in fills}
    for _ in range(args.steps):
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in fills]
        step(ev)
        torch.cuda.synchronize()
        for (name, *_), (a, b) in zip(fills, ev):
            per_kernel[name] += a.elapsed_time(b) / args.steps
    rows = {}
    for name, eng, dist, dtype, nbytes in fills:
        ms = per_kernel[name]
        rows[name] = {"ms": round(ms, 4), "gsamples_s": round(total / ms / 1e6, 2),
                      "write_gb_s": round(total * nbytes / ms / 1e6, 1),
                      "hbm_frac": round(total * nbytes / ms / 1e6 / HBM_PEAK_GBS, 4),
                      "alu_frac": round(total * alu_ops_per_value(name) / ms / 1e9 / ALU_PEAK_TOPS, 4)}
    dom = max(fills, key=lambda f: per_kernel[f[0]])
    dom_ms = per_kernel[dom[0]]
    achieved = total * dom[4] / dom_ms / 1e6
    ops = alu_ops_per_value(dom[0])
    alu_achieved = total * ops / dom_ms / 1e9  # Top/s
    # the binding roofline is the lower of the two ceilings on values per second
    alu_binds = ALU_PEAK_TOPS * 1e12 / ops < HBM_PEAK_GBS * 1e9 / dom[4]
    traffic = measured_traffic(dom[0])
    samples_step = total * len(fills)
    del buf
    result = {
        "metric": METRIC,
        "value": round(samples_step / ms_step / 1e6, 3),
        "unit": "Gsamples/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "substream bulk generation: philox4x32-10 (key = i) and pcg64 (inc = 2i+1), "
                               "seed 42, 2^16 substreams x 2^14 values; u64, u01 f32, u01 f64, normal f64, "
                               "exponential f64 (10 fills of 2^30 values per step)",
                   "substreams": n, "per_substream": per, "fills": [f[0] for f in fills]},
        "roofline": {"bound": "alu" if alu_binds else "hbm", "kernel": dom[0],
                     "achieved": round(alu_achieved, 3) if alu_binds else round(achieved, 1),
                     "peak": round(ALU_PEAK_TOPS, 2) if alu_binds else HBM_PEAK_GBS,
                     "unit": "Top/s" if alu_binds else "GB/s",
                     "frac": round(alu_achieved / ALU_PEAK_TOPS if alu_binds else achieved / HBM_PEAK_GBS, 4),
                     "traffic": traffic,
                     "hbm_frac": round(achieved / HBM_PEAK_GBS, 4),
                     "alu_frac": round(alu_achieved / ALU_PEAK_TOPS, 4),
                     "valu_frac": round(alu_achieved / ALU_PEAK_TOPS, 4),  # the same vector-ALU fraction
                     "alu_ops_per_value": round(ops, 2),
                     "algorithmic_bytes_per_launch": total * dom[4], "avg_launch_ms": round(dom_ms, 4)},
        "rows": rows,
    }
    want = args.parts if args.parts is not None else ("" if args.only else "serial,batched,elem,mvn,moments,laws,float,bitexact,engines,discrete,setup")
    if not args.no_parts and want:
        result["parts"] = parts(torch, rp, workloads, stream, set(want.split(",")))
    if not args.no_cpu_baseline:
        result["cpu_baseline"] = cpu_baseline()
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
