#!/usr/bin/env python3
"""Benchmark of the bulk substream-generation hot path on one MI355X.

Workload (one "step"): Philox4x32-10 substreams (key = substream index) and
PCG64 substreams (increment 2 i + 1), base seed 42, 2^16 substreams x 2^14
values each (2^30 values per fill), filled as raw uint64, uniform float32,
uniform float64, standard normal float64 and standard exponential float64:
ten fills, 10 x 2^30 values per step.  Inputs (the substream states) are
resident in HBM before timing; the fills run back to back on one HIP stream.

Prints one JSON line: whole-step throughput in Gsamples/s, the roofline of the
dominant kernel (its average duration measured with HIP events on the launch
stream), per-fill figures, and the CPU oracle timed on a bounded sample of the
same workload on the host cores.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "Gsamples/s per engine x distribution, % HBM-write roofline; gamma grad/s"


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=5)
    p.add_argument("--warmup", type=int, default=2)
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--only", default="", help="comma-separated fill names to run (profiling)")
    p.add_argument("--calibrate-copy", action="store_true",
                   help="run only plain fill/copy kernels of known size (counter calibration)")
    return p.parse_args()


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


def cpu_baseline(target_cpu_s=12.0):
    """The oracle on the host cores, on a bounded sample of the workload:
    whole substreams of 2^14 values, both engines, all five outputs."""
    import concurrent.futures as cf

    import numpy as np

    import oracle
    from paper_2605_05099_amd import workloads

    per = workloads.SUB_PER
    kinds = [("philox4x32", "key"), ("pcg64", "inc")]
    outs = ["raw", "u01f", "u01", "norm", "exp"]

    def one(task):
        eng, kind, i, what = task
        s = oracle.substream(eng, workloads.BASE_SEED, kind, i)
        t0 = time.perf_counter()
        getattr(s, what)(per)
        return time.perf_counter() - t0

    # calibrate: one substream per (engine, output)
    cal = [one((e, k, 0, w)) for e, k in kinds for w in outs]
    per_round = sum(cal)  # CPU seconds for one substream of every fill
    rounds = max(1, int(target_cpu_s / per_round))
    threads = min(os.cpu_count() or 1, 16)
    tasks = [(e, k, i, w) for i in range(1, rounds + 1) for e, k in kinds for w in outs]
    t0 = time.perf_counter()
    with cf.ThreadPoolExecutor(max_workers=threads) as ex:
        cpu_s = sum(ex.map(one, tasks))
    wall = time.perf_counter() - t0
    n_values = len(tasks) * per
    return {"value": n_values / wall / 1e9, "unit": "Gsamples/s", "cores": threads, "kind": "oracle",
            "sample": f"{rounds} substreams x 2^14 values for each of the 10 fills "
                      f"({n_values} values, {cpu_s:.1f} CPU-s on {threads} threads)"}


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py: this build measures one GPU only (single-GPU box); "
              "run with --gpus 1", file=sys.stderr)
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
    # timed region: K steps, no per-kernel events (whole-job wall clock on the GPU)
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0.record(stream)
    for _ in range(args.steps):
        step()
    t1.record(stream)
    torch.cuda.synchronize()
    ms_total = t0.elapsed_time(t1)
    ms_step = ms_total / args.steps
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
                      "hbm_frac": round(total * nbytes / ms / 1e6 / HBM_PEAK_GBS, 4)}
    dom = max(fills, key=lambda f: per_kernel[f[0]])
    dom_ms = per_kernel[dom[0]]
    achieved = total * dom[4] / dom_ms / 1e6
    samples_step = total * len(fills)
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
        "roofline": {"bound": "hbm", "kernel": dom[0], "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                     "algorithmic_bytes_per_launch": total * dom[4], "avg_launch_ms": round(dom_ms, 4)},
        "rows": rows,
    }
    if not args.no_cpu_baseline:
        result["cpu_baseline"] = cpu_baseline()
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
