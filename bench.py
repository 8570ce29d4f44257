#!/usr/bin/env python3
"""Benchmark: included and excluded sums of a 512^3 fp32 tensor, box 16^3.

One step = the whole hot path on one resident input: included and excluded
sums under + and under max (two library calls).  ``value`` is the excluded-sum
throughput in Gelem/s: elements of excluded-sum output per second
(2 * N per step).  Prints ONE JSON line.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]

Only one GPU is used; ``--gpus`` above 1 exits with a message.
"""
from __future__ import annotations

import argparse
import ctypes
import json
import os
import platform
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, HERE)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, 8 TB/s


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=10)
    p.add_argument("--warmup", type=int, default=3)
    p.add_argument("--workload", default="d3_512_f32")
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--no-check", action="store_true")
    p.add_argument("--no-copy-probe", action="store_true",
                   help="skip the plain device copy of the input (bandwidth ceiling)")
    p.add_argument("--no-configs", action="store_true",
                   help="skip the other single-tensor workloads (64x64 int64, 32^5 fp32, "
                        "128x128x64x64 int32)")
    p.add_argument("--sweep-d", action="store_true",
                   help="instead of the headline step: excluded sums of fp32 tensors of about "
                        "2^21, 2^24 and 2^27 elements for d = 1..8, box side 8 (strong and "
                        "weak, +)")
    p.add_argument("--sweep-log2n", type=int, nargs="+", default=[21, 24, 27],
                   help="log2 of the element counts of the rank sweep")
    p.add_argument("--sweep-n", action="store_true",
                   help="instead of the headline step: excluded sums of fp32 cubes n^3 for "
                        "n = 64..640, box 16^3, + (time per element against N)")
    p.add_argument("--sweep-op-cost", action="store_true",
                   help="instead of the headline step: included and excluded sums of a 3-D "
                        "fp32 tensor under an artificially slowed + (cost steps per "
                        "application), time per element divided by the time per application")
    p.add_argument("--op-costs", type=int, nargs="+", default=[0, 16, 64, 256, 1024, 4096])
    p.add_argument("--op-cost-shape", type=int, nargs="+", default=[128, 128, 128])
    p.add_argument("--op-cost-box", type=int, nargs="+", default=[4, 4, 4])
    p.add_argument("--case", type=str, default=None,
                   help="time one plain call instead of the default step: comma-separated "
                        "fp32 shape (device counter fill), with --box, --op and --mode")
    p.add_argument("--box", type=str, default=None, help="comma-separated box for --case")
    p.add_argument("--op", type=str, default="sum", help="operator for --case")
    p.add_argument("--mode", type=str, default="both", help="mode for --case (inc, exc, both)")
    p.add_argument("--no-corners", action="store_true",
                   help="skip the corners-algorithm comparison (2-D)")
    p.add_argument("--sweep-corners", action="store_true",
                   help="box-complement vs the corners algorithm on 2-D tensors of several "
                        "sizes and boxes: one JSON line per case")
    p.add_argument("--no-weak", action="store_true",
                   help="skip the weak excluded sums (total - included) for +")
    p.add_argument("--no-batched", action="store_true", help="skip the batched form")
    p.add_argument("--no-served", action="store_true", help="skip the serving form")
    p.add_argument("--batch-count", type=int, default=512)
    p.add_argument("--batch-check-points", type=int, default=500,
                   help="sampled cells per batched tensor checked against the oracle")
    p.add_argument("--serve-seconds", type=float, default=60.0,
                   help="window of the 2000 req/s Poisson stream that is served")
    p.add_argument("--serial-seconds", type=float, default=10.0,
                   help="window of the same arrivals run through the serial plain path")
    p.add_argument("--serve-check", type=int, default=48,
                   help="served requests whose results are checked at sampled cells")
    p.add_argument("--serve-budget-gib", type=float, default=32.0)
    p.add_argument("--serve-inflight", type=int, default=8)
    return p.parse_args()


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def read_timings(L):
    names = ctypes.create_string_buffer(64 * 64)
    launches = (ctypes.c_int64 * 64)()
    total = (ctypes.c_double * 64)()
    cnt = ctypes.c_int32()
    rc = L.exs_timing_read(64, names, launches, total, ctypes.byref(cnt))
    if rc != 0:
        raise RuntimeError(L.exs_last_error().decode())
    out = {}
    for i in range(cnt.value):
        nm = names.raw[64 * i: 64 * i + 64].split(b"\0", 1)[0].decode()
        out[nm] = (int(launches[i]), float(total[i]))
    return out


def algorithmic_bytes(kernel, N, es, outputs):
    """Bytes a launch of `kernel` must move at level 0: read the input once
    and write each output once (the read-A-once / write-outputs-once minimum
    of one pass)."""
    base = kernel.split("@")[0]
    if base in ("k_axis0", "k_plane_axis0"):
        return N * es * (1 + outputs)
    if base in ("k_bdbs", "k_plane_bdbs"):
        return 2 * N * es
    if base in ("k_blockagg", "k_blockagg4"):
        return N * es
    return None


def overhead_bytes(kernel, N, es, k0):
    """Reads a launch makes beyond its algorithmic bytes by design: the stream
    kernel reads the block-suffix plane (one element per point and block)."""
    base = kernel.split("@")[0]
    if base in ("k_axis0", "k_plane_axis0"):
        return (N // k0) * es
    return 0


TRAFFIC_SOURCES = ("exsum_plane.hpp", "exsum_device.hpp")


def kernel_source_hash():
    """sha256 over the sources of the fused streaming kernel."""
    import hashlib
    h = hashlib.sha256()
    d = os.path.join(HERE, "paper_2106_00124_amd", "csrc")
    for f in TRAFFIC_SOURCES:
        with open(os.path.join(d, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def profile_summary(kernel, workload):
    """The committed rocprofv3 summary of `kernel` on `workload`: its traced
    average launch duration and its HBM bytes per launch (FETCH_SIZE and
    WRITE_SIZE, calibrated by a plain copy), or None when there is none or the
    kernel source changed since it was taken."""
    path = os.path.join(HERE, "profiles", f"{kernel}_{workload}.md")
    if not os.path.exists(path):
        return None
    vals = {}
    with open(path) as fh:
        for line in fh:
            line = line.strip().lstrip("-* ").strip("`")
            if ":" in line:
                k, v = line.split(":", 1)
                vals[k.strip()] = v.strip()
    try:
        if vals.get("kernel_source_sha256") != kernel_source_hash():
            return None
        out = {"file": os.path.relpath(path, HERE),
               "trace_avg_launch_us": float(vals["trace_avg_launch_us"])}
        if "fetch_bytes_per_launch" in vals:
            out["fetch"] = int(vals["fetch_bytes_per_launch"])
            out["write"] = int(vals["write_bytes_per_launch"])
        return out
    except (KeyError, ValueError):
        return None


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or platform.machine()


def main():
    args = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus > 1 or world > 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; "
                                   "the multi-GPU sharding is a design, not a build",
                          "n_gpus": args.gpus}), flush=True)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2106_00124_amd as P
    if args.sweep_d:
        sweep_d(args, P, torch, np)
        return
    if args.sweep_n:
        sweep_n(args, P, torch, np)
        return
    if args.sweep_op_cost:
        sweep_op_cost(args, P, torch, np)
        return
    if args.case:
        bench_case(args, P, torch, np)
        return
    if args.sweep_corners:
        for n in (1024, 4096, 8192, 16384):
            for k in (4, 16, 64):
                r = bench_corners(args, P, torch, np, (n, n), (k, k), ("sum", "max"))
                print(json.dumps(r), flush=True)
        return
    from paper_2106_00124_amd import _lib
    from paper_2106_00124_amd.workloads import WORKLOADS

    w = WORKLOADS[args.workload]
    N = w.n
    dt = {"f32": torch.float32, "f64": torch.float64, "i32": torch.int32,
          "i64": torch.int64}[w.dtype]
    es = torch.tensor([], dtype=dt).element_size()
    log(f"workload {w.name} shape={w.shape} box={w.box} dtype={w.dtype} ops={w.ops}")

    t0 = time.time()
    a_host = w.tensor()
    log(f"input generated in {time.time() - t0:.1f}s")
    dev = torch.device("cuda:0")
    a = torch.from_numpy(a_host).to(dev)
    outs = {op: (torch.empty_like(a), torch.empty_like(a)) for op in w.ops}
    ws_bytes = max(P.workspace_size(w.shape, w.box, dt, op, "both") for op in w.ops)
    if "sum" in w.ops:
        ws_bytes = max(ws_bytes, P.workspace_size(w.shape, w.box, dt, "sum", "both_weak"))
    ws = torch.empty(max(ws_bytes, 1), dtype=torch.uint8, device=dev)
    stream = torch.cuda.current_stream()
    L = _lib.lib()

    def step():
        for op in w.ops:
            inc, exc = outs[op]
            P.run(a, w.box, op, "both", inc_out=inc, exc_out=exc, workspace=ws, stream=stream)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    log(f"warmup done ({args.warmup} steps)")

    # timed region: K whole steps, bracketed by synchronisation, no
    # instrumentation inside
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    for _ in range(args.steps):
        step()
    ev1.record(stream)
    torch.cuda.synchronize()
    t_wall = time.perf_counter() - t_start
    gpu_ms = ev0.elapsed_time(ev1)
    ms_per_step = gpu_ms / args.steps
    log(f"timed {args.steps} steps: {ms_per_step:.3f} ms/step (wall {1e3 * t_wall / args.steps:.3f})")

    # the same K steps again with a HIP event pair around every kernel launch,
    # recorded by the library on the launch stream: per-kernel durations
    L.exs_timing_enable(1)
    read_timings(L)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(args.steps):
        step()
    e1.record(stream)
    torch.cuda.synchronize()
    L.exs_timing_enable(0)
    kt = read_timings(L)
    inst_ms_per_step = e0.elapsed_time(e1) / args.steps
    log(f"instrumented: {inst_ms_per_step:.3f} ms/step")
    for nm, (n_l, tot) in sorted(kt.items(), key=lambda kv: -kv[1][1]):
        log(f"  {nm:28s} launches={n_l:5d} avg={tot / n_l * 1e3:9.1f} us total={tot:8.2f} ms")

    # per-op timing (separately, for the record)
    per_op = {}
    for op in w.ops:
        inc, exc = outs[op]
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(max(1, args.steps // 2)):
            P.run(a, w.box, op, "both", inc_out=inc, exc_out=exc, workspace=ws, stream=stream)
        e1.record(stream)
        torch.cuda.synchronize()
        per_op[op] = e0.elapsed_time(e1) / max(1, args.steps // 2)

    # weak excluded sums for + (total - included), for the record: timed and
    # spot-checked on their own, not part of the step
    weak = None
    if "sum" in w.ops and not args.no_weak:
        wi, we = torch.empty_like(a), torch.empty_like(a)
        P.run(a, w.box, "sum", "both_weak", inc_out=wi, exc_out=we, workspace=ws, stream=stream)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        reps = max(1, args.steps // 2)
        e0.record(stream)
        for _ in range(reps):
            P.run(a, w.box, "sum", "both_weak", inc_out=wi, exc_out=we, workspace=ws,
                  stream=stream)
        e1.record(stream)
        torch.cuda.synchronize()
        wms = e0.elapsed_time(e1) / reps
        weak = {"op": "sum", "outputs": ["included", "excluded (total - included)"],
                "ms_per_op": round(wms, 4), "gelem_per_s": round(N / (wms * 1e-3) / 1e9, 3),
                "strong_ms_per_op": round(per_op["sum"], 4)}
        if not args.no_check:
            weak["check"] = spot_check(a_host, w, {"sum": (wi, we)}, np, ops=("sum",))

    # min, the third operator, for the record: same tensor, both outputs, not
    # part of the step
    mn = None
    if not args.no_weak:
        mi, me = torch.empty_like(a), torch.empty_like(a)
        P.run(a, w.box, "min", "both", inc_out=mi, exc_out=me, workspace=ws, stream=stream)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        reps = max(1, args.steps // 2)
        e0.record(stream)
        for _ in range(reps):
            P.run(a, w.box, "min", "both", inc_out=mi, exc_out=me, workspace=ws, stream=stream)
        e1.record(stream)
        torch.cuda.synchronize()
        mms = e0.elapsed_time(e1) / reps
        mn = {"outputs": ["included", "excluded"], "ms_per_op": round(mms, 4),
              "gelem_per_s": round(N / (mms * 1e-3) / 1e9, 3)}
        if not args.no_check:
            mn["check"] = spot_check(a_host, w, {"min": (mi, me)}, np, ops=("min",))
        del wi, we

    excl_elems_per_step = N * len(w.ops)
    value = excl_elems_per_step / (ms_per_step * 1e-3) / 1e9

    # dominant kernel roofline: algorithmic bytes (read the input once, write
    # both outputs once) over the kernel's average launch, timed by HIP events
    # on its launch stream in the instrumented pass; the committed rocprofv3
    # summary of the same kernel gives the traced average and the HBM bytes
    k0 = w.box[0]
    dom_name, (dom_launches, dom_total) = max(kt.items(), key=lambda kv: kv[1][1])
    dom_avg_s = dom_total / dom_launches * 1e-3
    abytes = algorithmic_bytes(dom_name, N, es, outputs=2) if dom_name.endswith("@L0") else None
    roofline = None
    if abytes is not None:
        achieved = abytes / dom_avg_s / 1e9
        kname = dom_name.split("@")[0]
        prof = profile_summary(kname, w.name)
        tr = prof if prof and "fetch" in prof else None
        roofline = {"bound": "hbm", "kernel": kname, "achieved": round(achieved, 1),
                    "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                    "traffic": (tr["fetch"] + tr["write"]) if tr else None,
                    "traffic_split": {"fetch": tr["fetch"], "write": tr["write"]} if tr else None,
                    "avg_launch_us": round(dom_avg_s * 1e6, 1),
                    "launches": dom_launches,
                    "algorithmic_bytes_per_launch": int(abytes),
                    "algorithmic_rule": "12 B/elem: read the input once, write the included "
                                        "and excluded sums once",
                    "overhead_read_bytes_per_launch": int(overhead_bytes(kname, N, es, k0)),
                    "profile": prof["file"] if prof else None,
                    "profile_avg_launch_us": prof["trace_avg_launch_us"] if prof else None,
                    "profile_frac": round(abytes / (prof["trace_avg_launch_us"] * 1e-6) / 1e9
                                          / HBM_PEAK_GBS, 4) if prof else None}
    # whole-path figure: read A twice, write both outputs, per op
    path_bytes = len(w.ops) * N * es * (2 + 2)
    path_gbs = path_bytes / (ms_per_step * 1e-3) / 1e9

    copy = None
    if not args.no_copy_probe:
        # plain device copies of the input: the achievable read+write ceiling
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(10):
            b.copy_(a)
        e1.record(stream)
        torch.cuda.synchronize()
        cms = e0.elapsed_time(e1) / 10
        cgbs = 2 * N * es / (cms * 1e-3) / 1e9
        copy = {"ms": round(cms, 4), "GBps": round(cgbs, 1),
                "frac_of_peak": round(cgbs / HBM_PEAK_GBS, 4),
                "what": "torch copy_ of the %d MiB input (read + write)" % (N * es >> 20)}
        del b

    # parity spot check of the timed outputs against the oracle (sampled)
    check = None
    if not args.no_check:
        check = spot_check(a_host, w, outs, np)

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(a_host, w, N)

    del outs, ws
    torch.cuda.empty_cache()
    configs = None if args.no_configs else bench_configs(args, P, torch, np)
    corners = None if args.no_corners else bench_corners(args, P, torch, np, (8192, 8192),
                                                         (16, 16), ("sum", "max"))
    batched = None if args.no_batched else bench_batched(args, P, _lib, torch, np)
    served = None if args.no_served else bench_served(args, P, _lib, torch, np)

    line = {
        "metric": "excluded-sum Gelem/s + % HBM peak (d=3, 512^3 fp32); batched/served p50/p99",
        "value": round(value, 3),
        "unit": "Gelem/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"f32": "f32", "f64": "f64", "i32": "i32", "i64": "i64"}[w.dtype],
        "data": "synthetic",
        "config": {"workload": w.name, "shape": list(w.shape), "box": list(w.box),
                   "ops": list(w.ops), "outputs": ["included", "excluded"],
                   "values": "N(0,1) numpy PCG64 seed %d" % w.seed},
        "per_op_ms": {k: round(v, 4) for k, v in per_op.items()},
        "instrumented_ms_per_step": round(inst_ms_per_step, 4),
        "path_GBps": round(path_gbs, 1),
        "path_frac_hbm": round(path_gbs / HBM_PEAK_GBS, 4),
        "roofline": roofline,
        "cpu_baseline": cpu,
        "copy_probe": copy,
        "check": check,
        "weak": weak,
        "min": mn,
        "configs": configs,
        "corners": corners,
        "batched": batched,
        "served": served,
    }
    print(json.dumps(line), flush=True)


def sweep_d(args, P, torch, np):
    """Scaling in the rank d (the paper's higher-dimension experiment): fp32
    tensors (device counter fill, unit variance) of N = n^d elements with
    n = round(N^(1/d)) for N about 2^21, 2^24 and 2^27 and d = 1..8, box side
    min(8, n) on every axis; included and excluded sums under + by the
    box-complement path (strong) and by total - included (weak).  Every
    configuration is checked at sampled cells against the oracle."""
    import oracle
    from tests import tolerance
    from paper_2106_00124_amd import workloads as W
    o = oracle.default()
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    rows = []
    for e2 in args.sweep_log2n:
        for d in range(1, 9):
            n = max(2, int(round(2 ** (e2 / d))))
            shape = (n,) * d
            box = tuple(min(8, v) for v in shape)
            N = n ** d
            seed = 100 * e2 + d
            x = torch.empty(shape, dtype=torch.float32, device=dev)
            P.fill(x, W.FILL_NORMALISH, seed)
            ws_b = max(P.workspace_size(shape, box, torch.float32, "sum", m)
                       for m in ("both", "both_weak"))
            ws = torch.empty(max(ws_b, 1), dtype=torch.uint8, device=dev)
            inc, exc = torch.empty_like(x), torch.empty_like(x)
            res = {"log2_target": e2, "d": d, "shape": list(shape), "box": list(box),
                   "elements": N}
            host = None
            pts = np.random.default_rng(seed).integers(0, N, 16)
            for mode in ("both", "both_weak"):
                for _ in range(2):
                    P.run(x, box, "sum", mode, inc_out=inc, exc_out=exc, workspace=ws,
                          stream=stream)
                torch.cuda.synchronize()
                e0 = torch.cuda.Event(enable_timing=True)
                e1 = torch.cuda.Event(enable_timing=True)
                reps = max(3, args.steps)
                e0.record(stream)
                for _ in range(reps):
                    P.run(x, box, "sum", mode, inc_out=inc, exc_out=exc, workspace=ws,
                          stream=stream)
                e1.record(stream)
                torch.cuda.synchronize()
                ms = e0.elapsed_time(e1) / reps
                key = "strong" if mode == "both" else "weak"
                res[key + "_ms"] = round(ms, 4)
                res[key + "_gelem_per_s"] = round(N / (ms * 1e-3) / 1e9, 2)
                res[key + "_ns_per_elem"] = round(ms * 1e6 / N, 5)
                if args.no_check:
                    continue
                # sampled cells against the oracle on the input regenerated
                # on the host
                if host is None:
                    host = W.counter_fill(W.FILL_NORMALISH, "f32", N, seed).reshape(shape)
                ip = torch.from_numpy(pts).to(dev)
                gi = inc.reshape(-1)[ip].cpu().numpy()
                ge = exc.reshape(-1)[ip].cpu().numpy()
                try:
                    tolerance.check(gi, o.point_inc(host, box, "sum", "f32", pts), "f32", "sum",
                                    tolerance.sigma_points(o, host, box, "inc", pts))
                    tolerance.check(ge, o.point_exc(host, box, "sum", "f32", pts), "f32", "sum",
                                    tolerance.sigma_points(o, host, box, "exc", pts))
                    res[key + "_check"] = "ok"
                except AssertionError as err:
                    res[key + "_check"] = str(err)[:120]
            log(f"N~2^{e2} d={d} n={n} strong {res['strong_ms']:.3f} ms "
                f"({res['strong_gelem_per_s']} Gelem/s) weak {res['weak_ms']:.3f} ms")
            rows.append(res)
            del x, inc, exc, ws, host
            torch.cuda.empty_cache()
    print(json.dumps({"metric": "excluded-sum Gelem/s vs rank d (fp32, N about 2^21, 2^24, "
                                "2^27, box side 8, +)", "unit": "Gelem/s", "n_gpus": 1,
                      "data": "synthetic", "sweep": rows}), flush=True)


def sweep_op_cost(args, P, torch, np):
    """Scaling with the cost of the operator (the paper's experiment with an
    artificially slowed operator, Sec. 6): included and excluded sums of a
    3-D fp32 tensor under + slowed by `cost` dependent integer steps per
    application (exs_set_op_cost), against the time of one application per
    element at the same parallelism (exs_op_probe).  The ratio tends to the
    number of operator applications per element as the cost grows.  Results
    are checked to be bit-identical to those of the plain operator."""
    from paper_2106_00124_amd import _lib
    from paper_2106_00124_amd import workloads as W
    L = _lib.lib()
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    sp = ctypes.c_void_p(stream.cuda_stream)
    shape, box = tuple(args.op_cost_shape), tuple(args.op_cost_box)
    x = torch.empty(shape, dtype=torch.float32, device=dev)
    P.fill(x, W.FILL_NORMALISH, 300)
    N = x.numel()
    ws = torch.empty(max(P.workspace_size(shape, box, torch.float32, "sum", "both"), 1),
                     dtype=torch.uint8, device=dev)
    probe = torch.empty_like(x)
    reps_probe = 16

    def timed(fn, reps):
        fn()
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            fn()
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    ref = {}
    rows = []
    try:
        for cost in args.op_costs:
            _lib.check(L.exs_set_op_cost(cost))
            res = {"cost_steps": cost}
            for mode in ("inc", "exc", "both"):
                inc = torch.empty_like(x)
                exc = torch.empty_like(x)
                reps = 5 if cost <= 256 else 2
                ms = timed(lambda: P.run(x, box, "sum", mode, inc_out=inc, exc_out=exc,
                                         workspace=ws, stream=stream), reps)
                outs = [t for t, m in ((inc, "inc"), (exc, "exc")) if m in mode or mode == "both"]
                if cost == args.op_costs[0]:
                    ref[mode] = [t.clone() for t in outs]
                else:
                    res[mode + "_identical"] = all(torch.equal(a, b)
                                                   for a, b in zip(outs, ref[mode]))
                res[mode + "_ms"] = round(ms, 4)
                res[mode + "_ns_per_elem"] = round(ms * 1e6 / N, 4)
            probe.copy_(x)
            pms = timed(lambda: _lib.check(L.exs_op_probe(ctypes.c_void_p(probe.data_ptr()), N,
                                                          reps_probe, sp)),
                        3 if cost <= 256 else 1)
            op_ns = pms * 1e6 / N / reps_probe
            res["op_ns_per_elem"] = round(op_ns, 5)
            for mode in ("inc", "exc", "both"):
                res[mode + "_ops_per_elem"] = round(res[mode + "_ns_per_elem"] / op_ns, 2)
            log(f"cost {cost}: both {res['both_ms']:.3f} ms, one op per element "
                f"{op_ns * 1e3:.3f} ps, ratio inc {res['inc_ops_per_elem']} exc "
                f"{res['exc_ops_per_elem']} both {res['both_ops_per_elem']}")
            rows.append(res)
    finally:
        L.exs_set_op_cost(0)
    print(json.dumps({"metric": "time per element / time per operator application vs "
                                "operator cost (3-D fp32, +)",
                      "shape": list(shape), "box": list(box), "n_gpus": 1, "data": "synthetic",
                      "probe_reps": reps_probe, "sweep": rows}), flush=True)


def sweep_n(args, P, torch, np):
    """Scaling in the size N at d = 3: fp32 (device counter fill) cubes n^3
    for n from 64 to 640, box 16^3, included and excluded sums under + (the
    paper reports a flat time per element in 3-D).  Each size is checked at
    sampled cells against the oracle."""
    import oracle
    from tests import tolerance
    from paper_2106_00124_amd import workloads as W
    o = oracle.default()
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    rows = []
    for n in (64, 128, 192, 256, 384, 512, 640):
        shape, box = (n, n, n), (16, 16, 16)
        N = n ** 3
        x = torch.empty(shape, dtype=torch.float32, device=dev)
        P.fill(x, W.FILL_NORMALISH, 200 + n)
        ws = torch.empty(max(P.workspace_size(shape, box, torch.float32, "sum", "both"), 1),
                         dtype=torch.uint8, device=dev)
        inc, exc = torch.empty_like(x), torch.empty_like(x)
        for _ in range(2):
            P.run(x, box, "sum", "both", inc_out=inc, exc_out=exc, workspace=ws, stream=stream)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        reps = max(3, args.steps)
        e0.record(stream)
        for _ in range(reps):
            P.run(x, box, "sum", "both", inc_out=inc, exc_out=exc, workspace=ws, stream=stream)
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        res = {"n": n, "elements": N, "ms": round(ms, 4),
               "ns_per_elem": round(ms * 1e6 / N, 4),
               "gelem_per_s": round(N / (ms * 1e-3) / 1e9, 2)}
        pts = np.random.default_rng(n).integers(0, N, 8)
        host = W.counter_fill(W.FILL_NORMALISH, "f32", N, 200 + n).reshape(shape)
        got = exc.reshape(-1)[torch.from_numpy(pts).to(dev)].cpu().numpy()
        ref = o.point_exc(host, box, "sum", "f32", pts)
        sig = tolerance.sigma_points(o, host, box, "exc", pts)
        try:
            tolerance.check(got, ref, "f32", "sum", sig)
            res["check"] = "ok"
        except AssertionError as err:
            res["check"] = str(err)[:120]
        log(f"n={n} {ms:.3f} ms {res['ns_per_elem']:.4f} ns/elem check {res['check']}")
        rows.append(res)
        del x, inc, exc, ws, host
        torch.cuda.empty_cache()
    print(json.dumps({"metric": "excluded-sum Gelem/s vs N (fp32 cubes, box 16^3, +)",
                      "unit": "Gelem/s", "n_gpus": 1, "data": "synthetic", "sweep": rows}),
          flush=True)


def bench_case(args, P, torch, np):
    """One plain call on an fp32 tensor of the given shape (device counter
    fill, unit variance), timed over --steps calls after --warmup, with the
    per-kernel breakdown from the library's event timing and a check of
    sampled cells against the oracle."""
    import oracle
    from tests import tolerance
    from paper_2106_00124_amd import _lib, workloads as W
    shape = tuple(int(v) for v in args.case.split(","))
    box = tuple(int(v) for v in args.box.split(",")) if args.box else (8,) * len(shape)
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    x = torch.empty(shape, dtype=torch.float32, device=dev)
    seed = 300 + len(shape)
    P.fill(x, W.FILL_NORMALISH, seed)
    ws = torch.empty(max(P.workspace_size(shape, box, torch.float32, args.op, args.mode), 1),
                     dtype=torch.uint8, device=dev)
    inc, exc = torch.empty_like(x), torch.empty_like(x)

    def call():
        P.run(x, box, args.op, args.mode, inc_out=inc, exc_out=exc, workspace=ws, stream=stream)

    for _ in range(max(1, args.warmup)):
        call()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(args.steps):
        call()
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / args.steps
    L = _lib.lib()
    L.exs_timing_enable(1)
    read_timings(L)
    for _ in range(args.steps):
        call()
    torch.cuda.synchronize()
    L.exs_timing_enable(0)
    kt = read_timings(L)
    N = x.numel()
    res = {"shape": list(shape), "box": list(box), "op": args.op, "mode": args.mode,
           "dtype": "f32", "ms": round(ms, 4), "gelem_per_s": round(N / (ms * 1e-3) / 1e9, 2),
           "kernels_us": {k: round(t / n * 1e3, 1) for k, (n, t) in kt.items()},
           "launches_per_call": {k: n // args.steps for k, (n, t) in kt.items()}}
    if not args.no_check and args.mode in ("exc", "both"):
        o = oracle.default()
        host = W.counter_fill(W.FILL_NORMALISH, "f32", N, seed).reshape(shape)
        pts = np.random.default_rng(seed).integers(0, N, 64)
        got = exc.reshape(-1)[torch.from_numpy(pts).to(dev)].cpu().numpy()
        ref = o.point_exc(host, box, args.op, "f32", pts)
        sig = tolerance.sigma_points(o, host, box, "exc", pts) if args.op == "sum" else None
        try:
            tolerance.check(got, ref, "f32", args.op, sig)
            res["check"] = "ok (64 sampled excluded cells)"
        except AssertionError as err:
            res["check"] = str(err)[:160]
    log(f"case {shape} {box} {args.op} {args.mode}: {ms:.4f} ms")
    print(json.dumps(res), flush=True)


def bench_configs(args, P, torch, np):
    """The other single-tensor workloads: 64x64 int64 (+, launch-bound:
    microseconds per call), 32^5 fp32 and 128x128x64x64 int32 (+ and max),
    both outputs; each timed per operator (median of the event-timed calls)
    and checked at sampled cells against the oracle."""
    from paper_2106_00124_amd.workloads import WORKLOADS
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    res = {}
    for name in ("d2_64x64_i64", "d5_32_f32", "d4_128x128x64x64_i32"):
        w = WORKLOADS[name]
        dt = {"f32": torch.float32, "i32": torch.int32, "i64": torch.int64}[w.dtype]
        a_host = w.tensor()
        a = torch.from_numpy(a_host).to(dev)
        es = a.element_size()
        ws = torch.empty(max(max(P.workspace_size(w.shape, w.box, dt, op, "both")
                                 for op in w.ops), 1), dtype=torch.uint8, device=dev)
        outs = {op: (torch.empty_like(a), torch.empty_like(a)) for op in w.ops}
        r = {"shape": list(w.shape), "box": list(w.box), "dtype": w.dtype,
             "outputs": ["included", "excluded"], "per_op": {}}
        for op in w.ops:
            inc, exc = outs[op]
            for _ in range(3):
                P.run(a, w.box, op, "both", inc_out=inc, exc_out=exc, workspace=ws, stream=stream)
            torch.cuda.synchronize()
            times = []
            for _ in range(max(20, args.steps)):
                e0 = torch.cuda.Event(enable_timing=True)
                e1 = torch.cuda.Event(enable_timing=True)
                e0.record(stream)
                P.run(a, w.box, op, "both", inc_out=inc, exc_out=exc, workspace=ws, stream=stream)
                e1.record(stream)
                times.append((e0, e1))
            torch.cuda.synchronize()
            ms = _pct([x.elapsed_time(y) for x, y in times], 0.5)
            gbs = w.n * es * 4 / (ms * 1e-3) / 1e9
            r["per_op"][op] = {"ms": round(ms, 4), "us": round(ms * 1e3, 1),
                               "gelem_per_s": round(w.n / (ms * 1e-3) / 1e9, 2),
                               "path_GBps": round(gbs, 1),
                               "path_frac_hbm": round(gbs / HBM_PEAK_GBS, 4)}
        if not args.no_check:
            r["check"] = spot_check(a_host, w, outs, np)
        r["path_bytes_rule"] = "16 B/elem per op for 4-byte types (read the input twice, " \
                               "write both outputs), 32 for 8-byte"
        log(f"config {name}: " + ", ".join(f"{op} {v['ms']:.4f} ms ({v['gelem_per_s']} Gelem/s)"
                                           for op, v in r["per_op"].items()))
        res[name] = r
        del a, ws, outs
        torch.cuda.empty_cache()
    return res


def bench_corners(args, P, torch, np, shape, box, ops):
    """Strong excluded sums of one 2-D fp32 tensor (N(0,1), seeded) by the
    box-complement path (excluded output only) and by the corners algorithm,
    the paper's comparison system: median event-timed call of each, the ratio,
    and how far the two results are apart (max: bit-identical cells; +: the
    largest difference over sqrt(sum A^2), the scale of the excluded sums)."""
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    rng = np.random.default_rng(int(np.prod(shape)) + 31 * box[0] + box[1])
    a_host = rng.standard_normal(shape).astype(np.float32)
    a = torch.from_numpy(a_host).to(dev)
    N = a.numel()
    ws_bc = torch.empty(max(max(P.workspace_size(shape, box, torch.float32, op, "exc")
                                for op in ops), 1), dtype=torch.uint8, device=dev)
    ws_co = torch.empty(max(P.corners_workspace_size(shape, box, torch.float32), 1),
                        dtype=torch.uint8, device=dev)
    e_bc, e_co = torch.empty_like(a), torch.empty_like(a)
    res = {"shape": list(shape), "box": list(box), "dtype": "f32", "output": "excluded",
           "values": "N(0,1) numpy PCG64", "per_op": {},
           "corners_workspace_bytes": ws_co.numel(), "box_complement_workspace_bytes":
           ws_bc.numel()}

    def timed(fn, reps):
        for _ in range(3):
            fn()
        torch.cuda.synchronize()
        ev = []
        for _ in range(reps):
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            fn()
            e1.record(stream)
            ev.append((e0, e1))
        torch.cuda.synchronize()
        return _pct([x.elapsed_time(y) for x, y in ev], 0.5)

    scale = float(np.sqrt((a_host.astype(np.float64) ** 2).sum()))
    for op in ops:
        ms_bc = timed(lambda: P.run(a, box, op, "exc", exc_out=e_bc, workspace=ws_bc,
                                    stream=stream), 20)
        ms_co = timed(lambda: P.run_corners(a, box, op, exc_out=e_co, workspace=ws_co,
                                            stream=stream), 20)
        g, b = e_co.cpu().numpy(), e_bc.cpu().numpy()
        if op == "sum":
            agree = {"max_abs_diff_over_scale": float(np.max(np.abs(g.astype(np.float64) - b))
                                                      / scale)}
        else:
            agree = {"identical_cells": int(np.count_nonzero(g == b)), "cells": int(g.size)}
        res["per_op"][op] = {"box_complement_ms": round(ms_bc, 4),
                             "corners_ms": round(ms_co, 4),
                             "box_complement_gelem_per_s": round(N / (ms_bc * 1e-3) / 1e9, 2),
                             "corners_gelem_per_s": round(N / (ms_co * 1e-3) / 1e9, 2),
                             "corners_over_box_complement": round(ms_co / ms_bc, 3),
                             "agreement": agree}
        log(f"corners {shape} {box} {op}: box-complement {ms_bc:.4f} ms, corners {ms_co:.4f} ms "
            f"({ms_co / ms_bc:.2f}x)")
    del a, ws_bc, ws_co, e_bc, e_co
    torch.cuda.empty_cache()
    return res


def _pct(v, p):
    import math
    v = sorted(v)
    if not v:
        return None
    i = max(0, min(len(v) - 1, math.ceil(p * len(v)) - 1))
    return v[i]


def bench_batched(args, P, _lib, torch, np):
    """Batched form: the 512-tensor mixed workload as one graph launch, vs
    the same jobs as individual plain calls (exs_run per tensor, one stream)."""
    from paper_2106_00124_amd import workloads as W
    items = W.batch_workload(count=args.batch_count)
    dev = torch.device("cuda:0")
    L = _lib.lib()
    stream = torch.cuda.current_stream()
    t0 = time.perf_counter()
    hosts = [it.tensor() for it in items]   # f32 N(0,1), i32 uniform [-100, 100]
    xs = [torch.from_numpy(h).to(dev) for h in hosts]
    torch.cuda.synchronize()
    log(f"batched: inputs generated and uploaded in {time.perf_counter() - t0:.1f}s")
    total = sum(it.n for it in items)
    log(f"batched: {len(items)} tensors, {total / 1e6:.1f} M elements")
    cache = os.environ.get("EXSUM_TUNE_CACHE",
                           os.path.join(os.path.expanduser("~"), ".cache", "exsum_tune.json"))
    t0 = time.perf_counter()
    B = P.Batch([(x, it.box, it.op, "both") for x, it in zip(xs, items)], tune_cache=cache)
    build_s = time.perf_counter() - t0

    def timed(fn, reps):
        evs = []
        for _ in range(reps):
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            fn()
            e1.record(stream)
            evs.append((e0, e1))
        torch.cuda.synchronize()
        return [a.elapsed_time(b) for a, b in evs]

    for _ in range(3):
        B.launch(stream)
    torch.cuda.synchronize()
    reps = max(args.steps, 5)
    g = timed(lambda: B.launch(stream), reps)
    info = B.info()
    e = timed(lambda: B.launch_eager(stream), reps)
    graph_out = [(i.clone(), x.clone()) for i, x in B.outputs]

    # per-tensor plain calls with prebuilt jobs and one shared workspace
    jobs, outs = [], []
    wsz = 0
    for x, it in zip(xs, items):
        inc, exc = torch.empty_like(x), torch.empty_like(x)
        j = P.job_for(x, it.box, it.op, "both", inc, exc)
        n = ctypes.c_size_t()
        _lib.check(L.exs_workspace_size(ctypes.byref(j), ctypes.byref(n)))
        wsz = max(wsz, n.value)
        jobs.append(j)
        outs.append((inc, exc))
    ws = torch.empty(max(wsz, 1), dtype=torch.uint8, device=dev)
    sp = ctypes.c_void_p(stream.cuda_stream)
    wp = ctypes.c_void_p(ws.data_ptr())

    def per_tensor():
        for j in jobs:
            rc = L.exs_run(ctypes.byref(j), wp, ws.numel(), sp)
            if rc:
                _lib.check(rc)

    per_tensor()
    torch.cuda.synchronize()
    pt = timed(per_tensor, max(3, reps // 2))
    # the graph launch's results against the oracle at sampled cells of every
    # tensor (bit-exact for i32 and max, the per-cell f32 rule for +), and
    # against the plain calls (bit-exact where the result is unique)
    check = None
    if not args.no_check:
        check = check_batched(items, hosts, graph_out, np, args.batch_check_points)
    exact = 0
    for (gi, ge), (pi, pe), it in zip(graph_out, outs, items):
        if it.dtype == "i32" or it.op != "sum":
            exact += int(torch.equal(gi, pi)) + int(torch.equal(ge, pe))
    n_exact = sum(2 for it in items if it.dtype == "i32" or it.op != "sum")
    ms_g = _pct(g, 0.5)
    res = {
        "jobs": len(items), "elements": int(total), "outputs": ["included", "excluded"],
        "graph_ms_p50": round(ms_g, 4), "graph_ms_p99": round(_pct(g, 0.99), 4),
        "eager_ms_p50": round(_pct(e, 0.5), 4),
        "per_tensor_ms_p50": round(_pct(pt, 0.5), 4),
        "gelem_per_s": round(total / (ms_g * 1e-3) / 1e9, 2),
        "GBps_at_16B_per_elem": round(total * 16 / (ms_g * 1e-3) / 1e9, 1),
        "per_tensor_gelem_per_s": round(total / (_pct(pt, 0.5) * 1e-3) / 1e9, 2),
        "speedup_vs_per_tensor": round(_pct(pt, 0.5) / ms_g, 3),
        "graph_nodes": info["graph_nodes"], "work_items": info["work_items"],
        "build_s": round(build_s, 2),
        "check": check,
        "plain_call_bit_exact": f"{exact}/{n_exact} (integer and max outputs)",
        "values": "host numpy PCG64: f32 N(0,1), i32 uniform [-100,100], one seed per tensor",
    }
    log(f"batched: graph {ms_g:.3f} ms, eager {res['eager_ms_p50']:.3f} ms, "
        f"per-tensor {res['per_tensor_ms_p50']:.3f} ms")
    B.close()
    return res


def bench_served(args, P, _lib, torch, np):
    """Serving form: the Poisson request stream (excluded sums, inputs
    generated on the device) through the server, vs the serial plain path (one
    request at a time on one stream) on the first seconds of the same
    arrivals.  A sample of the served results (the largest requests, the
    longest boxes, and uniform draws) is checked at sampled cells against the
    oracle on the inputs regenerated on the host."""
    from paper_2106_00124_amd import workloads as W
    reqs = W.serving_workload(duration_s=args.serve_seconds)
    elems = sum(r.n for r in reqs)
    log(f"served: {len(reqs)} requests in {args.serve_seconds:.1f}s, "
        f"{elems / 1e9:.2f} G elements")
    S = P.Server(hbm_budget=int(args.serve_budget_gib * (1 << 30)),
                 max_inflight=args.serve_inflight)
    # warm the kernels of both operators and the generic/fused paths
    for r in reqs[:16]:
        S.submit_generated(r.shape, r.box, torch.float32, r.op, "exc", kind=W.FILL_LOGMAG,
                           seed=r.fill_seed)
    S.drain()
    S.close()

    # requests whose results are checked: the largest, the longest boxes, and
    # uniform draws from the rest
    rng = np.random.default_rng(606)
    want = sorted(range(len(reqs)), key=lambda i: -reqs[i].n)[:4]
    want += sorted(range(len(reqs)), key=lambda i: -max(reqs[i].box))[:4]
    want += [int(i) for i in rng.choice(len(reqs), size=max(0, args.serve_check - 8),
                                        replace=False)]
    want = set(want) if args.serve_check > 0 and not args.no_check else set()
    sampled = {}

    def open_loop(S):
        from collections import deque
        pend = deque()
        late = []
        t0 = time.perf_counter()

        def retire_head():
            t, i = pend.popleft()
            if i in want:
                r = reqs[i]
                _, exc, _ = S.result(t)
                pts = np.concatenate([rng.integers(0, r.n, 30), [0, r.n - 1]]).astype(np.int64)
                sampled[i] = (pts, exc.reshape(-1)[torch.from_numpy(pts).to(exc.device)]
                              .cpu().numpy())
            S.release(t)

        for i, r in enumerate(reqs):
            while True:
                now = time.perf_counter() - t0
                while pend and S.done(pend[0][0]):
                    retire_head()
                if now >= r.arrival_s:
                    break
                if r.arrival_s - now > 3e-4:
                    time.sleep(1e-4)
            late.append(time.perf_counter() - t0 - r.arrival_s)
            pend.append((S.submit_generated(r.shape, r.box, torch.float32, r.op, "exc",
                                            kind=W.FILL_LOGMAG, seed=r.fill_seed), i))
        while pend:
            if S.done(pend[0][0]):
                retire_head()
        wall = time.perf_counter() - t0
        return late, wall

    S = P.Server(hbm_budget=int(args.serve_budget_gib * (1 << 30)),
                 max_inflight=args.serve_inflight)
    late, wall = open_loop(S)
    st = S.stats()
    S.close()
    log(f"served: p50 {st['p50_ms']:.3f} ms p99 {st['p99_ms']:.3f} ms, {st['req_per_s']:.0f} req/s "
        f"over {wall:.1f}s")

    # saturated: every request submitted at once (throughput)
    S = P.Server(hbm_budget=int(args.serve_budget_gib * (1 << 30)),
                 max_inflight=args.serve_inflight)
    from collections import deque
    pend = deque()
    t0 = time.perf_counter()
    for r in reqs:
        pend.append(S.submit_generated(r.shape, r.box, torch.float32, r.op, "exc",
                                       kind=W.FILL_LOGMAG, seed=r.fill_seed))
        while pend and S.done(pend[0]):
            S.release(pend.popleft())
    while pend:
        if S.done(pend[0]):
            S.release(pend.popleft())
    sat_s = time.perf_counter() - t0
    S.close()
    log(f"served saturated: {len(reqs) / sat_s:.0f} req/s")

    # serial plain path on one stream, the first seconds of the same arrivals
    sreqs = [r for r in reqs if r.arrival_s < args.serial_seconds]
    selems = sum(r.n for r in sreqs)
    L = _lib.lib()
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    maxn = max(r.n for r in sreqs)
    wsz = 0
    for r in sreqs:
        wsz = max(wsz, P.workspace_size(r.shape, r.box, torch.float32, r.op, "exc"))
    xin = torch.empty(maxn, dtype=torch.float32, device=dev)
    xout = torch.empty(maxn, dtype=torch.float32, device=dev)
    ws = torch.empty(max(wsz, 1), dtype=torch.uint8, device=dev)
    sp = ctypes.c_void_p(stream.cuda_stream)

    def serial_one(r):
        _lib.check(L.exs_fill(ctypes.c_void_p(xin.data_ptr()), r.n, _lib.F32, W.FILL_LOGMAG,
                              ctypes.c_uint64(r.fill_seed), -100, 100, sp))
        j = _lib.make_job(len(r.shape), _lib.F32, _lib.SUM if r.op == "sum" else _lib.MAX,
                          _lib.EXCLUDED, list(r.shape), list(r.box), xin.data_ptr(), None,
                          xout.data_ptr())
        _lib.check(L.exs_run(ctypes.byref(j), ctypes.c_void_p(ws.data_ptr()), ws.numel(), sp))

    lat = []
    t0 = time.perf_counter()
    for r in sreqs:
        while time.perf_counter() - t0 < r.arrival_s:
            pass
        serial_one(r)
        stream.synchronize()
        lat.append((time.perf_counter() - t0 - r.arrival_s) * 1e3)
    t1 = time.perf_counter()
    for r in sreqs:
        serial_one(r)
    stream.synchronize()
    serial_sat = time.perf_counter() - t1
    del xin, xout, ws
    check = check_served(reqs, sampled, np) if sampled else None
    res = {
        "requests": len(reqs), "window_s": args.serve_seconds, "rate_per_s": 2000,
        "wall_s": round(wall, 2),
        "elements": int(elems), "outputs": ["excluded"], "hbm_budget_gib": args.serve_budget_gib,
        "max_inflight": args.serve_inflight,
        "p50_ms": round(st["p50_ms"], 4), "p99_ms": round(st["p99_ms"], 4),
        "completed": st["completed"],
        "req_per_s": round(st["req_per_s"], 1), "gelem_per_s": round(st["gelem_per_s"], 3),
        "max_queue": st["max_queue"], "peak_bytes": st["peak_bytes"],
        "submit_lateness_p99_ms": round(_pct(late, 0.99) * 1e3, 4),
        "saturated_req_per_s": round(len(reqs) / sat_s, 1),
        "saturated_gelem_per_s": round(elems / sat_s / 1e9, 3),
        "serial_window_s": args.serial_seconds, "serial_requests": len(sreqs),
        "serial_p50_ms": round(_pct(lat, 0.5), 4), "serial_p99_ms": round(_pct(lat, 0.99), 4),
        "serial_saturated_req_per_s": round(len(sreqs) / serial_sat, 1),
        "serial_saturated_gelem_per_s": round(selems / serial_sat / 1e9, 3),
        "latency": "submit to completion seen by the server (serial: arrival to stream sync)",
        "check": check,
    }
    log(f"serial: p50 {res['serial_p50_ms']:.3f} ms p99 {res['serial_p99_ms']:.3f} ms; "
        f"saturated {res['saturated_req_per_s']:.0f} vs {res['serial_saturated_req_per_s']:.0f} req/s")
    return res


def check_served(reqs, sampled, np):
    """Sampled cells of the checked served requests against the oracle on the
    inputs regenerated on the host from each request's seed."""
    import concurrent.futures as cf
    import oracle
    from paper_2106_00124_amd import workloads as W
    from tests import tolerance
    o = oracle.default()
    t0 = time.perf_counter()

    def one(i):
        r = reqs[i]
        pts, got = sampled[i]
        host = W.counter_fill(W.FILL_LOGMAG, "f32", r.n, r.fill_seed).reshape(r.shape)
        ref = o.point_exc(host, r.box, r.op, "f32", pts)
        sig = tolerance.sigma_points(o, host, r.box, "exc", pts) if r.op == "sum" else None
        try:
            st = tolerance.check(got, ref, "f32", r.op, sig, what=f"request {r.rid}")
            return None, st.get("max_scaled_err", 0.0)
        except AssertionError as e:
            return str(e)[:160], 0.0

    with cf.ThreadPoolExecutor(8) as ex:
        out = list(ex.map(one, sorted(sampled)))
    bad = [e for e, _ in out if e]
    return {"ok": not bad, "requests": len(sampled),
            "largest_elements": max(reqs[i].n for i in sampled),
            "longest_box_side": max(max(reqs[i].box) for i in sampled),
            "cells_per_request": len(next(iter(sampled.values()))[0]),
            "f32_sum_max_scaled_err": max(v for _, v in out), "failures": bad[:5],
            "host_s": round(time.perf_counter() - t0, 1)}


def check_batched(items, hosts, outs, np, npts):
    """Every tensor of the batch at `npts` sampled cells (and its first and
    last cell) against the oracle."""
    import oracle
    from tests import tolerance
    o = oracle.default()
    rng = np.random.default_rng(515)
    t0 = time.perf_counter()
    worst = 0.0
    bad = []
    cells = 0
    for t, (it, a, (inc, exc)) in enumerate(zip(items, hosts, outs)):
        pts = np.concatenate([rng.integers(0, it.n, npts), [0, it.n - 1]]).astype(np.int64)
        idx = __import__("torch").from_numpy(pts).to(inc.device)
        gi = inc.reshape(-1)[idx].cpu().numpy()
        ge = exc.reshape(-1)[idx].cpu().numpy()
        ri = o.point_inc(a, it.box, it.op, it.dtype, pts)
        re_ = o.point_exc(a, it.box, it.op, it.dtype, pts)
        si = se = None
        if it.dtype == "f32" and it.op == "sum":
            si = tolerance.sigma_points(o, a, it.box, "inc", pts)
            se = tolerance.sigma_points(o, a, it.box, "exc", pts)
        try:
            s1 = tolerance.check(gi, ri, it.dtype, it.op, si, what=f"tensor {t} inc")
            s2 = tolerance.check(ge, re_, it.dtype, it.op, se, what=f"tensor {t} exc")
            worst = max(worst, s1.get("max_scaled_err", 0.0), s2.get("max_scaled_err", 0.0))
        except AssertionError as e:
            bad.append(str(e)[:160])
        cells += 2 * len(pts)
    return {"ok": not bad, "tensors": len(items), "cells_per_tensor": npts + 2,
            "cells_checked": cells, "f32_sum_max_scaled_err": worst, "failures": bad[:5],
            "rule": "bit-exact for i32 and max; f32 + |got-ref| <= 1e-5 max(|ref|, sigma)",
            "host_s": round(time.perf_counter() - t0, 1)}


def spot_check(a_host, w, outs, np, ops=None):
    import oracle
    from tests import tolerance
    o = oracle.default()
    rng = np.random.default_rng(123)
    pts = rng.integers(0, w.n, size=2000)
    pts = np.concatenate([pts, [0, w.n - 1]])
    res = {}
    for op in (ops or w.ops):
        inc, exc = (t.reshape(-1)[pts].cpu().numpy() for t in outs[op])
        ri = o.point_inc(a_host, w.box, op, w.dtype, pts)
        re_ = o.point_exc(a_host, w.box, op, w.dtype, pts)
        si = se = None
        if op == "sum" and w.dtype in ("f32", "f64"):
            si = tolerance.sigma_points(o, a_host, w.box, "inc", pts)
            se = tolerance.sigma_points(o, a_host, w.box, "exc", pts)
        try:
            s1 = tolerance.check(inc, ri, w.dtype, op, si, what=f"{op} inc")
            s2 = tolerance.check(exc, re_, w.dtype, op, se, what=f"{op} exc")
            res[op] = {"ok": True, "inc": s1, "exc": s2}
        except AssertionError as e:
            res[op] = {"ok": False, "error": str(e)[:200]}
    return {"points": int(len(pts)), **res}


def cpu_baseline(a_host, w, N):
    """The oracle (plain C, OpenMP, FP64) on the full step: included and
    excluded sums for every op of the workload; the median of three runs."""
    import oracle
    o = oracle.default()
    times = []
    for _ in range(3):
        t0 = time.perf_counter()
        for op in w.ops:
            o.scale(a_host, w.box, op, w.dtype)
        times.append(time.perf_counter() - t0)
    dt = sorted(times)[1]
    return {"value": round(N * len(w.ops) / dt / 1e9, 4), "unit": "Gelem/s",
            "cores": o.num_threads(), "kind": "oracle", "seconds": round(dt, 2), "runs": 3,
            "sample": "full step: included+excluded sums, ops %s, on the whole %s tensor "
                      "(median of 3 runs)" % ("+".join(w.ops), "x".join(map(str, w.shape))),
            "cpu": cpu_model(), "host_logical_cpus": os.cpu_count()}


if __name__ == "__main__":
    main()
