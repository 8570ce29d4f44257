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
    p.add_argument("--copy-probe", action="store_true",
                   help="also time a plain device copy of the input (bandwidth ceiling)")
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


def algorithmic_bytes(kernel, N, es, k0, outputs):
    """Bytes a launch of `kernel` must move at level 0 (per launch): read the
    input once, write each output once, plus the per-block suffix table."""
    base = kernel.split("@")[0]
    if base in ("k_axis0", "k_plane_axis0"):
        return N * es * (1 + outputs) + (N // k0) * es
    if base in ("k_bdbs", "k_plane_bdbs"):
        return 2 * N * es
    if base == "k_blockagg":
        return N * es + (N // k0) * es
    return None


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

    # timed region: per-kernel HIP events recorded on the launch stream
    L.exs_timing_enable(1)
    read_timings(L)
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
    L.exs_timing_enable(0)
    kt = read_timings(L)
    gpu_ms = ev0.elapsed_time(ev1)
    ms_per_step = gpu_ms / args.steps
    log(f"timed {args.steps} steps: {ms_per_step:.3f} ms/step (wall {1e3 * t_wall / args.steps:.3f})")
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

    excl_elems_per_step = N * len(w.ops)
    value = excl_elems_per_step / (ms_per_step * 1e-3) / 1e9

    # dominant kernel roofline
    k0 = w.box[0]
    dom_name, (dom_launches, dom_total) = max(kt.items(), key=lambda kv: kv[1][1])
    dom_avg_s = dom_total / dom_launches * 1e-3
    abytes = algorithmic_bytes(dom_name, N, es, k0, outputs=2) if dom_name.endswith("@L0") else None
    roofline = None
    if abytes is not None:
        achieved = abytes / dom_avg_s / 1e9
        roofline = {"bound": "hbm", "kernel": dom_name.split("@")[0], "achieved": round(achieved, 1),
                    "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                    "traffic": None, "avg_launch_us": round(dom_avg_s * 1e6, 1),
                    "algorithmic_bytes_per_launch": int(abytes)}
    # whole-path figure: read A twice, write both outputs, per op
    path_bytes = len(w.ops) * N * es * (2 + 2)
    path_gbs = path_bytes / (ms_per_step * 1e-3) / 1e9

    copy = None
    if args.copy_probe:
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
        copy = {"ms": round(cms, 4), "GBps": round(2 * N * es / (cms * 1e-3) / 1e9, 1)}
        del b

    # parity spot check of the timed outputs against the oracle (sampled)
    check = None
    if not args.no_check:
        check = spot_check(a_host, w, outs, np)

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(a_host, w, N)

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
        "path_GBps": round(path_gbs, 1),
        "path_frac_hbm": round(path_gbs / HBM_PEAK_GBS, 4),
        "roofline": roofline,
        "cpu_baseline": cpu,
        "copy_probe": copy,
        "check": check,
    }
    print(json.dumps(line), flush=True)


def spot_check(a_host, w, outs, np):
    import oracle
    from tests import tolerance
    o = oracle.default()
    rng = np.random.default_rng(123)
    pts = rng.integers(0, w.n, size=2000)
    pts = np.concatenate([pts, [0, w.n - 1]])
    res = {}
    for op in w.ops:
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
    excluded sums for every op of the workload."""
    import oracle
    o = oracle.default()
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    t0 = time.perf_counter()
    for op in w.ops:
        o.scale(a_host, w.box, op, w.dtype)
    dt = time.perf_counter() - t0
    return {"value": round(N * len(w.ops) / dt / 1e9, 4), "unit": "Gelem/s", "cores": cores,
            "kind": "oracle", "seconds": round(dt, 2),
            "sample": "full step: included+excluded sums, ops %s, on the whole %s tensor"
                      % ("+".join(w.ops), "x".join(map(str, w.shape))),
            "cpu": platform.processor() or platform.machine()}


if __name__ == "__main__":
    main()
