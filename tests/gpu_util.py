"""Helpers for the GPU parity tests: run the HIP path, get the oracle's answer."""
from __future__ import annotations

import sys
import zlib

import numpy as np

from tests import tolerance

NP = {"f32": np.float32, "f64": np.float64, "i32": np.int32, "i64": np.int64}


def torch_dtype(dt):
    import torch
    return {"f32": torch.float32, "f64": torch.float64, "i32": torch.int32,
            "i64": torch.int64}[dt]


def make_input(shape, dtype, seed, op):
    rng = np.random.default_rng(seed)
    if dtype in ("f32", "f64"):
        if op in ("max", "min"):
            # distinct nonzero values: no ties between +0 and -0
            n = int(np.prod(shape))
            v = (rng.permutation(n) + 1.0) * rng.choice([-1.0, 1.0], n) / n
            return v.astype(NP[dtype]).reshape(shape)
        return rng.standard_normal(shape).astype(NP[dtype])
    if dtype == "i32":
        return rng.integers(-2**31, 2**31, size=shape, dtype=np.int64).astype(np.int32)
    return rng.integers(-2**62, 2**62, size=shape, dtype=np.int64)


def gpu_run(a, box, op, mode="both"):
    import torch
    import paper_2106_00124_amd as P
    t = torch.from_numpy(np.ascontiguousarray(a)).cuda()
    inc, exc = P.run(t, box, op, mode)
    torch.cuda.synchronize()
    return (inc.cpu().numpy() if inc is not None else None,
            exc.cpu().numpy() if exc is not None else None)


def oracle_full(orc, a, box, op, dtype):
    if a.size <= 4096:
        return orc.brute(a, box, op, dtype)
    return orc.scale(a, box, op, dtype)


def compare_full(orc, a, box, op, dtype, inc, exc, what=""):
    ri, re_ = oracle_full(orc, a, box, op, dtype)
    si = se = None
    if dtype in ("f32", "f64") and op == "sum":
        si = tolerance.sigma_full(orc, a, box, "inc")
        se = tolerance.sigma_full(orc, a, box, "exc")
    stats = {}
    if inc is not None:
        stats["inc"] = tolerance.check(inc, ri, dtype, op, si, what=f"{what} inc")
    if exc is not None:
        stats["exc"] = tolerance.check(exc, re_, dtype, op, se, what=f"{what} exc")
    return stats


def seed_of(*params) -> int:
    """A seed derived from the test parameters that is the same in every
    process (Python's str hash is salted per process)."""
    return zlib.crc32(repr(params).encode())


def say(*args):
    print(*args, flush=True)
    sys.stdout.flush()
