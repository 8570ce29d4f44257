"""Seeded synthetic workloads (inputs only; none of the method's arithmetic).

This module is shared by the tests, the benchmark and the serving driver.  It
draws input tensors, box sizes and request streams; it never computes an
included or excluded sum.  Two kinds of generators live here:

* numpy ``Generator(PCG64(seed))`` draws for host-side inputs;
* a host twin of the counter-based generator that the library's device fill
  kernel implements (``exs_fill``): the i-th output of a SplitMix64 stream
  (Steele, Lea and Flood, OOPSLA 2014) started at ``seed`` is
  ``mix(seed + (i + 1) * 0x9E3779B97F4A7C15)``, with the published mixing
  function below.  Values are built from the 64-bit output with integer
  operations and one float32 multiply (or bit assembly), so the host and the
  device produce bit-identical tensors.

The paper measures on no public dataset; these shapes and value
distributions stand in for its synthetic workloads.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

GOLDEN = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)

# counter-based value kinds (must match the device fill kernel)
FILL_NORMALISH = 0    # f32: (sum of four 16-bit uniforms - 2*65535) * c, var ~= 1
FILL_UNIFORM_INT = 1  # i32/i64: lo + (h mod (hi - lo + 1))
FILL_LOGMAG = 2       # f32: random sign * 2^e * (1 + m / 2^23), e uniform in [-10, 9]

# c = sqrt(3) / 65535 rounded to float32: the sum of four U[0,1) has variance 1/3
NORMALISH_SCALE = np.float32(math.sqrt(3.0) / 65535.0)


def splitmix64(seed: int, count: int, start: int = 0) -> np.ndarray:
    """Outputs ``start .. start+count-1`` of the SplitMix64 stream at ``seed``."""
    with np.errstate(over="ignore"):
        i = np.arange(start + 1, start + count + 1, dtype=np.uint64)
        z = np.uint64(seed & 0xFFFFFFFFFFFFFFFF) + i * GOLDEN
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        z = z ^ (z >> np.uint64(31))
    return z


def counter_fill(kind: int, dtype: str, count: int, seed: int,
                 lo: int = -100, hi: int = 100) -> np.ndarray:
    """Host twin of the device fill kernel (bit-identical by construction)."""
    h = splitmix64(seed, count)
    if kind == FILL_NORMALISH:
        m = np.uint64(0xFFFF)
        s = ((h & m).astype(np.int64) + ((h >> np.uint64(16)) & m).astype(np.int64)
             + ((h >> np.uint64(32)) & m).astype(np.int64)
             + ((h >> np.uint64(48)) & m).astype(np.int64) - 2 * 65535)
        return (s.astype(np.float32) * NORMALISH_SCALE).astype(np.float32)
    if kind == FILL_UNIFORM_INT:
        span = np.uint64(hi - lo + 1)
        v = (h % span).astype(np.int64) + lo
        return v.astype(np.int32 if dtype == "i32" else np.int64)
    if kind == FILL_LOGMAG:
        sign = (h >> np.uint64(63)).astype(np.uint32)
        e = ((h >> np.uint64(32)) % np.uint64(20)).astype(np.int64) - 10
        mant = (h & np.uint64(0x7FFFFF)).astype(np.uint32)
        bits = (sign << np.uint32(31)) | ((e + 127).astype(np.uint32) << np.uint32(23)) | mant
        return bits.view(np.float32)
    raise ValueError(kind)


NP_DTYPE = {"f32": np.float32, "f64": np.float64, "i32": np.int32, "i64": np.int64}


def gen_tensor(shape, dtype: str, seed: int, dist: str = "normal",
               lo: int = -100, hi: int = 100) -> np.ndarray:
    """Host-side tensor: N(0,1) floats or uniform integers in [lo, hi]."""
    rng = np.random.Generator(np.random.PCG64(seed))
    shape = tuple(int(s) for s in shape)
    if dtype in ("f32", "f64"):
        if dist == "normal":
            return rng.standard_normal(shape, dtype=NP_DTYPE[dtype])
        if dist == "uniform":
            return rng.uniform(lo, hi, shape).astype(NP_DTYPE[dtype])
        if dist == "distinct":
            # distinct nonzero values (no ties, no signed zeros) for max tests
            n = int(np.prod(shape))
            v = (rng.permutation(n).astype(np.float64) + 1.0) * rng.choice([-1.0, 1.0], n)
            return (v / n).astype(NP_DTYPE[dtype]).reshape(shape)
        raise ValueError(dist)
    return rng.integers(lo, hi, size=shape, endpoint=True, dtype=NP_DTYPE[dtype])


# --------------------------------------------------------------------------
# The single-tensor workloads (shapes, boxes, value distributions, seeds)
# --------------------------------------------------------------------------

@dataclass(frozen=True)
class Workload:
    name: str
    shape: tuple
    box: tuple
    dtype: str
    ops: tuple
    dist: str
    lo: int = -100
    hi: int = 100
    seed: int = 0

    @property
    def n(self) -> int:
        return int(np.prod(self.shape))

    def tensor(self) -> np.ndarray:
        return gen_tensor(self.shape, self.dtype, self.seed, self.dist, self.lo, self.hi)


WORKLOADS = {
    # d=2, 64x64 int64 in [-100, 100], box (8, 8), +
    "d2_64x64_i64": Workload("d2_64x64_i64", (64, 64), (8, 8), "i64", ("sum",), "int",
                             -100, 100, seed=1),
    # d=3, 512^3 fp32 N(0,1), box (16, 16, 16), + and max
    "d3_512_f32": Workload("d3_512_f32", (512, 512, 512), (16, 16, 16), "f32",
                           ("sum", "max"), "normal", seed=2),
    # d=5, 32^5 fp32 N(0,1), box 4^5, + and max
    "d5_32_f32": Workload("d5_32_f32", (32,) * 5, (4,) * 5, "f32", ("sum", "max"),
                          "normal", seed=3),
    # d=4, 128x128x64x64 int32 in [-1000, 1000], box (8, 8, 4, 4), + and max
    "d4_128x128x64x64_i32": Workload("d4_128x128x64x64_i32", (128, 128, 64, 64),
                                     (8, 8, 4, 4), "i32", ("sum", "max"), "int",
                                     -1000, 1000, seed=4),
}


# --------------------------------------------------------------------------
# Batched workload: many tensors of uneven ranks, shapes, boxes, dtypes, ops
# --------------------------------------------------------------------------

@dataclass
class BatchItem:
    shape: tuple
    box: tuple
    dtype: str
    op: str
    seed: int

    @property
    def n(self) -> int:
        return int(np.prod(self.shape))

    def tensor(self) -> np.ndarray:
        if self.dtype == "f32":
            return gen_tensor(self.shape, "f32", self.seed, "normal")
        return gen_tensor(self.shape, self.dtype, self.seed, "int", -100, 100)


def batch_workload(count: int = 512, seed: int = 5, max_elems: int = 1 << 22,
                   dim_lo: int = 16, dim_hi: int = 256, box_hi: int = 32,
                   ranks=(2, 3, 4)) -> list:
    """Rank uniform over ``ranks``; each dim log-uniform in [dim_lo, dim_hi];
    shapes above ``max_elems`` have their dims redrawn (the rank stays); box side per dim uniform in
    [2, min(box_hi, n_i)]; f32 N(0,1) or i32 uniform [-100, 100] (50/50);
    op + or max (50/50, independent of dtype)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    items = []
    for t in range(count):
        d = int(rng.choice(ranks))
        while True:
            dims = tuple(int(round(math.exp(rng.uniform(math.log(dim_lo), math.log(dim_hi)))))
                         for _ in range(d))
            if int(np.prod(dims)) <= max_elems:
                break
        box = tuple(int(rng.integers(2, min(box_hi, n) + 1)) if n >= 2 else 1 for n in dims)
        dtype = "f32" if rng.random() < 0.5 else "i32"
        op = "sum" if rng.random() < 0.5 else "max"
        items.append(BatchItem(dims, box, dtype, op, seed=int(seed * 1_000_003 + t)))
    return items


# --------------------------------------------------------------------------
# Serving workload: a Poisson stream of excluded-sum requests
# --------------------------------------------------------------------------

@dataclass
class Request:
    rid: int
    arrival_s: float
    shape: tuple
    box: tuple
    op: str
    fill_seed: int

    @property
    def n(self) -> int:
        return int(np.prod(self.shape))


def serving_workload(rate_per_s: float = 2000.0, duration_s: float = 60.0, seed: int = 6,
                     max_elems: int = 1 << 26, dim_lo: int = 32, dim_hi: int = 1024,
                     box_hi: int = 64, ranks=(2, 3), sum_frac: float = 0.8) -> list:
    """Poisson arrivals; rank uniform over ``ranks``; dims log-uniform in
    [dim_lo, dim_hi] with dims redrawn (rank kept) while above ``max_elems``; box side uniform
    in [2, min(box_hi, n_i)]; op + with probability ``sum_frac`` else max.
    Values are f32 with log-uniform magnitudes in [2^-10, 2^10) and random
    sign, produced on the device by the counter-based fill (FILL_LOGMAG)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    t = 0.0
    reqs = []
    rid = 0
    while True:
        t += rng.exponential(1.0 / rate_per_s)
        if t >= duration_s:
            break
        d = int(rng.choice(ranks))
        while True:
            dims = tuple(int(round(math.exp(rng.uniform(math.log(dim_lo), math.log(dim_hi)))))
                         for _ in range(d))
            if int(np.prod(dims)) <= max_elems:
                break
        box = tuple(int(rng.integers(2, min(box_hi, n) + 1)) for n in dims)
        op = "sum" if rng.random() < sum_frac else "max"
        reqs.append(Request(rid, t, dims, box, op, fill_seed=int(seed * 7_919 + rid * 2 + 1)))
        rid += 1
    return reqs
