"""HIP path vs the CPU oracle, element by element, on small seeded inputs.

Shapes span several tiles/blocks and ragged tails (n mod k != 0), k = 1, k = n,
boxes longer than 64 (the two-sweep kernels), ranks 1..8, every dtype x op.
"""
import numpy as np
import pytest

from tests import tolerance
from tests.gpu_util import compare_full, gpu_run, make_input, say, seed_of

pytestmark = pytest.mark.gpu

CASES = [
    ((1,), (1,)),
    ((37,), (5,)),
    ((300,), (300,)),
    ((1000,), (64,)),
    ((777,), (100,)),            # k > 64: two-sweep kernels
    ((64, 64), (8, 8)),
    ((13, 70), (4, 9)),
    ((70, 13), (13, 1)),
    ((5, 300), (5, 65)),
    ((9, 10, 11), (2, 3, 4)),
    ((33, 17, 65), (16, 16, 16)),
    ((4, 5, 6, 7), (4, 1, 3, 7)),
    ((6, 5, 4, 3, 2), (3, 2, 4, 1, 2)),
    ((3, 2, 3, 2, 3, 2), (2, 2, 1, 2, 3, 1)),
    ((2, 2, 2, 2, 2, 2, 2, 3), (1, 2, 2, 1, 2, 2, 1, 2)),
    # 2-D tensors through the fused row stream: ragged rows and blocks, runs
    ((1000, 777), (7, 13)),
    ((200, 4096), (16, 16)),
    ((33, 300), (16, 3)),
    ((517, 64), (2, 1)),
    # contiguous-axis box sums by wavefront segmented scans: boxes of 17 to 64
    # on rows shorter and longer than one 64-column window, blocks straddling
    # the windows, ragged last blocks, several row groups per task
    ((300, 130), (3, 64)),
    ((100, 127), (5, 63)),
    ((70, 65), (3, 33)),
    ((50, 200), (2, 17)),
    ((9, 1000), (2, 64)),
    ((40, 30, 45), (2, 3, 45)),
    ((700, 24), (3, 24)),
    # many blocks along an axis with few points (segmented block scans)
    ((300000,), (3,)),
    ((50000, 3), (2, 2)),
    # a last level longer than the one-workgroup kernel takes (4-byte types
    # with k <= 16: in chunks with a one-workgroup scan of the chunk totals;
    # k = 16 and k = 15 give the shortest and longest chunks, k = 1 a chunk
    # per 4096 elements, ragged chunks and blocks throughout)
    ((3, 9000), (2, 5)),
    ((2, 3, 8193), (1, 2, 100)),
    ((100003,), (7,)),
    ((50000,), (16,)),
    ((61441,), (15,)),
    ((20000,), (1,)),
    ((5,), (5,)),
    ((2, 40000), (2, 16)),
    ((3, 3, 20000), (2, 2, 11)),
    # trailing axes box-summed in one LDS-staged pass: all of them (3024
    # elements), or the last two with the third by a separate pass
    ((5, 6, 7, 8, 9), (2, 3, 2, 3, 4)),
    ((40, 30, 20, 10), (3, 4, 5, 6)),
    # enough rows along the contiguous axis for the LDS-staged row kernel
    ((65536, 130), (3, 5)),
    ((256, 64, 200), (2, 3, 64)),
    # boxes of 17 to 64 along strided axes and axis 0 (2 or 4 lanes per
    # column): fewer columns than a wavefront's group (columns of several
    # outer indices in one group), ragged groups, k = n, many runs along a
    # long axis with few columns, lower levels adding their terms
    ((200, 47, 3), (1, 40, 1)),
    ((90, 33), (17, 1)),
    ((3000, 5), (64, 2)),
    ((64, 100, 16), (3, 33, 2)),
    ((50, 129, 40), (20, 64, 3)),
    ((2, 2000, 70), (2, 37, 5)),
    ((100, 48), (48, 48)),
    ((65, 64, 64), (64, 17, 32)),
    ((33, 20, 30, 40), (33, 20, 18, 3)),
    # ... and along the contiguous axis of many rows (LDS-staged tiles of
    # 64 / G rows)
    ((20000, 70), (2, 33)),
    ((8192, 100), (3, 20)),
]

DTYPE_OPS = [("f32", "sum"), ("f32", "max"), ("f32", "min"), ("f64", "sum"), ("f64", "max"),
             ("f64", "min"), ("i32", "sum"), ("i32", "max"), ("i32", "min"), ("i64", "sum"),
             ("i64", "max"), ("i64", "min")]


@pytest.mark.parametrize("shape,box", CASES, ids=lambda v: "x".join(map(str, v)))
@pytest.mark.parametrize("dtype,op", DTYPE_OPS, ids=lambda v: str(v))
def test_parity_small(orc, shape, box, dtype, op):
    say(f"[parity] shape={shape} box={box} dtype={dtype} op={op} seed={seed_of(shape, box, dtype, op)}")
    a = make_input(shape, dtype, seed=seed_of(shape, box, dtype, op), op=op)
    inc, exc = gpu_run(a, box, op, "both")
    compare_full(orc, a, box, op, dtype, inc, exc, what=f"{shape} {box} {dtype} {op}")


# rank >= 3 cases that take the fused plane kernel: several tiles in both
# plane axes, several runs of blocks along axis 0, each k0 bucket (which sets
# the workgroup size and tile), boxes at the tile limit, middle axes (d >= 4)
PLANE_CASES = [
    ((40, 70, 90), (5, 7, 9)),
    ((100, 33, 65), (16, 16, 16)),
    ((70, 40, 50), (33, 5, 6)),
    ((64, 20, 30), (20, 16, 16)),
    ((130, 17, 19), (1, 1, 1)),
    ((3, 100, 100), (3, 16, 16)),
    ((7, 45, 70), (2, 32, 32)),
    ((5, 6, 7, 40, 50), (2, 3, 4, 5, 6)),
    ((16, 8, 64, 64), (8, 8, 4, 4)),
    # every (k0 bucket, plane-box bucket) pair, odd boxes, ragged tile edges
    ((37, 50, 41), (3, 2, 1)),
    ((29, 45, 70), (3, 3, 4)),
    ((40, 33, 35), (5, 7, 6)),
    ((41, 70, 39), (7, 11, 13)),
    ((50, 20, 100), (12, 2, 16)),
    ((33, 64, 31), (16, 5, 3)),
    ((65, 47, 48), (13, 16, 9)),
    # 32 blocks along axis 0 and 33, 40, 63 and 64 (one-pass block scans with
    # the 32- and 64-block register tables), 65 (separate passes)
    ((64, 40, 40), (2, 5, 5)),
    ((66, 40, 40), (2, 5, 5)),
    ((160, 36, 41), (4, 5, 6)),
    ((630, 20, 40), (10, 3, 4)),
    ((256, 33, 20), (4, 16, 2)),
    ((130, 40, 40), (2, 5, 5)),
    ((96, 8, 40, 30), (2, 2, 5, 3)),
    # levels 1 and 2 from the level-0 scan's block aggregates in one
    # workgroup: the largest table it takes (32 blocks x 512) and one block
    # more (the separate passes), the longest last level it takes (4096) and
    # a table too big with a long last level
    ((6, 128, 512), (3, 4, 8)),
    ((6, 132, 512), (3, 4, 8)),
    ((4, 32, 4096), (2, 16, 16)),
    ((4, 160, 2048), (2, 16, 16)),
    # 64 tiles: four runs of eight blocks along axis 0
    ((64, 256, 256), (2, 16, 16)),
    # rank >= 4: the block aggregates taken with the box sums along the
    # innermost middle axis with k > 1 (runs of 1, 2 or 4 of its blocks, a
    # ragged last block, a middle axis with k = 1 skipped, the other middle
    # axes as separate passes, a partial last block of axis 0, k0 = 1)
    ((20, 37, 40, 30), (3, 5, 6, 7)),
    ((19, 9, 70, 40, 30), (4, 3, 16, 5, 6)),
    ((18, 41, 1, 50, 40), (5, 9, 1, 4, 4)),
    ((17, 6, 7, 5, 30, 40), (2, 2, 3, 1, 3, 4)),
    ((33, 12, 25, 36), (1, 11, 2, 3)),
    ((10, 50, 35, 33), (8, 2, 4, 5)),
]


@pytest.mark.parametrize("shape,box", PLANE_CASES, ids=lambda v: "x".join(map(str, v)))
@pytest.mark.parametrize("dtype,op", DTYPE_OPS, ids=lambda v: str(v))
def test_parity_plane(orc, shape, box, dtype, op):
    say(f"[plane] shape={shape} box={box} dtype={dtype} op={op} seed={seed_of(shape, box, dtype, op, 1)}")
    a = make_input(shape, dtype, seed=seed_of(shape, box, dtype, op, 1), op=op)
    inc, exc = gpu_run(a, box, op, "both")
    compare_full(orc, a, box, op, dtype, inc, exc, what=f"{shape} {box} {dtype} {op}")
    if dtype == "i32" and op == "sum":
        for mode in ("inc", "exc"):
            i2, e2 = gpu_run(a, box, op, mode)
            assert np.array_equal(i2 if mode == "inc" else e2, inc if mode == "inc" else exc)


@pytest.mark.parametrize("mode", ["inc", "exc"])
@pytest.mark.parametrize("shape,box", [((20, 30, 40), (3, 5, 7)), ((50001,), (9,))],
                         ids=lambda v: "x".join(map(str, v)))
def test_single_output_modes(orc, mode, shape, box):
    a = make_input(shape, "i32", seed=5, op="sum")
    inc, exc = gpu_run(a, box, "sum", mode)
    assert (inc is None) == (mode == "exc") and (exc is None) == (mode == "inc")
    compare_full(orc, a, box, "sum", "i32", inc, exc, what=mode)


def test_config_d2_64x64_i64(orc):
    """64x64 int64 in [-100, 100], box (8, 8), +: against brute force and corners."""
    from paper_2106_00124_amd.workloads import WORKLOADS
    w = WORKLOADS["d2_64x64_i64"]
    a = w.tensor()
    say(f"[config] {w.name}")
    inc, exc = gpu_run(a, w.box, "sum", "both")
    ri, re_ = orc.brute(a, w.box, "sum", "i64")
    assert np.array_equal(inc, ri)
    assert np.array_equal(exc, re_)
    assert np.array_equal(exc, orc.corners2d(a, w.box, "sum", "i64"))
    assert np.all(inc + exc == a.sum())


def test_deterministic(orc):
    a = make_input((40, 50, 60), "f32", seed=9, op="sum")
    i1, e1 = gpu_run(a, (5, 6, 7), "sum")
    i2, e2 = gpu_run(a, (5, 6, 7), "sum")
    assert np.array_equal(i1, i2) and np.array_equal(e1, e2)


WEAK_CASES = [
    ((1000,), (64,)),
    ((50001,), (9,)),
    ((64, 64), (8, 8)),
    ((13, 70), (4, 9)),
    ((33, 17, 65), (16, 16, 16)),
    ((40, 70, 90), (5, 7, 9)),
    ((16, 8, 64, 64), (8, 8, 4, 4)),
    ((5, 6, 7, 40, 50), (2, 3, 4, 5, 6)),
    ((64, 256, 256), (2, 16, 16)),
    ((70, 40, 50), (33, 5, 6)),
]


@pytest.mark.parametrize("shape,box", WEAK_CASES, ids=lambda v: "x".join(map(str, v)))
@pytest.mark.parametrize("dtype", ["f32", "f64", "i32", "i64"])
def test_parity_weak(orc, shape, box, dtype):
    """Weak excluded sums (total - included, + only) against the oracle; the
    included output of the same call is the strong path's."""
    say(f"[weak] shape={shape} box={box} dtype={dtype} seed={seed_of(shape, box, dtype, 7)}")
    a = make_input(shape, dtype, seed=seed_of(shape, box, dtype, 7), op="sum")
    inc, exc = gpu_run(a, box, "sum", "both_weak")
    compare_full(orc, a, box, "sum", dtype, inc, exc, what=f"weak {shape} {box} {dtype}")
    _, exc_only = gpu_run(a, box, "sum", "weak")
    inc_strong, _ = gpu_run(a, box, "sum", "inc")
    if dtype in ("i32", "i64"):
        assert np.array_equal(exc_only, exc)
        assert np.array_equal(inc, inc_strong)
    else:
        compare_full(orc, a, box, "sum", dtype, None, exc_only, what="weak exc only")


def test_weak_max_unsupported():
    import torch
    import paper_2106_00124_amd as P
    from paper_2106_00124_amd import ExsError
    x = torch.zeros((8, 8), device="cuda")
    for op in ("max", "min"):
        with pytest.raises(ExsError, match="EUNSUPPORTED"):
            P.run(x, (2, 2), op, "weak")


@pytest.mark.parametrize("n,k", [(33566777, 7), (73000000, 16)])
@pytest.mark.parametrize("dtype,op", [("i32", "sum"), ("f32", "max")], ids=lambda v: str(v))
def test_parity_long1d_many_chunks(orc, n, k, dtype, op):
    """A 1-D tensor of more chunk totals than one tile of the chunk-total scan
    (8192): two and three tiles, the carries across them in both directions."""
    seed = seed_of(n, k, dtype, op, "long1d")
    say(f"[long1d] n={n} k={k} dtype={dtype} op={op} seed={seed}")
    a = make_input((n,), dtype, seed=seed, op=op)
    inc, exc = gpu_run(a, (k,), op, "both")
    ri, re_ = orc.scale(a, (k,), op, dtype)
    tolerance.check(inc, ri, dtype, op, what=f"long1d {n} {k} inc")
    tolerance.check(exc, re_, dtype, op, what=f"long1d {n} {k} exc")


# one output at a time through the axis-0 stream for boxes of 17 to 64 along
# axis 0 (the single-output forms keep one block array, not two)
AX0_ONE_OUTPUT = [
    ((200, 33, 40), (40, 3, 5)),
    ((130, 70), (64, 2)),
    ((3000, 5), (33, 2)),
    ((90, 16, 16), (17, 1, 1)),
]


@pytest.mark.parametrize("mode", ["inc", "exc"])
@pytest.mark.parametrize("shape,box", AX0_ONE_OUTPUT, ids=lambda v: "x".join(map(str, v)))
@pytest.mark.parametrize("dtype,op", [("f32", "sum"), ("i32", "max"), ("f64", "min")],
                         ids=lambda v: str(v))
def test_parity_axis0_one_output(orc, mode, shape, box, dtype, op):
    seed = seed_of(shape, box, dtype, op, mode, "ax0one")
    say(f"[ax0-one] shape={shape} box={box} dtype={dtype} op={op} mode={mode} seed={seed}")
    a = make_input(shape, dtype, seed=seed, op=op)
    inc, exc = gpu_run(a, box, op, mode)
    compare_full(orc, a, box, op, dtype, inc, exc, what=f"{shape} {box} {dtype} {op} {mode}")


# fused levels with more than 64 blocks along axis 0: the trailing-axes pass
# (or the row pass of a 2-D level), then the block scans, which store the block prefix only where the stream's
# runs start; at least 2^18 points take the direct scan, fewer the segmented
# one (a ragged last block and segment, boxes of different buckets on the
# trailing axes)
TWO_PASS = [
    ((141, 512, 520), (2, 5, 3)),
    ((133, 520, 512), (2, 3, 16)),
    ((301, 100, 120), (2, 5, 7)),
    ((1030, 64, 40), (4, 3, 16)),
    # 2-D levels streamed by the fused row kernel
    ((2001, 300), (8, 5)),
    ((141, 262150), (2, 7)),
]


@pytest.mark.parametrize("shape,box", TWO_PASS, ids=lambda v: "x".join(map(str, v)))
@pytest.mark.parametrize("dtype,op", [("i32", "sum"), ("f32", "max"), ("f32", "sum")],
                         ids=lambda v: str(v))
def test_parity_fused_two_pass_scan(orc, shape, box, dtype, op):
    seed = seed_of(shape, box, dtype, op, "twopass")
    say(f"[two-pass] shape={shape} box={box} dtype={dtype} op={op} seed={seed}")
    a = make_input(shape, dtype, seed=seed, op=op)
    inc, exc = gpu_run(a, box, op, "both")
    compare_full(orc, a, box, op, dtype, inc, exc, what=f"two-pass {shape} {box}")


# rank-2 tensors small enough for the one-workgroup kernel (at most 128 rows,
# 1024 columns, 32 KiB, boxes of at most 64 along axis 1) and just past each of
# its limits (the general chain of launches): both outputs and each alone
SMALL2D = [
    ((1, 1), (1, 1)),
    ((1, 1024), (1, 64)),
    ((8, 1024), (3, 17)),
    ((128, 64), (128, 64)),
    ((128, 64), (5, 1)),
    ((127, 33), (10, 7)),
    ((129, 2), (4, 2)),
    ((100, 90), (9, 65)),
    ((2, 1025), (2, 3)),
]


@pytest.mark.parametrize("shape,box", SMALL2D, ids=lambda v: "x".join(map(str, v)))
@pytest.mark.parametrize("dtype,op", [("f32", "sum"), ("f64", "sum"), ("i32", "max"),
                                      ("i64", "min"), ("f32", "max")], ids=lambda v: str(v))
@pytest.mark.parametrize("mode", ["both", "inc", "exc"])
def test_parity_small2d(orc, shape, box, dtype, op, mode):
    seed = seed_of(shape, box, dtype, op, mode, "small2d")
    say(f"[small2d] shape={shape} box={box} dtype={dtype} op={op} mode={mode} seed={seed}")
    a = make_input(shape, dtype, seed=seed, op=op)
    inc, exc = gpu_run(a, box, op, mode)
    compare_full(orc, a, box, op, dtype, inc if mode != "exc" else None,
                 exc if mode != "inc" else None, what=f"small2d {shape} {box} {mode}")


# boxes longer than 64 with few columns: the sweeps in chunks of rows (chunks
# shorter and longer than the box, a ragged last chunk, k = n, the excluded
# part along axis 0 and BDBS along strided and contiguous axes)
LONG_BOX = [
    ((300, 50), (100, 3)),
    ((4100, 3), (65, 3)),
    ((1000, 7, 90), (130, 2, 70)),
    ((200, 300), (7, 200)),
    ((129, 130), (129, 130)),
    ((70, 5000), (66, 1)),
]


@pytest.mark.parametrize("shape,box", LONG_BOX, ids=lambda v: "x".join(map(str, v)))
@pytest.mark.parametrize("dtype,op", [("f32", "sum"), ("i32", "max"), ("f64", "min"),
                                      ("i64", "sum")], ids=lambda v: str(v))
def test_parity_long_box_chunked(orc, shape, box, dtype, op):
    seed = seed_of(shape, box, dtype, op, "longbox")
    say(f"[long-box] shape={shape} box={box} dtype={dtype} op={op} seed={seed}")
    a = make_input(shape, dtype, seed=seed, op=op)
    inc, exc = gpu_run(a, box, op, "both")
    compare_full(orc, a, box, op, dtype, inc, exc, what=f"long-box {shape} {box}")
