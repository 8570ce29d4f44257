"""The corners algorithm (the paper's comparison system, two dimensions) on
the GPU: against the CPU oracle element by element, and against the
box-complement path of the same library (bit-exact wherever the arithmetic is
exact: integer +, max, min)."""
import numpy as np
import pytest

from tests import tolerance
from tests.gpu_util import compare_full, gpu_run, make_input, say, seed_of

pytestmark = pytest.mark.gpu

# one segment and several (64 rows each, ragged last), rows shorter and longer
# than a 256-column chunk, k = 1 and k = n, single rows and columns
CASES = [
    ((1, 1), (1, 1)),
    ((1, 9), (1, 4)),
    ((9, 1), (3, 1)),
    ((64, 64), (8, 8)),
    ((13, 70), (4, 9)),
    ((70, 13), (13, 1)),
    ((130, 77), (7, 5)),
    ((65, 300), (64, 1)),
    ((200, 1000), (16, 16)),
    ((1000, 3), (5, 3)),
    ((3, 1000), (3, 100)),
    ((257, 513), (257, 1)),
    ((100, 100), (100, 100)),
    ((129, 257), (1, 1)),
]

DTYPE_OPS = [("f32", "sum"), ("f32", "max"), ("f32", "min"), ("f64", "sum"), ("i32", "sum"),
             ("i32", "max"), ("i64", "sum"), ("i64", "min")]


def corners(a, box, op):
    import torch
    import paper_2106_00124_amd as P
    t = torch.from_numpy(np.ascontiguousarray(a)).cuda()
    e = P.run_corners(t, box, op)
    torch.cuda.synchronize()
    return e.cpu().numpy()


@pytest.mark.parametrize("shape,box", CASES, ids=lambda v: "x".join(map(str, v)))
@pytest.mark.parametrize("dtype,op", DTYPE_OPS, ids=lambda v: str(v))
def test_corners_parity(orc, shape, box, dtype, op):
    seed = seed_of(shape, box, dtype, op, "corners")
    say(f"[corners] shape={shape} box={box} dtype={dtype} op={op} seed={seed}")
    a = make_input(shape, dtype, seed=seed, op=op)
    exc = corners(a, box, op)
    compare_full(orc, a, box, op, dtype, None, exc, what=f"corners {shape} {box} {dtype} {op}")
    if dtype in ("i32", "i64") or op != "sum":
        _, exc_bc = gpu_run(a, box, op, "exc")
        assert np.array_equal(exc, exc_bc)


def test_corners_config_d2_64x64_i64(orc):
    """The 64x64 int64 workload, box (8, 8), +: equal to brute force, to the
    oracle's own corners form and to the box-complement path."""
    from paper_2106_00124_amd.workloads import WORKLOADS
    w = WORKLOADS["d2_64x64_i64"]
    a = w.tensor()
    exc = corners(a, w.box, "sum")
    _, ref = orc.brute(a, w.box, "sum", "i64")
    assert np.array_equal(exc, ref)
    assert np.array_equal(exc, orc.corners2d(a, w.box, "sum", "i64"))
    _, exc_bc = gpu_run(a, w.box, "sum", "exc")
    assert np.array_equal(exc, exc_bc)


@pytest.mark.parametrize("op", ["sum", "max"])
def test_corners_large_sampled(orc, op):
    """4096 x 4096 f32 (the size the corners comparison is timed at), box
    (16, 16): every cell against the box-complement path (max bit-exact, +
    within the tolerance relative to that path's own error), and sampled cells
    against the oracle."""
    import torch
    import paper_2106_00124_amd as P
    shape, box = (4096, 4096), (16, 16)
    seed = seed_of(shape, box, op, "corners-large")
    say(f"[corners-large] op={op} seed={seed}")
    rng = np.random.default_rng(seed)
    a = rng.standard_normal(shape).astype(np.float32)
    t = torch.from_numpy(a).cuda()
    exc = P.run_corners(t, box, op)
    _, exc_bc = P.run(t, box, op, "exc")
    torch.cuda.synchronize()
    g, b = exc.cpu().numpy(), exc_bc.cpu().numpy()
    # flat indices: random cells, the four corners and one near the last block
    pts = np.concatenate([rng.integers(0, a.size, 2000),
                          [0, a.size - 1, 4095, 4095 * 4096, 4080 * 4096 + 17]]).astype(np.int64)
    ref = orc.point_exc(a, box, op, "f32", pts)
    sig = tolerance.sigma_points(orc, a, box, "exc", pts) if op == "sum" else None
    got = g.reshape(-1)[pts]
    tolerance.check(got, ref, "f32", op, sig, what=f"corners 4096^2 {op}")
    if op == "max":
        assert np.array_equal(g, b)
    else:
        sig_all = np.sqrt(float((a.astype(np.float64) ** 2).sum()))
        assert np.max(np.abs(g.astype(np.float64) - b)) <= 2e-5 * sig_all


def test_corners_rejects():
    import torch
    import paper_2106_00124_amd as P
    from paper_2106_00124_amd import ExsError
    x3 = torch.zeros((4, 4, 4), device="cuda")
    with pytest.raises(ExsError, match="EUNSUPPORTED"):
        P.run_corners(x3, (2, 2, 2))
    x = torch.zeros((8, 8), device="cuda")
    with pytest.raises(ExsError, match="EINVAL"):
        P.run_corners(x, (9, 2))
