"""The CPU oracle against its pins (no GPU)."""
import os
import tempfile
import zlib

import numpy as np
import pytest

import oracle
from tests import oracle_pins as pins

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")


@pytest.mark.parametrize("pin", pins.ALL_PINS, ids=lambda p: p.__name__)
def test_pin(orc, pin):
    pin(orc)


AGREE_CASES = [
    ((13,), (5,)), ((16,), (16,)), ((1,), (1,)), ((9, 7), (4, 3)), ((8, 8), (8, 1)),
    ((5, 6, 7), (2, 3, 4)), ((4, 4, 4, 4), (3, 2, 1, 4)), ((3, 2, 4, 2, 3), (2, 2, 3, 1, 2)),
    ((2, 3, 2, 3, 2, 2), (2, 1, 2, 3, 1, 2)),
]


@pytest.mark.parametrize("shape,k", AGREE_CASES)
@pytest.mark.parametrize("dtype", ["f32", "f64", "i32", "i64"])
@pytest.mark.parametrize("op", ["sum", "max", "min"])
def test_brute_scale_point_agree(orc, shape, k, dtype, op):
    rng = np.random.default_rng(zlib.crc32(repr((shape, k, dtype, op)).encode()))
    if dtype in ("f32", "f64"):
        a = rng.standard_normal(shape).astype(np.float32 if dtype == "f32" else np.float64)
    else:
        a = rng.integers(-2**31, 2**31, size=shape).astype(np.int64)
    bi, be = orc.brute(a, k, op, dtype)
    si, se = orc.scale(a, k, op, dtype)
    N = a.size
    pts = np.arange(N)
    pi = orc.point_inc(a, k, op, dtype, pts).reshape(shape)
    pe = orc.point_exc(a, k, op, dtype, pts).reshape(shape)
    pd = orc.point_exc_direct(a, k, op, dtype, pts).reshape(shape)
    if dtype in ("f32", "f64") and op == "sum":
        scale = np.abs(a).astype(np.float64).sum()
        for x, y in ((bi, si), (bi, pi), (be, se), (be, pe), (be, pd)):
            assert np.max(np.abs(x - y)) <= 1e-13 * scale
    else:
        for x, y in ((bi, si), (bi, pi), (be, se), (be, pe), (be, pd)):
            assert np.array_equal(x, y)
    if len(shape) == 2:
        ce = orc.corners2d(a, k, op, dtype)
        if dtype in ("f32", "f64") and op == "sum":
            assert np.max(np.abs(ce - be)) <= 1e-13 * np.abs(a).astype(np.float64).sum()
        else:
            assert np.array_equal(ce, be)


def test_rejects_bad_args(orc):
    a = np.zeros((4, 4))
    for k in ([0, 1], [5, 1], [1, 1, 1]):
        with pytest.raises(ValueError):
            orc.brute(a, k, "sum", "f64")
        with pytest.raises(ValueError):
            orc.scale_inc(a, k, "sum", "f64")


# Each mutant plants one mistake in the oracle source (see ORC_MUTANT there):
#   1 closed box (off by one at the high edge)   2 wrong identity for max
#   3 axes reversed in the point oracle          4 no wrap of i32 sums
#   5 suffix half-space dropped in the max cover
#   6 wrong identity for integer min             7 the higher index wins ties of pairs
@pytest.mark.parametrize("mutant", [1, 2, 3, 4, 5, 6, 7])
def test_pins_catch_planted_mistakes(mutant):
    with tempfile.TemporaryDirectory() as td:
        path = oracle.build(mutant=mutant, out=os.path.join(td, f"m{mutant}.so"))
        bad = oracle.Oracle(path)
        with pytest.raises(AssertionError):
            pins.run_all(bad)
