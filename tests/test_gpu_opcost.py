"""The artificially slowed + (measurement support for the operator-cost
experiment): the same results as the plain operator, bit for bit, on every
kernel path it runs through, and the probe applies it the stated number of
times."""
import ctypes

import numpy as np
import pytest

from tests.gpu_util import make_input, say, seed_of

pytestmark = pytest.mark.gpu

CASES = [((5000,), (7,)), ((300, 200), (5, 9)), ((40, 50, 60), (4, 5, 6)),
         ((64, 64, 64), (16, 16, 16)), ((12, 10, 9, 8), (3, 2, 4, 5)), ((33, 17, 9), (33, 17, 9))]


@pytest.mark.parametrize("shape,box", CASES, ids=lambda v: "x".join(map(str, v)))
def test_slowed_sum_identical(shape, box):
    import torch
    import paper_2106_00124_amd as P
    from paper_2106_00124_amd import _lib
    L = _lib.lib()
    seed = seed_of(shape, box, "opcost")
    say(f"[opcost] shape={shape} box={box} seed={seed}")
    x = torch.from_numpy(make_input(shape, "f32", seed, "sum")).cuda()
    ri, re_ = P.run(x, box, "sum", "both")
    torch.cuda.synchronize()
    try:
        _lib.check(L.exs_set_op_cost(24))
        si, se = P.run(x, box, "sum", "both")
        torch.cuda.synchronize()
    finally:
        _lib.check(L.exs_set_op_cost(0))
    assert torch.equal(si, ri) and torch.equal(se, re_)


def test_probe_applies_reps_times():
    import torch
    from paper_2106_00124_amd import _lib
    L = _lib.lib()
    v = torch.arange(1, 1001, dtype=torch.float32, device="cuda")
    try:
        _lib.check(L.exs_set_op_cost(5))
        _lib.check(L.exs_op_probe(ctypes.c_void_p(v.data_ptr()), v.numel(), 8,
                                  ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)))
        torch.cuda.synchronize()
    finally:
        _lib.check(L.exs_set_op_cost(0))
    assert torch.equal(v.cpu(), torch.arange(1, 1001, dtype=torch.float32) * 8)
    assert L.exs_set_op_cost(-1) == _lib.EINVAL
