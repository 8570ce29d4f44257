"""The struct monoid: (value, index) pairs under argmax / argmin through the
plain call, bit-exact against the oracle (the order is total, so every result
is unique).  Values are drawn from a few integers so that ties decide many
cells; indices are a random permutation, so that the lowest index among equal
values is not simply the first position."""
import numpy as np
import pytest

from tests.gpu_util import say, seed_of

pytestmark = pytest.mark.gpu

CASES = [
    ((1,), (1,)), ((50,), (7,)), ((300,), (300,)), ((9000,), (13,)),
    ((37, 41), (5, 9)), ((64, 64), (8, 8)), ((200, 3), (17, 3)),
    ((20, 30, 40), (3, 7, 40)), ((33, 17, 65), (16, 16, 16)), ((70, 40, 50), (33, 5, 6)),
    ((9, 8, 7, 6), (2, 3, 4, 5)), ((6, 5, 4, 5, 6), (3, 1, 2, 5, 2)),
    ((3, 4, 3, 4, 3, 4), (2, 2, 3, 1, 3, 2)),
]


def _pairs(shape, seed, ties=True):
    rng = np.random.default_rng(seed)
    vals = (rng.integers(-3, 4, size=shape) if ties else rng.standard_normal(shape))
    idx = rng.permutation(int(np.prod(shape))).reshape(shape).astype(np.int32)
    return vals.astype(np.float32), idx


@pytest.mark.parametrize("shape,box", CASES, ids=lambda v: "x".join(map(str, v)))
@pytest.mark.parametrize("op", ["max", "min"])
def test_pairs_match_oracle(orc, shape, box, op):
    import torch
    import paper_2106_00124_amd as P
    seed = seed_of(shape, box, op, "pairs")
    say(f"[pairs] shape={shape} box={box} op={op} seed={seed}")
    vals, idx = _pairs(shape, seed)
    x = P.pack_pairs(torch.from_numpy(vals).cuda(), torch.from_numpy(idx).cuda())
    inc, exc = P.run_pairs(x, box, op, "both")
    torch.cuda.synchronize()
    iv, ii = (t.cpu().numpy() for t in P.unpack_pairs(inc))
    ev, ei = (t.cpu().numpy() for t in P.unpack_pairs(exc))
    fn = orc.brute_vi if vals.size <= 2048 else orc.scale_vi
    rv, ri, qv, qi = fn(vals, idx, box, op)
    assert np.array_equal(iv.astype(np.float64), rv), "inc values"
    assert np.array_equal(ii.astype(np.int64), ri), "inc index"
    assert np.array_equal(ev.astype(np.float64), qv), "exc values"
    assert np.array_equal(ei.astype(np.int64), qi), "exc index"


@pytest.mark.parametrize("mode", ["inc", "exc"])
def test_pairs_single_output_and_positions(orc, mode):
    """One output at a time; default indices (flat positions) and distinct
    normal values: the index is the position of the best value."""
    import torch
    import paper_2106_00124_amd as P
    shape, box = (48, 37, 29), (5, 4, 6)
    vals, _ = _pairs(shape, 5, ties=False)
    xv = torch.from_numpy(vals).cuda()
    x = P.pack_pairs(xv)
    inc, exc = P.run_pairs(x, box, "max", mode)
    torch.cuda.synchronize()
    out = inc if mode == "inc" else exc
    assert (inc is None) == (mode == "exc") and (exc is None) == (mode == "inc")
    ov, oi = (t.cpu().numpy() for t in P.unpack_pairs(out))
    pos = np.arange(vals.size).reshape(shape)
    rv, ri, qv, qi = orc.scale_vi(vals, pos, box, "max")
    want_v, want_i = (rv, ri) if mode == "inc" else (qv, qi)
    assert np.array_equal(ov.astype(np.float64), want_v)
    assert np.array_equal(oi.astype(np.int64), want_i)
    # the index points at a cell holding the value
    assert np.array_equal(vals.reshape(-1)[oi.reshape(-1)], ov.reshape(-1))


def test_pairs_sum_rejected():
    import torch
    import paper_2106_00124_amd as P
    from paper_2106_00124_amd import ExsError
    x = P.pack_pairs(torch.zeros((8, 8), device="cuda"))
    with pytest.raises(ExsError, match="EUNSUPPORTED"):
        P.run_pairs(x, (2, 2), "sum", "both")
