"""The full-size workloads, in the launch configuration the benchmark times
(preallocated outputs and workspace, torch's current stream), against the
oracle on every element, plus directly summed excluded sums at sampled
cells and the + invariant on integers."""
import numpy as np
import pytest

from tests import tolerance
from tests.gpu_util import say

pytestmark = pytest.mark.gpu


def _run_like_bench(a_host, box, ops):
    import torch
    import paper_2106_00124_amd as P
    a = torch.from_numpy(a_host).cuda()
    ws_bytes = max(P.workspace_size(a_host.shape, box, a.dtype, op, "both") for op in ops)
    ws = torch.empty(max(ws_bytes, 1), dtype=torch.uint8, device=a.device)
    stream = torch.cuda.current_stream()
    res = {}
    for op in ops:
        inc, exc = torch.empty_like(a), torch.empty_like(a)
        P.run(a, box, op, "both", inc_out=inc, exc_out=exc, workspace=ws, stream=stream)
        res[op] = (inc, exc)
    torch.cuda.synchronize()
    return {op: (i.cpu().numpy(), e.cpu().numpy()) for op, (i, e) in res.items()}


def _check_config(orc, name, direct_points):
    from paper_2106_00124_amd.workloads import WORKLOADS
    w = WORKLOADS[name]
    say(f"[config] {w.name} shape={w.shape} box={w.box}")
    a = w.tensor()
    out = _run_like_bench(a, w.box, w.ops)
    rng = np.random.default_rng(17)
    pts = np.concatenate([rng.integers(0, a.size, direct_points), [0, a.size - 1]])
    for op in w.ops:
        inc, exc = out[op]
        ri, re_ = orc.scale(a, w.box, op, w.dtype)
        si = se = None
        if op == "sum" and w.dtype == "f32":
            si = tolerance.sigma_full(orc, a, w.box, "inc")
            se = tolerance.sigma_full(orc, a, w.box, "exc")
        s1 = tolerance.check(inc, ri, w.dtype, op, si, what=f"{name} {op} inc")
        s2 = tolerance.check(exc, re_, w.dtype, op, se, what=f"{name} {op} exc")
        say(f"  {op}: inc {s1} exc {s2}")
        del ri, re_, si, se
        # excluded sums summed directly over the complement at sampled cells
        pd = orc.point_exc_direct(a, w.box, op, w.dtype, pts)
        spd = None
        if op == "sum" and w.dtype == "f32":
            spd = tolerance.sigma_points(orc, a, w.box, "exc", pts)
        tolerance.check(exc.reshape(-1)[pts], pd, w.dtype, op, spd, what=f"{name} {op} direct")
        if w.dtype in ("i32", "i64") and op == "sum":
            # included + excluded = the total, in the dtype's wrapping arithmetic
            tot = a.astype(np.int64).sum()
            if w.dtype == "i32":
                tot = np.int64(np.int32(np.int64(tot).astype(np.int32)))
                s = inc.astype(np.int64) + exc.astype(np.int64)
                s = s.astype(np.int32).astype(np.int64)
            else:
                s = inc + exc
            assert np.all(s == tot)


def test_config_d3_512_f32(orc):
    _check_config(orc, "d3_512_f32", direct_points=24)


def test_config_d5_32_f32(orc):
    _check_config(orc, "d5_32_f32", direct_points=64)


def test_config_d4_128x128x64x64_i32(orc):
    _check_config(orc, "d4_128x128x64x64_i32", direct_points=64)


@pytest.mark.parametrize("shape,box", [
    ((64, 4096, 4096), (16, 16, 16)),   # 2^30 elements through the fused plane kernel
    ((3, 715827883), (2, 7)),           # more than 2^31 elements (64-bit indexing)
    ((1 << 25,), (8,)),                 # the most chunks the chunked 1-D kernels take (8192)
    (((1 << 25) + 1,), (8,)),          # one element more: the generic 1-D path
], ids=["2^30_plane", "over_2^31", "1d_8192_chunks", "1d_8193_chunks"])
def test_max_size_closed_form(shape, box):
    """All-ones int32 tensors at the largest sizes: included sums have the
    closed form prod_i min(k_i, n_i - x_i) and excluded sums N - included
    (two's-complement wrapping), checked on every cell (on the device) and at
    sampled cells (on the host)."""
    import torch
    import paper_2106_00124_amd as P
    say(f"[max size] {shape} {box}")
    x = torch.ones(shape, dtype=torch.int32, device="cuda")
    inc, exc = P.run(x, box, "sum", "both")
    torch.cuda.synchronize()
    N = int(np.prod(shape))
    wrapN = np.int64(N).astype(np.int32)   # N mod 2^32 as int32
    # every cell: inc + exc == N (mod 2^32), via wrapping int32 addition
    assert bool(torch.all(inc + exc == int(wrapN)).item())
    del x
    # sampled cells against the closed form
    rng = np.random.default_rng(5)
    flat = np.concatenate([rng.integers(0, N, 256), [0, N - 1]])
    coords = np.array(np.unravel_index(flat, shape)).T
    ref = np.ones(len(flat), dtype=np.int64)
    for i, (n, k) in enumerate(zip(shape, box)):
        ref *= np.minimum(k, n - coords[:, i])
    idx = torch.from_numpy(flat).cuda()
    got_inc = inc.reshape(-1)[idx].cpu().numpy().astype(np.int64)
    got_exc = exc.reshape(-1)[idx].cpu().numpy()
    assert np.array_equal(got_inc, ref)
    assert np.array_equal(got_exc, (N - ref).astype(np.int64).astype(np.int32))
