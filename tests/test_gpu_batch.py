"""Batched form: one graph launch over many uneven jobs vs the oracle and vs
the plain per-tensor call."""
import json
import os

import numpy as np
import pytest

from tests import tolerance
from tests.gpu_util import make_input, say

pytestmark = pytest.mark.gpu

DT = {"f32": "float32", "i32": "int32", "f64": "float64", "i64": "int64"}


def _mixed_items(seed, count):
    """Uneven ranks, shapes, boxes, dtypes and operators (small sizes)."""
    rng = np.random.default_rng(seed)
    items = []
    for t in range(count):
        d = int(rng.integers(1, 5))
        shape = tuple(int(rng.integers(2, 40 if d >= 3 else 90)) for _ in range(d))
        box = tuple(int(rng.integers(1, n + 1)) for n in shape)
        dtype = ["f32", "i32", "f64", "i64"][t % 4]
        op = ["sum", "max", "min"][(t // 4) % 3]
        mode = ["both", "exc", "inc"][t % 3]
        items.append((shape, box, dtype, op, mode, int(rng.integers(0, 2**31))))
    # a long box (two-sweep kernels) and a 1-element tensor
    items.append(((300, 7), (100, 3), "i32", "sum", "both", 11))
    items.append(((1, 1, 1), (1, 1, 1), "f32", "max", "both", 12))
    # many rows along the contiguous axis (LDS-staged row tasks)
    items.append(((40000, 70), (3, 9), "f32", "sum", "both", 13))
    items.append(((300, 200, 64), (5, 4, 33), "i32", "max", "both", 14))
    # many blocks for few points (segmented block scans)
    items.append(((20000, 5), (3, 2), "f32", "sum", "both", 15))
    items.append(((60000,), (2,), "i32", "max", "exc", 16))
    items.append(((50, 60, 70), (4, 5, 6), "f32", "min", "both", 17))
    return items


def _run_batch(items, tune_cache=None, graph=True):
    import torch
    import paper_2106_00124_amd as P
    host = [make_input(s, dt, seed, op) for (s, b, dt, op, m, seed) in items]
    dev = [torch.from_numpy(np.ascontiguousarray(a)).cuda() for a in host]
    B = P.Batch([(x, it[1], it[3], it[4]) for x, it in zip(dev, items)], tune_cache=tune_cache)
    if graph:
        B.launch()
    else:
        B.launch_eager()
    torch.cuda.synchronize()
    outs = [(i.cpu().numpy() if i is not None else None, e.cpu().numpy() if e is not None else None)
            for i, e in B.outputs]
    return B, host, dev, outs


def test_batch_matches_oracle_and_plain(orc):
    import torch
    import paper_2106_00124_amd as P
    items = _mixed_items(3, 40)
    say(f"[batch] {len(items)} jobs")
    B, host, dev, outs = _run_batch(items)
    for (shape, box, dt, op, mode, seed), a, x, (inc, exc) in zip(items, host, dev, outs):
        ri, re_ = (orc.brute(a, box, op, dt) if a.size <= 2048 else orc.scale(a, box, op, dt))
        si = se = None
        if dt in ("f32", "f64") and op == "sum":
            si = tolerance.sigma_full(orc, a, box, "inc")
            se = tolerance.sigma_full(orc, a, box, "exc")
        what = f"{shape} {box} {dt} {op} {mode}"
        if inc is not None:
            tolerance.check(inc, ri, dt, op, si, what=what + " inc")
        if exc is not None:
            tolerance.check(exc, re_, dt, op, se, what=what + " exc")
        # the plain call: identical for integers and max (order-free)
        pi, pe = P.run(x, box, op, mode)
        torch.cuda.synchronize()
        if dt in ("i32", "i64") or op != "sum":
            if inc is not None:
                assert np.array_equal(pi.cpu().numpy(), inc), what
            if exc is not None:
                assert np.array_equal(pe.cpu().numpy(), exc), what
    info = B.info()
    assert info["graph_nodes"] > 0 and info["work_items"] >= len(items)


def test_graph_replay_equals_eager(orc):
    import torch
    items = _mixed_items(5, 16)
    B, host, dev, outs = _run_batch(items, graph=True)
    for rep in range(3):
        B.launch()
        torch.cuda.synchronize()
        again = [(i.cpu().numpy() if i is not None else None,
                  e.cpu().numpy() if e is not None else None) for i, e in B.outputs]
        for (a0, b0), (a1, b1) in zip(outs, again):
            for u, v in ((a0, a1), (b0, b1)):
                if u is not None:
                    assert np.array_equal(u, v)
    B.launch_eager()
    torch.cuda.synchronize()
    for (a0, b0), (i, e) in zip(outs, B.outputs):
        if a0 is not None:
            assert np.array_equal(a0, i.cpu().numpy())
        if b0 is not None:
            assert np.array_equal(b0, e.cpu().numpy())


def test_autotune_cache_written_and_reused(tmp_path, orc):
    items = _mixed_items(7, 8)
    path = str(tmp_path / "tune.json")
    B, host, dev, outs = _run_batch(items, tune_cache=path)
    data = json.load(open(path))
    assert len(data["entries"]) == 1
    entry = next(iter(data["entries"].values()))
    assert entry["min_tasks"] > 0 and entry["wg_per_cu"] > 0
    mtime = os.path.getmtime(path)
    B2, _, _, outs2 = _run_batch(items, tune_cache=path)
    assert os.path.getmtime(path) == mtime  # served from the cache
    for (a0, b0), (a1, b1) in zip(outs, outs2):
        for u, v in ((a0, a1), (b0, b1)):
            if u is not None:
                assert np.array_equal(u, v) or u.dtype.kind == "f"


def test_autotune_leaves_a_foreign_file_alone(tmp_path):
    # a file at the cache path that is not a cache: tuned, not overwritten
    items = _mixed_items(11, 5)
    path = tmp_path / "tune.json"
    foreign = '{"note": "} not a cache {", "entries": [1, 2]}'
    path.write_text(foreign)
    B, host, dev, outs = _run_batch(items, tune_cache=str(path))
    assert path.read_text() == foreign
    B2, _, _, outs2 = _run_batch(items)
    for (a0, b0), (a1, b1) in zip(outs, outs2):
        for u, v in ((a0, a1), (b0, b1)):
            if u is not None:
                assert np.array_equal(u, v) or u.dtype.kind == "f"


def test_batch_rejects_invalid_job():
    import torch
    import paper_2106_00124_amd as P
    from paper_2106_00124_amd import ExsError
    x = torch.zeros((4, 4), device="cuda")
    with pytest.raises(ExsError):
        P.Batch([(x, (5, 1), "sum", "both")])


def test_batch_rejects_weak_jobs():
    import torch
    import paper_2106_00124_amd as P
    from paper_2106_00124_amd import ExsError
    x = torch.zeros((16, 16), device="cuda")
    with pytest.raises(ExsError, match="EUNSUPPORTED"):
        P.Batch([(x, (2, 2), "sum", "weak")])


def test_stated_batch_matches_oracle(orc):
    """The stated batched workload (512 tensors: rank 2-4, dims log-uniform in
    [16, 256] up to 2^22 elements, box sides up to 32, f32 N(0,1) / i32
    uniform [-100, 100], + or max) in one graph launch: 2000 sampled cells of
    every tensor's included and excluded sums, and every cell of the 32
    largest tensors, against the oracle (bit-exact for i32 and max, the
    per-cell f32 rule otherwise)."""
    import torch
    import paper_2106_00124_amd as P
    from paper_2106_00124_amd import workloads as W
    items = W.batch_workload()
    assert len(items) == 512
    host = [it.tensor() for it in items]
    dev = [torch.from_numpy(np.ascontiguousarray(a)).cuda() for a in host]
    say(f"[batch] stated workload: {len(items)} tensors, "
        f"{sum(it.n for it in items) / 1e6:.0f} M elements")
    B = P.Batch([(x, it.box, it.op, "both") for x, it in zip(dev, items)])
    B.launch()
    torch.cuda.synchronize()
    rng = np.random.default_rng(515)
    largest = set(sorted(range(len(items)), key=lambda i: -items[i].n)[:32])
    for t, (it, a, (inc, exc)) in enumerate(zip(items, host, B.outputs)):
        what = f"tensor {t} {it.shape} {it.box} {it.dtype} {it.op}"
        if t in largest:
            ri, re_ = orc.scale(a, it.box, it.op, it.dtype)
            si = se = None
            if it.dtype == "f32" and it.op == "sum":
                si = tolerance.sigma_full(orc, a, it.box, "inc")
                se = tolerance.sigma_full(orc, a, it.box, "exc")
            tolerance.check(inc.cpu().numpy(), ri, it.dtype, it.op, si, what=what + " inc")
            tolerance.check(exc.cpu().numpy(), re_, it.dtype, it.op, se, what=what + " exc")
            continue
        pts = np.concatenate([rng.integers(0, it.n, 2000), [0, it.n - 1]]).astype(np.int64)
        ip = torch.from_numpy(pts).cuda()
        gi = inc.reshape(-1)[ip].cpu().numpy()
        ge = exc.reshape(-1)[ip].cpu().numpy()
        ri = orc.point_inc(a, it.box, it.op, it.dtype, pts)
        re_ = orc.point_exc(a, it.box, it.op, it.dtype, pts)
        si = se = None
        if it.dtype == "f32" and it.op == "sum":
            si = tolerance.sigma_points(orc, a, it.box, "inc", pts)
            se = tolerance.sigma_points(orc, a, it.box, "exc", pts)
        tolerance.check(gi, ri, it.dtype, it.op, si, what=what + " inc")
        tolerance.check(ge, re_, it.dtype, it.op, se, what=what + " exc")
    say("[batch] stated workload checked")
    B.close()
