"""Serving form: results alone equal results in the mix, admission by HBM
budget queues instead of failing, bad requests are rejected while the loop
keeps serving, and device-generated inputs equal their host twin."""
import numpy as np
import pytest

from tests import tolerance
from tests.gpu_util import make_input, say
from paper_2106_00124_amd import workloads as W

pytestmark = pytest.mark.gpu


def _mix(seed, count):
    rng = np.random.default_rng(seed)
    items = []
    for t in range(count):
        d = int(rng.integers(2, 4))
        shape = tuple(int(rng.integers(3, 70 if d == 3 else 300)) for _ in range(d))
        box = tuple(int(rng.integers(1, min(64, n) + 1)) for n in shape)
        dtype = ["f32", "i32", "i64", "f32"][t % 4]
        op = "max" if (t % 5 == 4 and dtype != "i64") else ("min" if t % 7 == 3 else "sum")
        mode = ["exc", "both", "inc"][t % 3]
        items.append((shape, box, dtype, op, mode, 1000 + t))
    return items


def _wait(S, tickets):
    import time
    out = {}
    deadline = time.time() + 60
    while len(out) < len(tickets):
        for t in tickets:
            if t not in out:
                r = S.result(t)
                if r is not None:
                    out[t] = r
        assert time.time() < deadline, "server did not complete the requests"
    return out


def test_alone_equals_mix(orc):
    """Each request's result is the same when served in a mix as when run
    alone through the plain call (the same kernels: bit-identical), and both
    match the oracle."""
    import torch
    import paper_2106_00124_amd as P
    from tests.gpu_util import torch_dtype
    items = _mix(21, 24)
    host = [make_input(s, dt, seed, op) for (s, b, dt, op, m, seed) in items]
    dev = [torch.from_numpy(np.ascontiguousarray(a)).cuda() for a in host]
    alone = []
    for (shape, box, dt, op, mode, seed), x in zip(items, dev):
        i, e = P.run(x, box, op, mode)
        torch.cuda.synchronize()
        alone.append((i.cpu().numpy() if i is not None else None,
                      e.cpu().numpy() if e is not None else None))
    say(f"[server] mix of {len(items)} requests, 4 streams")
    S = P.Server(hbm_budget=64 << 20, max_inflight=4)
    tickets = [S.submit(x, it[1], it[3], it[4]) for x, it in zip(dev, items)]
    res = _wait(S, tickets)
    for (shape, box, dt, op, mode, seed), a, t, (ai, ae) in zip(items, host, tickets, alone):
        inc, exc, lat = res[t]
        what = f"{shape} {box} {dt} {op} {mode}"
        assert lat > 0
        assert (inc is None) == (ai is None) and (exc is None) == (ae is None), what
        if inc is not None:
            assert inc.dtype == torch_dtype(dt) and tuple(inc.shape) == shape
            assert np.array_equal(inc.cpu().numpy(), ai), what
        if exc is not None:
            assert np.array_equal(exc.cpu().numpy(), ae), what
        ri, re_ = orc.brute(a, box, op, dt) if a.size <= 2048 else orc.scale(a, box, op, dt)
        si = se = None
        if dt == "f32" and op == "sum":
            si = tolerance.sigma_full(orc, a, box, "inc")
            se = tolerance.sigma_full(orc, a, box, "exc")
        if inc is not None:
            tolerance.check(inc.cpu().numpy(), ri, dt, op, si, what=what + " inc")
        if exc is not None:
            tolerance.check(exc.cpu().numpy(), re_, dt, op, se, what=what + " exc")
        S.release(t)
    st = S.stats()
    assert st["completed"] == len(items)
    assert st["p99_ms"] >= st["p50_ms"] > 0
    S.close()


def test_small_budget_queues_not_fails():
    """A budget that holds about two requests: later requests wait in the
    queue and complete once earlier ones are released."""
    import time
    import torch
    import paper_2106_00124_amd as P
    shape, box = (64, 64, 64), (8, 8, 8)
    x = torch.from_numpy(make_input(shape, "f32", 5, "sum")).cuda()
    ref_i, ref_e = P.run(x, box, "sum", "both")
    torch.cuda.synchronize()
    need = 2 * x.numel() * 4 + P.workspace_size(shape, box, torch.float32, "sum", "both")
    S = P.Server(hbm_budget=int(need * 2.5), max_inflight=4)
    tickets = [S.submit(x, box, "sum", "both") for _ in range(10)]
    done = 0
    deadline = time.time() + 60
    pending = list(tickets)
    while pending:
        assert time.time() < deadline
        t = pending[0]
        r = S.result(t)
        if r is None:
            continue
        inc, exc, _ = r
        assert torch.equal(inc, ref_i) and torch.equal(exc, ref_e)
        S.release(t)
        pending.pop(0)
        done += 1
    st = S.stats()
    assert done == 10 and st["completed"] == 10
    assert st["max_queue"] >= 5
    assert st["peak_bytes"] <= int(need * 2.5) + 4096
    S.close()


def test_bad_requests_rejected_loop_continues():
    import torch
    import paper_2106_00124_amd as P
    from paper_2106_00124_amd import ExsError
    S = P.Server(hbm_budget=8 << 20, max_inflight=2)
    x = torch.from_numpy(make_input((20, 30), "i32", 3, "sum")).cuda()
    with pytest.raises(ExsError, match="EINVAL"):
        S.submit(x, (21, 2), "sum", "exc")          # box longer than the axis
    with pytest.raises(ExsError, match="EINVAL"):
        S.submit(x, (0, 2), "sum", "exc")           # empty box
    big = torch.zeros((1024, 1024), dtype=torch.float32, device="cuda")
    with pytest.raises(ExsError, match="ENOMEM"):
        S.submit(big, (4, 4), "sum", "both")        # larger than the whole budget
    with pytest.raises(ExsError, match="EINVAL"):
        S.submit_generated((8, 8), (2, 2), torch.float64, "sum", "exc", kind=0, seed=1)
    t = S.submit(x, (4, 5), "sum", "exc")
    S.drain()
    _, exc, _ = S.result(t)
    _, ref = P.run(x, (4, 5), "sum", "exc")
    torch.cuda.synchronize()
    assert torch.equal(exc, ref)
    with pytest.raises(ExsError, match="ENOTFOUND"):
        S.result(t + 100)
    S.release(t)
    with pytest.raises(ExsError, match="ENOTFOUND"):
        S.release(t)
    S.close()


def test_drain_reports_blocked_queue():
    import torch
    import paper_2106_00124_amd as P
    from paper_2106_00124_amd import ExsError
    shape, box = (128, 128), (4, 4)
    x = torch.from_numpy(make_input(shape, "f32", 9, "sum")).cuda()
    need = x.numel() * 4 + P.workspace_size(shape, box, torch.float32, "sum", "exc")
    S = P.Server(hbm_budget=int(need * 1.5), max_inflight=2)
    t1 = S.submit(x, box, "sum", "exc")
    t2 = S.submit(x, box, "sum", "exc")
    with pytest.raises(ExsError, match="EAGAIN"):
        S.drain()                     # t1 done but unreleased: t2 cannot fit
    S.release(t1)
    S.drain()
    assert S.result(t2) is not None
    S.release(t2)
    S.close()


def test_generated_input_matches_host_twin(orc):
    """The server fills request tensors on the device; they equal the host
    twin of the generator and the results match the oracle on them."""
    import torch
    import paper_2106_00124_amd as P
    S = P.Server(hbm_budget=64 << 20, max_inflight=3)
    cases = [((40, 50, 30), (3, 7, 30), torch.float32, "sum", W.FILL_LOGMAG, 77, "f32"),
             ((200, 90), (64, 2), torch.float32, "max", W.FILL_LOGMAG, 78, "f32"),
             ((33, 17, 9), (5, 5, 5), torch.int32, "sum", W.FILL_UNIFORM_INT, 79, "i32")]
    tickets = [S.submit_generated(s, b, dt, op, "exc", kind=k, seed=sd, lo=-1000, hi=1000)
               for (s, b, dt, op, k, sd, _) in cases]
    S.drain()
    for (shape, box, dt, op, kind, seed, code), t in zip(cases, tickets):
        x = S.input(t).cpu().numpy()
        host = W.counter_fill(kind, code, int(np.prod(shape)), seed, -1000, 1000).reshape(shape)
        assert np.array_equal(x.view(np.uint8), host.view(np.uint8))
        _, exc, _ = S.result(t)
        _, ref = orc.scale(host, box, op, code)
        se = tolerance.sigma_full(orc, host, box, "exc") if code == "f32" and op == "sum" else None
        tolerance.check(exc.cpu().numpy(), ref, code, op, se, what=f"gen {shape} {box} {op}")
        S.release(t)
    S.close()


def test_input_on_caller_stream_and_clone_before_release(orc):
    """The request waits for the caller's stream that is still writing its
    input, and a clone of the result enqueued right before release (on the
    stream given to release) reads the finished result, not a range that a
    later request already reuses."""
    import torch
    import paper_2106_00124_amd as P
    shape, box = (96, 80, 72), (6, 5, 4)
    ref_host = make_input(shape, "f32", 31, "sum")
    src = torch.from_numpy(ref_host).cuda()
    torch.cuda.synchronize()
    side = torch.cuda.Stream()
    S = P.Server(hbm_budget=3 * (2 * src.numel() * 4 + P.workspace_size(
        shape, box, torch.float32, "sum", "exc")), max_inflight=2)
    clones = []
    tickets = []
    for rep in range(3):
        x = torch.empty_like(src)
        with torch.cuda.stream(side):
            x.fill_(float("nan"))
            torch.cuda._sleep(20_000_000)       # the input is written well after submit
            x.copy_(src)
        tickets.append(S.submit(x, box, "sum", "exc", stream=side))  # keeps x alive
    for t in tickets:
        while S.result(t) is None:
            pass
        _, exc, _ = S.result(t)
        clones.append(exc.clone())                  # enqueued on the current stream
        S.release(t)                                # range reused only after the clone
        # a later request may now take the range
        y = torch.from_numpy(make_input(shape, "f32", 32, "sum")).cuda()
        S.submit(y, box, "sum", "exc")
    S.drain()
    torch.cuda.synchronize()
    _, ref = orc.scale(ref_host, box, "sum", "f32")
    se = tolerance.sigma_full(orc, ref_host, box, "exc")
    for c in clones:
        tolerance.check(c.cpu().numpy(), ref, "f32", "sum", se, what="caller-stream clone")
    S.close()


def _c5_sample(reqs, count, seed):
    """Indices of a sample of the serving stream: its largest requests, those
    with the longest box sides, and uniform draws from the rest."""
    rng = np.random.default_rng(seed)
    by_n = sorted(range(len(reqs)), key=lambda i: -reqs[i].n)[:6]
    by_k = sorted(range(len(reqs)), key=lambda i: -max(reqs[i].box))[:6]
    chosen = list(dict.fromkeys(by_n + by_k))
    rest = [i for i in rng.permutation(len(reqs)) if i not in set(chosen)]
    chosen += [int(i) for i in rest[:count - len(chosen)]]
    return chosen


def _check_sampled(orc, host, box, op, dtype, pts, got, what):
    ref = orc.point_exc(host, box, op, dtype, pts)
    sig = tolerance.sigma_points(orc, host, box, "exc", pts) \
        if dtype == "f32" and op == "sum" else None
    return tolerance.check(got, ref, dtype, op, sig, what=what)


def test_serving_stream_sample_matches_oracle(orc):
    """200 requests of the stated serving stream (Poisson 2000 req/s for 60 s,
    rank 2-3, dims log-uniform in [32, 1024] up to 2^26 elements, box sides up
    to 64, + or max), including its largest requests and its longest boxes,
    served together; sampled cells of each result against the oracle on the
    input regenerated on the host from the request's seed."""
    import concurrent.futures as cf
    import torch
    import paper_2106_00124_amd as P
    reqs = W.serving_workload()
    idx = _c5_sample(reqs, 200, 606)
    sample = [reqs[i] for i in idx]
    assert max(r.n for r in sample) > (1 << 25)
    assert max(max(r.box) for r in sample) == 64
    say(f"[server] {len(sample)} requests of the serving stream, "
        f"{sum(r.n for r in sample) / 1e6:.0f} M elements")
    S = P.Server(hbm_budget=24 << 30, max_inflight=8)
    tickets = [S.submit_generated(r.shape, r.box, torch.float32, r.op, "exc",
                                  kind=W.FILL_LOGMAG, seed=r.fill_seed) for r in sample]
    got = {}
    pts_of = {}
    rng = np.random.default_rng(607)
    pending = list(zip(tickets, sample))
    while pending:
        t, r = pending[0]
        res = S.result(t)
        if res is None:
            continue
        pts = np.concatenate([rng.integers(0, r.n, 62), [0, r.n - 1]]).astype(np.int64)
        got[t] = res[1].reshape(-1)[torch.from_numpy(pts).cuda()].cpu().numpy()
        pts_of[t] = pts
        S.release(t)
        pending.pop(0)
    S.close()

    def one(tr):
        t, r = tr
        host = W.counter_fill(W.FILL_LOGMAG, "f32", r.n, r.fill_seed).reshape(r.shape)
        _check_sampled(orc, host, r.box, r.op, "f32", pts_of[t], got[t],
                       what=f"request {r.rid} {r.shape} {r.box} {r.op}")
        return r.n

    with cf.ThreadPoolExecutor(8) as ex:
        done = sum(ex.map(one, zip(tickets, sample)))
    say(f"[server] checked {len(sample)} requests ({done / 1e6:.0f} M elements)")
