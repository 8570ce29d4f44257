"""Pins that tie the CPU oracle to the paper and to mathematics, not to itself.

Each pin takes an ``oracle.Oracle`` and raises AssertionError on a mismatch, so
the same battery runs against the real oracle (``test_oracle.py``) and against
builds with a planted mistake (which must fail at least one pin).

Sources of truth used here (none of them calls the oracle twice to agree with
itself):
  * hand-derived values from the Definition of included/excluded sums (Sec. 2);
  * closed forms (all-ones and one-hot tensors);
  * textbook routines written independently in numpy: the summed-area table
    (Sec. 1, "Summed-area Table for Weak Excluded Sums") for +, a sliding
    window maximum (minimum) on an identity-padded array for max (min), numpy
    masks over the complement of each box for excluded sums;
  * invariants: with + on integers, included plus excluded equals the total;
    with max (min), the larger (smaller) of the two equals the global maximum
    (minimum); the 1-D
    excluded sum is prefix(x-1) op suffix(x+k); permuting axes permutes the
    result; k = n leaves an empty complement at the origin.
"""
from __future__ import annotations

import itertools
import os

import numpy as np
from numpy.lib.stride_tricks import sliding_window_view

I32_MIN = np.iinfo(np.int32).min
I64_MIN = np.iinfo(np.int64).min
I32_MAX = np.iinfo(np.int32).max
I64_MAX = np.iinfo(np.int64).max


# --------------------------------------------------------------------------
# hand-derived cases (from the Definition, Sec. 2)
# --------------------------------------------------------------------------

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def load_golden(name):
    """A hand-derived fixture of tests/golden/: shape, box, the input A and the
    expected included/excluded sums per operator (each file states its
    derivation and citation)."""
    out = {}
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.split("#", 1)[0].split()
            if not line:
                continue
            if line[0] in ("shape", "box"):
                out[line[0]] = [int(v) for v in line[1:]]
            elif line[0] == "A":
                out["A"] = np.array([int(v) for v in line[1:]], np.int64)
            else:
                out[(line[0], line[1])] = np.array([int(v) for v in line[2:]], np.int64)
    out["A"] = out["A"].reshape(out["shape"])
    for key in list(out):
        if isinstance(key, tuple):
            out[key] = out[key].reshape(out["shape"])
    return out


def pin_hand_1d(o):
    # A = 1..8, k = 4 (tests/golden/hand_1d_n8_k4.txt)
    g = load_golden("hand_1d_n8_k4.txt")
    a, k = g["A"], g["box"]
    for fn in ("brute", "scale"):
        for dt in ("i64", "i32", "f64", "f32"):
            for op in ("sum", "max", "min"):
                i, e = getattr(o, fn)(a, k, op, dt)
                assert np.array_equal(i, g[("inc", op)]) and np.array_equal(e, g[("exc", op)]), \
                    (fn, dt, op, i, e)
    pts = np.arange(a.size)
    for op in ("sum", "max", "min"):
        assert np.array_equal(o.point_inc(a, k, op, "i64", pts), g[("inc", op)]), op
        assert np.array_equal(o.point_exc(a, k, op, "i64", pts), g[("exc", op)]), op
        assert np.array_equal(o.point_exc_direct(a, k, op, "i64", pts), g[("exc", op)]), op


def pin_hand_2d(o):
    # 3 x 4 matrix 1..12, box (2, 2) (tests/golden/hand_2d_3x4_k2x2.txt)
    g = load_golden("hand_2d_3x4_k2x2.txt")
    a, k = g["A"], g["box"]
    for dt in ("i64", "f64"):
        for op in ("sum", "max", "min"):
            for fn in ("brute", "scale"):
                i, e = getattr(o, fn)(a, k, op, dt)
                assert np.array_equal(i, g[("inc", op)]) and np.array_equal(e, g[("exc", op)]), \
                    (fn, dt, op)
            assert np.array_equal(o.corners2d(a, k, op, dt), g[("exc", op)]), (dt, op)


# --------------------------------------------------------------------------
# closed forms
# --------------------------------------------------------------------------

CLOSED_SHAPES = [((7,), (3,)), ((5, 6), (2, 4)), ((4, 3, 5), (3, 1, 2)),
                 ((3, 4, 2, 3), (2, 4, 2, 1)), ((6, 5), (6, 5)), ((2, 3, 2, 2, 3), (1, 2, 2, 1, 3))]


def pin_closed_forms(o):
    for shape, k in CLOSED_SHAPES:
        n = np.array(shape)
        N = int(n.prod())
        grids = np.meshgrid(*[np.arange(s) for s in shape], indexing="ij")
        expect_inc = np.ones(shape, np.int64)
        for ax in range(len(shape)):
            expect_inc *= np.minimum(k[ax], shape[ax] - grids[ax])
        ones = np.ones(shape, np.int64)
        for fn in ("brute", "scale"):
            i, e = getattr(o, fn)(ones, k, "sum", "i64")
            assert np.array_equal(i, expect_inc), (fn, shape, k)
            assert np.array_equal(e, N - expect_inc), (fn, shape, k)
        # one-hot at p: included sum is 1 iff p lies in box(x)
        rng = np.random.default_rng(len(shape))
        p = tuple(int(rng.integers(0, s)) for s in shape)
        hot = np.zeros(shape, np.int64)
        hot[p] = 1
        in_box = np.ones(shape, bool)
        for ax in range(len(shape)):
            in_box &= (grids[ax] <= p[ax]) & (p[ax] < grids[ax] + k[ax])
        for fn in ("brute", "scale"):
            i, e = getattr(o, fn)(hot, k, "sum", "i64")
            assert np.array_equal(i, in_box.astype(np.int64)), (fn, shape, k, p)
            assert np.array_equal(e, 1 - in_box.astype(np.int64)), (fn, shape, k, p)
            # with max over {0, 1}, the same indicator
            i, e = getattr(o, fn)(hot, k, "max", "i64")
            if N > 1:
                assert np.array_equal(i, in_box.astype(np.int64)), (fn, "max", shape, k, p)


# --------------------------------------------------------------------------
# textbook routines, written independently in numpy
# --------------------------------------------------------------------------

def sat_included_sum(a, k):
    """Summed-area table (Crow): d-dim prefix sums plus inclusion-exclusion over
    the 2^d corners of each box.  Integers only (exact)."""
    a = np.asarray(a, dtype=np.int64)
    d = a.ndim
    S = np.zeros(tuple(s + 1 for s in a.shape), np.int64)
    S[tuple(slice(1, None) for _ in range(d))] = a
    for ax in range(d):
        S = np.cumsum(S, axis=ax)
    grids = np.meshgrid(*[np.arange(s) for s in a.shape], indexing="ij")
    out = np.zeros(a.shape, np.int64)
    for corner in itertools.product((0, 1), repeat=d):
        idx = []
        for ax in range(d):
            hi = np.minimum(grids[ax] + k[ax], a.shape[ax])
            idx.append(hi if corner[ax] else grids[ax])
        sign = (-1) ** (d - sum(corner))
        out += sign * S[tuple(idx)]
    return out


def window_max_included(a, k, ident, reduce=np.max):
    """Sliding-window maximum (or ``reduce``) over an identity-padded array."""
    a = np.asarray(a)
    pad = [(0, kk - 1) for kk in k]
    p = np.pad(a, pad, constant_values=ident)
    w = sliding_window_view(p, tuple(k))
    return reduce(w, axis=tuple(range(a.ndim, 2 * a.ndim)))


def masked_excluded(a, k, op, ident):
    """For each cell, reduce A over a boolean mask of the complement of its box."""
    a = np.asarray(a)
    grids = np.meshgrid(*[np.arange(s) for s in a.shape], indexing="ij")
    out = np.empty(a.shape, dtype=np.int64 if op == "sum" else a.dtype)
    for x in itertools.product(*[range(s) for s in a.shape]):
        inside = np.ones(a.shape, bool)
        for ax in range(a.ndim):
            inside &= (grids[ax] >= x[ax]) & (grids[ax] < x[ax] + k[ax])
        vals = a[~inside]
        if op == "sum":
            out[x] = vals.astype(np.int64).sum()
        elif op == "max":
            out[x] = vals.max() if vals.size else ident
        else:
            out[x] = vals.min() if vals.size else ident
    return out


TEXTBOOK_CASES = [((9,), (4,)), ((8, 5), (3, 2)), ((5, 4, 6), (2, 3, 4)),
                  ((4, 3, 3, 5), (3, 2, 1, 2)), ((10,), (10,)), ((3, 7), (3, 1))]


def pin_textbook(o):
    rng = np.random.default_rng(7)
    for shape, k in TEXTBOOK_CASES:
        a = rng.integers(-50, 51, size=shape).astype(np.int64)
        sat = sat_included_sum(a, k)
        tot = int(a.sum())
        for fn in ("brute", "scale"):
            i, e = getattr(o, fn)(a, k, "sum", "i64")
            assert np.array_equal(i, sat), (fn, shape, k)
            assert np.array_equal(e, tot - sat), (fn, shape, k)
        wm = window_max_included(a, k, I64_MIN)
        me = masked_excluded(a, k, "max", I64_MIN)
        for fn in ("brute", "scale"):
            i, e = getattr(o, fn)(a, k, "max", "i64")
            assert np.array_equal(i, wm), (fn, "max", shape, k)
            assert np.array_equal(e, me), (fn, "max", shape, k)
        wn = window_max_included(a, k, I64_MAX, np.min)
        mn = masked_excluded(a, k, "min", I64_MAX)
        for fn in ("brute", "scale"):
            i, e = getattr(o, fn)(a, k, "min", "i64")
            assert np.array_equal(i, wn), (fn, "min", shape, k)
            assert np.array_equal(e, mn), (fn, "min", shape, k)
        # floats: the window max is exact; the masked + is exact on integers
        af = a.astype(np.float64) / 4.0
        i, e = o.brute(af, k, "max", "f64")
        assert np.array_equal(i, window_max_included(af, k, -np.inf))
        assert np.array_equal(e, masked_excluded(af, k, "max", -np.inf))
        i, e = o.scale(af, k, "min", "f64")
        assert np.array_equal(i, window_max_included(af, k, np.inf, np.min))
        assert np.array_equal(e, masked_excluded(af, k, "min", np.inf))
        i, e = o.scale(af, k, "sum", "f64")
        assert np.array_equal(i, sat / 4.0) and np.array_equal(e, (tot - sat) / 4.0)


def pin_i32_wrap(o):
    # sums that overflow int32 wrap modulo 2^32 (numpy int32 arithmetic wraps)
    a = np.full((4, 5), 2_000_000_000, dtype=np.int64)
    a[1, 2] = -2_147_483_648
    k = (2, 3)
    sat64 = sat_included_sum(a, k)
    expect_inc = sat64.astype(np.int32).astype(np.int64)  # mod 2^32
    expect_exc = (int(a.sum()) - sat64).astype(np.int32).astype(np.int64)
    for fn in ("brute", "scale"):
        i, e = getattr(o, fn)(a, k, "sum", "i32")
        assert np.array_equal(i, expect_inc), fn
        assert np.array_equal(e, expect_exc), fn
    pts = np.arange(20)
    assert np.array_equal(o.point_inc(a, k, "sum", "i32", pts), expect_inc.reshape(-1))
    assert np.array_equal(o.point_exc(a, k, "sum", "i32", pts), expect_exc.reshape(-1))


# --------------------------------------------------------------------------
# invariants
# --------------------------------------------------------------------------

def pin_invariants(o):
    rng = np.random.default_rng(11)
    for shape, k in [((6, 7), (3, 2)), ((4, 5, 3), (2, 5, 2)), ((3, 3, 3, 3), (2, 1, 3, 2))]:
        a = rng.integers(-1000, 1001, size=shape).astype(np.int64)
        i, e = o.brute(a, k, "sum", "i64")
        assert np.all(i + e == a.sum())
        i, e = o.brute(a, k, "max", "i64")
        assert np.all(np.maximum(i, e) == a.max())
        i, e = o.scale(a, k, "min", "i64")
        assert np.all(np.minimum(i, e) == a.min())
        # permuting axes permutes the outputs
        perm = tuple(reversed(range(len(shape))))
        kp = tuple(k[p] for p in perm)
        ip, ep = o.brute(np.transpose(a, perm).copy(), kp, "sum", "i64")
        i, e = o.brute(a, k, "sum", "i64")
        assert np.array_equal(ip, np.transpose(i, perm)) and np.array_equal(ep, np.transpose(e, perm))
    # 1-D: excluded sum = prefix up to x-1 op suffix from x+k
    for n, kk in [(11, 3), (12, 4), (5, 5), (9, 1)]:
        a = rng.integers(-9, 10, size=n).astype(np.int64)
        pre = np.concatenate([[0], np.cumsum(a)])                 # pre[t] = sum a[:t]
        suf = np.concatenate([np.cumsum(a[::-1])[::-1], [0]])    # suf[t] = sum a[t:]
        x = np.arange(n)
        expect = pre[x] + suf[np.minimum(x + kk, n)]
        for fn in ("brute", "scale"):
            _, e = getattr(o, fn)(a, [kk], "sum", "i64")
            assert np.array_equal(e, expect), (fn, n, kk)
        premax = np.concatenate([[I64_MIN], np.maximum.accumulate(a)])
        sufmax = np.concatenate([np.maximum.accumulate(a[::-1])[::-1], [I64_MIN]])
        expect = np.maximum(premax[x], sufmax[np.minimum(x + kk, n)])
        for fn in ("brute", "scale"):
            _, e = getattr(o, fn)(a, [kk], "max", "i64")
            assert np.array_equal(e, expect), (fn, "max", n, kk)
        premin = np.concatenate([[I64_MAX], np.minimum.accumulate(a)])
        sufmin = np.concatenate([np.minimum.accumulate(a[::-1])[::-1], [I64_MAX]])
        expect = np.minimum(premin[x], sufmin[np.minimum(x + kk, n)])
        for fn in ("brute", "scale"):
            _, e = getattr(o, fn)(a, [kk], "min", "i64")
            assert np.array_equal(e, expect), (fn, "min", n, kk)
    # k = n: the box at the origin covers the tensor, so its complement is empty
    for dt, ident, ident_min in (("i32", I32_MIN, I32_MAX), ("i64", I64_MIN, I64_MAX),
                                 ("f64", -np.inf, np.inf)):
        a = rng.integers(-5, 6, size=(3, 4)).astype(np.float64 if dt == "f64" else np.int64)
        for fn in ("brute", "scale"):
            _, e = getattr(o, fn)(a, [3, 4], "max", dt)
            assert e[0, 0] == ident, (fn, dt, e[0, 0])
            _, e = getattr(o, fn)(a, [3, 4], "min", dt)
            assert e[0, 0] == ident_min, (fn, dt, e[0, 0])
            _, e = getattr(o, fn)(a, [3, 4], "sum", dt)
            assert e[0, 0] == 0, (fn, dt)
    # ... also for real-valued + on data whose two orders of summation differ
    # in rounding (total - included would leave a residue): exactly 0, by
    # every form, and 0 at the other cells only where the brute force says so
    a = rng.standard_normal((50, 90))
    _, eb = o.brute(a, [50, 90], "sum", "f64")
    _, es = o.scale(a, [50, 90], "sum", "f64")
    ep = o.point_exc(a, [50, 90], "sum", "f64", np.array([0, 1, 90]))
    assert eb[0, 0] == 0.0 and es[0, 0] == 0.0 and ep[0] == 0.0
    assert ep[1] != 0.0 and ep[2] != 0.0 and es[0, 1] != 0.0


# --------------------------------------------------------------------------
# the struct monoid: (value, index) pairs under argmax / argmin
# --------------------------------------------------------------------------

def brute_pairs_numpy(vals, idx, k, op):
    """Tiny-input brute force with numpy reductions: per cell, the best value
    over the masked region (box or complement), then the lowest index among
    the cells holding it."""
    n = vals.shape
    grids = np.meshgrid(*[np.arange(s) for s in n], indexing="ij")
    ident_v = -np.inf if op == "max" else np.inf
    best = np.max if op == "max" else np.min
    out = [np.empty(n), np.empty(n, np.int64), np.empty(n), np.empty(n, np.int64)]
    for x in itertools.product(*[range(s) for s in n]):
        inside = np.ones(n, bool)
        for j, g in enumerate(grids):
            inside &= (g >= x[j]) & (g < x[j] + k[j])
        for slot, mask in ((0, inside), (2, ~inside)):
            if not mask.any():
                out[slot][x], out[slot + 1][x] = ident_v, I32_MAX
                continue
            bv = best(vals[mask])
            out[slot][x] = bv
            out[slot + 1][x] = idx[mask & (vals == bv)].min()
    return out


def pin_pairs(o):
    # hand-derived 1-D case with ties (tests/golden/hand_vi_1d_n8_k4.txt)
    g = load_golden("hand_vi_1d_n8_k4.txt")
    vals, k = g["A"].astype(np.float64), g["box"]
    idx = np.arange(vals.size)
    for op in ("max", "min"):
        want = [g[("inc_value", op)], g[("inc_index", op)], g[("exc_value", op)],
                g[("exc_index", op)]]
        for fn in ("brute_vi", "scale_vi"):
            got = getattr(o, fn)(vals, idx, k, op)
            for a, b in zip(got, want):
                assert np.array_equal(a, b), (fn, op, got, want)
        pts = np.arange(vals.size)
        pv, pi = o.point_inc_vi(vals, idx, k, op, pts)
        ev, ei = o.point_exc_vi(vals, idx, k, op, pts)
        assert np.array_equal(pv, want[0]) and np.array_equal(pi, want[1]), op
        assert np.array_equal(ev, want[2]) and np.array_equal(ei, want[3]), op
    rng = np.random.default_rng(77)
    for shape, k in (((7,), (3,)), ((5, 6), (2, 4)), ((4, 3, 5), (2, 3, 2)),
                     ((3, 3, 2, 3), (2, 1, 2, 3))):
        # few distinct values (many ties), indices a permutation so that the
        # lowest index is not the first position
        vals = rng.integers(-2, 3, size=shape).astype(np.float64)
        idx = rng.permutation(vals.size).reshape(shape).astype(np.int64)
        for op in ("max", "min"):
            want = brute_pairs_numpy(vals, idx, k, op)
            for fn in ("brute_vi", "scale_vi"):
                got = getattr(o, fn)(vals, idx, k, op)
                for a, b in zip(got, want):
                    assert np.array_equal(a, b), (fn, op, shape, k)
            # the value part is the scalar max / min of the same regions
            si, se = o.scale(vals, k, op, "f64")
            got = o.scale_vi(vals, idx, k, op)
            assert np.array_equal(got[0], si) and np.array_equal(got[2], se), (op, shape)
            # the box and its complement cover the tensor: the better of the
            # two is the global argmax / argmin
            flat_v, flat_i = vals.reshape(-1), idx.reshape(-1)
            bv = flat_v.max() if op == "max" else flat_v.min()
            bi = flat_i[flat_v == bv].min()
            take_inc = (got[0] > got[2]) if op == "max" else (got[0] < got[2])
            tie = got[0] == got[2]
            comb_v = np.where(take_inc | tie, got[0], got[2])
            comb_i = np.where(take_inc, got[1], np.where(tie, np.minimum(got[1], got[3]), got[3]))
            assert np.all(comb_v == bv) and np.all(comb_i == bi), (op, shape)


ALL_PINS = [pin_hand_1d, pin_hand_2d, pin_closed_forms, pin_textbook, pin_i32_wrap, pin_invariants,
            pin_pairs]


def run_all(o):
    for pin in ALL_PINS:
        pin(o)
