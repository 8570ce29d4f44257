"""CPU oracle for multidimensional included and excluded sums (test infrastructure).

TEST INFRASTRUCTURE ONLY: the plain, slow, obviously correct reference that the
GPU library is checked against.  Only ``tests/``, ``__graft_entry__.smoke()`` and
the CPU-baseline leg of ``bench.py`` may import this package.  The GPU library
(``paper_2106_00124_amd``) never imports it, and it imports nothing from there.

Paper: Xu, Fraser, Leiserson, "Multidimensional Included and Excluded Sums"
(SIAM ACDA 2021, arXiv 2106.00124).  The arithmetic lives in ``exsum_oracle.c``;
this module only builds it, marshals numpy arrays and widens dtypes:

* floating dtypes ("f32", "f64") are evaluated in float64 (the FP64 reference
  for f32 inputs; ``max`` and ``min`` are exact);
* integer dtypes ("i32", "i64") are evaluated in int64 with wrapping ``+``; an
  "i32" ``+`` result is reduced modulo 2**32 (returned sign-extended in int64).

Every function takes a row-major numpy array ``a`` of any rank 1..8, a box
``k`` (sequence of ints, 1 <= k_i <= n_i), ``op`` in {"sum", "max", "min"} and the
element ``dtype`` the GPU computes in, and returns float64 or int64 arrays.

Functions (their sources are cited in ``exsum_oracle.c``):

* ``brute``       -- O1, the Definition of included/excluded sums (Sec. 2), O(N^2).
* ``scale_inc``   -- O2, nested window reductions (Sec. 2 reduction over a subtensor).
* ``scale_exc``   -- O2, total minus included for ``+``; half-space cover for ``max``
  and ``min``.
* ``point_inc`` / ``point_exc`` / ``point_exc_direct`` -- one output at a time.
* ``corners2d``   -- O3, 2-D corners cross-check (Sec. 1 / App. A idea).
* ``brute_vi`` / ``scale_vi`` / ``point_inc_vi`` / ``point_exc_vi`` -- the
  same for a struct element: (value, index) pairs under "argmax" (``op``
  "max": the largest value, the lowest index among equal values) or "argmin"
  ("min"); values are f32 widened to float64, indices int32 widened to int64.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "exsum_oracle.c")
_LIB_DEFAULT = os.path.join(_HERE, "liboracle.so")

_DT = {"f32": 0, "f64": 1, "i32": 2, "i64": 3}
_OP = {"sum": 0, "max": 1, "min": 2}

_libs: dict = {}


def build(mutant: int = 0, out: str | None = None) -> str:
    """Compile the oracle with gcc (OpenMP).  ``mutant`` plants a known mistake."""
    out = out or (_LIB_DEFAULT if mutant == 0 else
                  os.path.join(_HERE, f"liboracle_mutant{mutant}.so"))
    cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared",
           f"-DORC_MUTANT={int(mutant)}", _SRC, "-o", out + ".tmp", "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(out + ".tmp", out)
    return out


def _bind(lib):
    P = ctypes.c_void_p
    I = ctypes.c_int
    L = ctypes.c_int64
    sigs = {
        "orc_brute_f64": [I, P, P, I, P, P, P],
        "orc_brute_i64": [I, P, P, I, I, P, P, P],
        "orc_scale_inc_f64": [I, P, P, I, P, P],
        "orc_scale_inc_i64": [I, P, P, I, I, P, P],
        "orc_scale_exc_f64": [I, P, P, I, P, P, P],
        "orc_scale_exc_i64": [I, P, P, I, I, P, P, P],
        "orc_point_inc_f64": [I, P, P, I, P, L, P, P],
        "orc_point_inc_i64": [I, P, P, I, I, P, L, P, P],
        "orc_point_exc_direct_f64": [I, P, P, I, P, L, P, P],
        "orc_point_exc_direct_i64": [I, P, P, I, I, P, L, P, P],
        "orc_point_exc_cover_f64": [I, P, P, I, P, L, P, P],
        "orc_point_exc_cover_i64": [I, P, P, I, I, P, L, P, P],
        "orc_corners2d_f64": [L, L, L, L, I, P, P],
        "orc_corners2d_i64": [L, L, L, L, I, I, P, P],
    }
    for name, args in sigs.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = ctypes.c_int
    lib.orc_total_f64.argtypes = [L, I, P]
    lib.orc_total_f64.restype = ctypes.c_double
    lib.orc_total_i64.argtypes = [L, I, I, P]
    lib.orc_total_i64.restype = ctypes.c_int64
    vi = {
        "orc_brute_vi": [I, P, P, I, P, P, P, P, P, P],
        "orc_scale_inc_vi": [I, P, P, I, P, P, P, P],
        "orc_exc_cover_vi": [I, P, P, I, P, P, L, P, P, P],
        "orc_point_inc_vi": [I, P, P, I, P, P, L, P, P, P],
    }
    for name, args in vi.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = ctypes.c_int
    lib.orc_num_threads.argtypes = []
    lib.orc_num_threads.restype = ctypes.c_int
    return lib


def load(path: str | None = None):
    """Load the compiled oracle (building it only if it is not there)."""
    path = path or _LIB_DEFAULT
    if path in _libs:
        return _libs[path]
    if not os.path.exists(path):
        if path != _LIB_DEFAULT:
            raise FileNotFoundError(path)
        build()
    lib = _bind(ctypes.CDLL(path))
    _libs[path] = lib
    return lib


class Oracle:
    """Bound view of one compiled oracle library (the default, or a mutant)."""

    def __init__(self, path: str | None = None):
        self.lib = load(path)

    # -- helpers ---------------------------------------------------------
    @staticmethod
    def _prep(a, k, op, dtype):
        if dtype not in _DT:
            raise ValueError(f"dtype {dtype!r}")
        if op not in _OP:
            raise ValueError(f"op {op!r}")
        a = np.asarray(a)
        d = a.ndim
        if not 1 <= d <= 8:
            raise ValueError("rank must be 1..8")
        k = [int(v) for v in k]
        if len(k) != d:
            raise ValueError("box rank must equal tensor rank")
        n = np.ascontiguousarray(a.shape, dtype=np.int64)
        kk = np.ascontiguousarray(k, dtype=np.int64)
        if dtype in ("f32", "f64"):
            w = np.ascontiguousarray(a, dtype=np.float64)
        else:
            w = np.ascontiguousarray(a, dtype=np.int64)
        return d, n, kk, w

    @staticmethod
    def _p(x):
        return x.ctypes.data_as(ctypes.c_void_p)

    def _check(self, rc, name):
        if rc != 0:
            raise ValueError(f"{name} rejected its arguments (rc={rc})")

    # -- O1 ----------------------------------------------------------------
    def brute(self, a, k, op, dtype):
        d, n, kk, w = self._prep(a, k, op, dtype)
        inc = np.empty(w.shape, w.dtype)
        exc = np.empty(w.shape, w.dtype)
        p = self._p
        if w.dtype == np.float64:
            rc = self.lib.orc_brute_f64(d, p(n), p(kk), _OP[op], p(w), p(inc), p(exc))
        else:
            rc = self.lib.orc_brute_i64(d, p(n), p(kk), _OP[op], _DT[dtype], p(w), p(inc), p(exc))
        self._check(rc, "brute")
        return inc, exc

    # -- O2 ----------------------------------------------------------------
    def scale_inc(self, a, k, op, dtype):
        d, n, kk, w = self._prep(a, k, op, dtype)
        inc = np.empty(w.shape, w.dtype)
        p = self._p
        if w.dtype == np.float64:
            rc = self.lib.orc_scale_inc_f64(d, p(n), p(kk), _OP[op], p(w), p(inc))
        else:
            rc = self.lib.orc_scale_inc_i64(d, p(n), p(kk), _OP[op], _DT[dtype], p(w), p(inc))
        self._check(rc, "scale_inc")
        return inc

    def scale_exc(self, a, k, op, dtype, inc=None):
        """Excluded sums; for ``sum`` the included sums are needed (computed if absent)."""
        d, n, kk, w = self._prep(a, k, op, dtype)
        if op == "sum" and inc is None:
            inc = self.scale_inc(a, k, op, dtype)
        if inc is None:
            inc = np.zeros(w.shape, w.dtype)
        inc = np.ascontiguousarray(inc, dtype=w.dtype)
        exc = np.empty(w.shape, w.dtype)
        p = self._p
        if w.dtype == np.float64:
            rc = self.lib.orc_scale_exc_f64(d, p(n), p(kk), _OP[op], p(w), p(inc), p(exc))
        else:
            rc = self.lib.orc_scale_exc_i64(d, p(n), p(kk), _OP[op], _DT[dtype], p(w), p(inc), p(exc))
        self._check(rc, "scale_exc")
        return exc

    def scale(self, a, k, op, dtype):
        inc = self.scale_inc(a, k, op, dtype)
        return inc, self.scale_exc(a, k, op, dtype, inc)

    # -- point oracles -----------------------------------------------------
    def point_inc(self, a, k, op, dtype, pts):
        d, n, kk, w = self._prep(a, k, op, dtype)
        pts = np.ascontiguousarray(pts, dtype=np.int64)
        out = np.empty(pts.shape[0], w.dtype)
        p = self._p
        if w.dtype == np.float64:
            rc = self.lib.orc_point_inc_f64(d, p(n), p(kk), _OP[op], p(w), pts.shape[0], p(pts), p(out))
        else:
            rc = self.lib.orc_point_inc_i64(d, p(n), p(kk), _OP[op], _DT[dtype], p(w),
                                            pts.shape[0], p(pts), p(out))
        self._check(rc, "point_inc")
        return out

    def point_exc_direct(self, a, k, op, dtype, pts):
        d, n, kk, w = self._prep(a, k, op, dtype)
        pts = np.ascontiguousarray(pts, dtype=np.int64)
        out = np.empty(pts.shape[0], w.dtype)
        p = self._p
        if w.dtype == np.float64:
            rc = self.lib.orc_point_exc_direct_f64(d, p(n), p(kk), _OP[op], p(w),
                                                   pts.shape[0], p(pts), p(out))
        else:
            rc = self.lib.orc_point_exc_direct_i64(d, p(n), p(kk), _OP[op], _DT[dtype], p(w),
                                                   pts.shape[0], p(pts), p(out))
        self._check(rc, "point_exc_direct")
        return out

    def point_exc(self, a, k, op, dtype, pts):
        """Excluded sums at ``pts``: total minus included for ``sum``, the
        half-space cover for ``max`` and ``min``."""
        d, n, kk, w = self._prep(a, k, op, dtype)
        pts = np.ascontiguousarray(pts, dtype=np.int64)
        p = self._p
        if op != "sum":
            out = np.empty(pts.shape[0], w.dtype)
            if w.dtype == np.float64:
                rc = self.lib.orc_point_exc_cover_f64(d, p(n), p(kk), _OP[op], p(w),
                                                      pts.shape[0], p(pts), p(out))
            else:
                rc = self.lib.orc_point_exc_cover_i64(d, p(n), p(kk), _OP[op], _DT[dtype], p(w),
                                                      pts.shape[0], p(pts), p(out))
            self._check(rc, "point_exc_cover")
            return out
        inc = self.point_inc(a, k, op, dtype, pts)
        if w.dtype == np.float64:
            total = self.lib.orc_total_f64(w.size, 0, p(w))
            out = total - inc
            # k = n on every axis: the origin's complement is empty, its sum
            # exactly the identity (Sec. 2), not total - inc's rounding residue
            if np.array_equal(kk, n):
                out[pts == 0] = 0.0
            return out
        total = np.uint64(np.int64(self.lib.orc_total_i64(w.size, 0, 3, p(w))).view(np.uint64))
        out = (total - inc.view(np.uint64)).view(np.int64)
        if dtype == "i32":
            out = out.astype(np.int32).astype(np.int64)
        return out

    def num_threads(self) -> int:
        """OpenMP threads the oracle's parallel loops use."""
        return int(self.lib.orc_num_threads())

    def total(self, a, op, dtype):
        a = np.asarray(a)
        p = self._p
        if dtype in ("f32", "f64"):
            w = np.ascontiguousarray(a, dtype=np.float64).reshape(-1)
            return self.lib.orc_total_f64(w.size, _OP[op], p(w))
        w = np.ascontiguousarray(a, dtype=np.int64).reshape(-1)
        return self.lib.orc_total_i64(w.size, _OP[op], _DT[dtype], p(w))

    # -- (value, index) pairs ---------------------------------------------
    @staticmethod
    def _prep_vi(values, index, k, op):
        if op not in ("max", "min"):
            raise ValueError("pairs take op 'max' (argmax) or 'min' (argmin)")
        v = np.ascontiguousarray(values, dtype=np.float64)
        i = np.ascontiguousarray(index, dtype=np.int64)
        if v.shape != i.shape:
            raise ValueError("values and index must have the same shape")
        d = v.ndim
        k = [int(t) for t in k]
        if not 1 <= d <= 8 or len(k) != d:
            raise ValueError("rank 1..8 and a box of the same rank")
        n = np.ascontiguousarray(v.shape, dtype=np.int64)
        return d, n, np.ascontiguousarray(k, dtype=np.int64), v, i

    def brute_vi(self, values, index, k, op):
        """O1 for pairs: (inc_values, inc_index, exc_values, exc_index)."""
        d, n, kk, v, i = self._prep_vi(values, index, k, op)
        out = [np.empty(v.shape, np.float64), np.empty(v.shape, np.int64),
               np.empty(v.shape, np.float64), np.empty(v.shape, np.int64)]
        p = self._p
        self._check(self.lib.orc_brute_vi(d, p(n), p(kk), _OP[op], p(v), p(i), *map(p, out)),
                    "brute_vi")
        return tuple(out)

    def scale_vi(self, values, index, k, op):
        """O2 for pairs: nested windows (included), half-space cover (excluded)."""
        d, n, kk, v, i = self._prep_vi(values, index, k, op)
        out = [np.empty(v.shape, np.float64), np.empty(v.shape, np.int64),
               np.empty(v.shape, np.float64), np.empty(v.shape, np.int64)]
        p = self._p
        self._check(self.lib.orc_scale_inc_vi(d, p(n), p(kk), _OP[op], p(v), p(i), p(out[0]),
                                              p(out[1])), "scale_inc_vi")
        self._check(self.lib.orc_exc_cover_vi(d, p(n), p(kk), _OP[op], p(v), p(i), 0, None,
                                              p(out[2]), p(out[3])), "exc_cover_vi")
        return tuple(out)

    def point_inc_vi(self, values, index, k, op, pts):
        d, n, kk, v, i = self._prep_vi(values, index, k, op)
        pts = np.ascontiguousarray(pts, dtype=np.int64)
        ov, oi = np.empty(pts.shape[0], np.float64), np.empty(pts.shape[0], np.int64)
        p = self._p
        self._check(self.lib.orc_point_inc_vi(d, p(n), p(kk), _OP[op], p(v), p(i), pts.shape[0],
                                              p(pts), p(ov), p(oi)), "point_inc_vi")
        return ov, oi

    def point_exc_vi(self, values, index, k, op, pts):
        d, n, kk, v, i = self._prep_vi(values, index, k, op)
        pts = np.ascontiguousarray(pts, dtype=np.int64)
        ov, oi = np.empty(pts.shape[0], np.float64), np.empty(pts.shape[0], np.int64)
        p = self._p
        self._check(self.lib.orc_exc_cover_vi(d, p(n), p(kk), _OP[op], p(v), p(i), pts.shape[0],
                                              p(pts), p(ov), p(oi)), "exc_cover_vi")
        return ov, oi

    # -- O3 ----------------------------------------------------------------
    def corners2d(self, a, k, op, dtype):
        d, n, kk, w = self._prep(a, k, op, dtype)
        if d != 2:
            raise ValueError("corners2d is 2-D only")
        exc = np.empty(w.shape, w.dtype)
        p = self._p
        if w.dtype == np.float64:
            rc = self.lib.orc_corners2d_f64(int(n[0]), int(n[1]), int(kk[0]), int(kk[1]),
                                            _OP[op], p(w), p(exc))
        else:
            rc = self.lib.orc_corners2d_i64(int(n[0]), int(n[1]), int(kk[0]), int(kk[1]),
                                            _OP[op], _DT[dtype], p(w), p(exc))
        self._check(rc, "corners2d")
        return exc


_default: Oracle | None = None


def default() -> Oracle:
    global _default
    if _default is None:
        _default = Oracle()
    return _default


def brute(a, k, op, dtype):
    return default().brute(a, k, op, dtype)


def scale(a, k, op, dtype):
    return default().scale(a, k, op, dtype)


def scale_inc(a, k, op, dtype):
    return default().scale_inc(a, k, op, dtype)


def scale_exc(a, k, op, dtype, inc=None):
    return default().scale_exc(a, k, op, dtype, inc)


def point_inc(a, k, op, dtype, pts):
    return default().point_inc(a, k, op, dtype, pts)


def point_exc(a, k, op, dtype, pts):
    return default().point_exc(a, k, op, dtype, pts)


def point_exc_direct(a, k, op, dtype, pts):
    return default().point_exc_direct(a, k, op, dtype, pts)


def corners2d(a, k, op, dtype):
    return default().corners2d(a, k, op, dtype)


def total(a, op, dtype):
    return default().total(a, op, dtype)
