"""Acceptance rules for comparing the GPU results with the oracle.

* Integer dtypes (wrapping +, max) and max on floats: bit-exact.
* f32 / f64 with +: elementwise, per cell,

      |got - ref| <= tol * max(|ref|, sigma)

  where ``ref`` is the FP64 oracle value and ``sigma = sqrt(sum of A[y]^2)``
  over the same region (the box for included sums, its complement for excluded
  sums): the natural magnitude of a random-sign sum over that region.  A pure
  relative test is not attainable for cells whose sum nearly cancels (any
  non-correctly-rounded f32 sum errs there by about eps * sigma), so the rule
  scales by whichever of |ref| and sigma is larger.  ``tol`` = 1e-5 for f32 and
  1e-12 for f64.
"""
from __future__ import annotations

import numpy as np

TOL = {"f32": 1e-5, "f64": 1e-12}


def sigma_full(orc, a, k, which):
    """sigma for every cell from the oracle on A^2 (FP64, op +)."""
    a2 = np.asarray(a, dtype=np.float64) ** 2
    inc2 = orc.scale_inc(a2, k, "sum", "f64")
    if which == "inc":
        return np.sqrt(np.maximum(inc2, 0.0))
    tot = float(a2.sum())
    return np.sqrt(np.maximum(tot - inc2, 0.0))


def sigma_points(orc, a, k, which, pts):
    a2 = np.asarray(a, dtype=np.float64) ** 2
    inc2 = orc.point_inc(a2, k, "sum", "f64", pts)
    if which == "inc":
        return np.sqrt(np.maximum(inc2, 0.0))
    tot = float(a2.sum())
    return np.sqrt(np.maximum(tot - inc2, 0.0))


def check(got, ref, dtype, op, sigma=None, tol=None, what=""):
    """Assert acceptance; returns a dict of error statistics."""
    got = np.asarray(got)
    ref = np.asarray(ref)
    assert got.shape == ref.shape, (got.shape, ref.shape)
    if dtype in ("i32", "i64") or op in ("max", "min"):
        if dtype in ("i32", "i64"):
            g = got.astype(np.int64)
            bad = np.nonzero(g != ref.astype(np.int64))[0] if g.ndim == 1 else \
                np.argwhere(g != ref.astype(np.int64))
        else:
            g = got.astype(np.float64)
            bad = np.nonzero(g != ref)[0] if g.ndim == 1 else np.argwhere(g != ref)
        assert len(bad) == 0, f"{what}: {len(bad)} mismatches, first at {bad[:5].tolist()}"
        return {"mismatches": 0}
    tol = TOL[dtype] if tol is None else tol
    g = got.astype(np.float64)
    err = np.abs(g - ref)
    scale = np.abs(ref) if sigma is None else np.maximum(np.abs(ref), sigma)
    scale = np.maximum(scale, np.finfo(np.float64).tiny)
    ratio = err / scale
    worst = float(ratio.max()) if ratio.size else 0.0
    stats = {"max_scaled_err": worst,
             "normwise": float(err.max() / max(np.abs(ref).max(), 1e-300)) if ref.size else 0.0}
    assert worst <= tol, f"{what}: max scaled error {worst:.3e} > {tol:.1e} ({stats})"
    return stats
