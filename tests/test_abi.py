"""The C-ABI library loads, exports every declared symbol, and validates jobs
on the host (no GPU needed: no call here launches work)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "exsum.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(exs_[a-z_0-9]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ("exs_workspace_size", "exs_run", "exs_status_str", "exs_last_error",
                 "exs_batch_create", "exs_batch_launch", "exs_server_create",
                 "exs_server_submit", "exs_server_poll", "exs_server_stats"):
        assert must in names


def test_library_exports_every_declared_symbol():
    from paper_2106_00124_amd import _lib
    h = ctypes.CDLL(_lib.LIB_PATH)
    missing = [n for n in declared_functions() if not hasattr(h, n)]
    assert not missing, missing
    assert set(declared_functions()) == set(_lib.SIGNATURES), \
        set(declared_functions()) ^ set(_lib.SIGNATURES)


def test_status_strings():
    from paper_2106_00124_amd import _lib
    L = _lib.lib()
    for code, name in _lib.STATUS.items():
        assert L.exs_status_str(code).decode() == name


def _ws(shape, box, dtype=0, op=0, mode=3):
    from paper_2106_00124_amd import _lib
    j = _lib.make_job(len(shape), dtype, op, mode, shape, box, None, None, None)
    n = ctypes.c_size_t()
    st = _lib.lib().exs_workspace_size(ctypes.byref(j), ctypes.byref(n))
    return st, n.value


@pytest.mark.parametrize("shape,box,dtype,op,mode", [
    ((4, 4), (0, 1), 0, 0, 3),       # k < 1
    ((4, 4), (5, 1), 0, 0, 3),       # k > n
    ((0, 4), (1, 1), 0, 0, 3),       # empty axis
    ((4, 4), (1, 1), 9, 0, 3),       # bad dtype
    ((4, 4), (1, 1), 0, 7, 3),       # bad op
    ((4, 4), (1, 1), 0, 0, 0),       # no output
    ((4, 4), (1, 1), 0, 0, 4),       # unknown mode bit
])
def test_invalid_jobs_rejected(shape, box, dtype, op, mode):
    st, _ = _ws(shape, box, dtype, op, mode)
    assert st == 1  # EXS_EINVAL


def test_rank_limits():
    from paper_2106_00124_amd import _lib
    j = _lib.make_job(1, 0, 0, 3, [4], [2], None, None, None)
    j.d = 9
    n = ctypes.c_size_t()
    assert _lib.lib().exs_workspace_size(ctypes.byref(j), ctypes.byref(n)) == 1
    j.d = 0
    assert _lib.lib().exs_workspace_size(ctypes.byref(j), ctypes.byref(n)) == 1


def test_workspace_sizes_sane():
    st, inc_only = _ws((512, 512, 512), (16, 16, 16), 0, 0, 1)
    assert st == 0
    st, both = _ws((512, 512, 512), (16, 16, 16), 0, 0, 3)
    assert st == 0 and both >= inc_only
    st, one_d = _ws((100,), (7,), 3, 1, 3)
    assert st == 0 and one_d > 0
    for d in range(1, 9):
        st, n = _ws((3,) * d, (2,) * d, 2, 0, 3)
        assert st == 0


def test_workspace_sizes_random_jobs():
    """The planner's sizing pass (the same code path as the launches, with
    nothing launched) over random valid jobs: every rank, dtype, operator and
    mode, boxes from 1 to the full extent, shapes from tiny to 2^33 elements,
    so that every special path (fused levels, tail scan, chunked 1-D levels,
    staged trailing axes, segmented block scans) is planned somewhere."""
    import numpy as np
    rng = np.random.default_rng(2024)
    planned = 0
    for _ in range(3000):
        d = int(rng.integers(1, 9))
        shape = [int(v) + 1 for v in np.exp(rng.uniform(0, np.log(700), d)).astype(int)]
        if np.prod(shape, dtype=np.float64) > 2.0 ** 33:
            continue
        box = [int(rng.integers(1, n + 1)) if rng.random() < 0.6 else min(n, int(rng.integers(1, 17)))
               for n in shape]
        dtype, op = int(rng.integers(0, 4)), int(rng.integers(0, 3))
        mode = [1, 2, 3, 6, 7][int(rng.integers(0, 5))]
        if mode & 4 and op != 0:
            mode = 3
        st, n = _ws(shape, box, dtype, op, mode)
        assert st == 0, (shape, box, dtype, op, mode)
        planned += 1
    assert planned > 2000


def test_run_rejects_null_and_aliasing_on_host():
    """Argument checks happen before anything touches the device."""
    from paper_2106_00124_amd import _lib
    L = _lib.lib()
    j = _lib.make_job(2, 0, 0, 3, [8, 8], [2, 2], 0x1000, None, 0x9000)
    assert L.exs_run(ctypes.byref(j), None, 0, None) == 1          # inc_out NULL
    j = _lib.make_job(2, 0, 0, 2, [8, 8], [2, 2], 0x1000, None, 0x1080)
    assert L.exs_run(ctypes.byref(j), None, 0, None) == 1          # overlaps input
    assert b"overlaps" in L.exs_last_error()
    # (a shape past the one-workgroup rank-2 kernel, which needs no workspace)
    j = _lib.make_job(2, 0, 0, 2, [300, 300], [2, 2], 0x1000, None, 0x100000)
    assert L.exs_run(ctypes.byref(j), None, 0, None) == 3          # workspace too small
    j = _lib.make_job(2, 0, 0, 2, [8, 8], [2, 2], 0x1002, None, 0x9000)
    assert L.exs_run(ctypes.byref(j), None, 0, None) == 1          # misaligned input
    assert b"aligned" in L.exs_last_error()


def test_weak_mode_validation():
    """Weak excluded sums: + only, and only together with the excluded output."""
    from paper_2106_00124_amd import _lib
    L = _lib.lib()
    n = ctypes.c_size_t()
    j = _lib.make_job(2, _lib.F32, _lib.SUM, _lib.EXCLUDED | _lib.WEAK, [8, 9], [2, 3],
                      None, None, None)
    assert L.exs_workspace_size(ctypes.byref(j), ctypes.byref(n)) == 0
    j = _lib.make_job(2, _lib.F32, _lib.MAX, _lib.EXCLUDED | _lib.WEAK, [8, 9], [2, 3],
                      None, None, None)
    assert L.exs_workspace_size(ctypes.byref(j), ctypes.byref(n)) == _lib.EUNSUPPORTED
    j = _lib.make_job(2, _lib.I32, _lib.SUM, _lib.INCLUDED | _lib.WEAK, [8, 9], [2, 3],
                      None, None, None)
    assert L.exs_workspace_size(ctypes.byref(j), ctypes.byref(n)) == _lib.EINVAL


def test_pair_dtype_validation():
    """(value, index) pairs: max and min plan like the 8-byte types; + and
    weak sums are refused, and the batched form refuses pairs, all on the host."""
    from paper_2106_00124_amd import _lib
    L = _lib.lib()
    n = ctypes.c_size_t()
    for op in (_lib.MAX, _lib.MIN):
        for d in range(1, 9):
            j = _lib.make_job(d, _lib.VALIDX, op, _lib.INCLUDED | _lib.EXCLUDED, [5] * d,
                              [3] * d, None, None, None)
            assert L.exs_workspace_size(ctypes.byref(j), ctypes.byref(n)) == 0
    j = _lib.make_job(2, _lib.VALIDX, _lib.SUM, _lib.EXCLUDED, [8, 9], [2, 3], None, None, None)
    assert L.exs_workspace_size(ctypes.byref(j), ctypes.byref(n)) == _lib.EUNSUPPORTED
    j = _lib.make_job(2, _lib.VALIDX, _lib.MAX, _lib.EXCLUDED | _lib.WEAK, [8, 9], [2, 3],
                      None, None, None)
    assert L.exs_workspace_size(ctypes.byref(j), ctypes.byref(n)) == _lib.EUNSUPPORTED
    jobs = (_lib.ExsJob * 1)()
    jobs[0] = _lib.make_job(2, _lib.VALIDX, _lib.MAX, _lib.EXCLUDED, [8, 9], [2, 3], 0x1000,
                            None, 0x9000)
    h = ctypes.c_void_p()
    assert L.exs_batch_create(jobs, 1, None, ctypes.byref(h)) == _lib.EUNSUPPORTED


def test_corners_validation_and_workspace():
    """The corners entry points: d = 2 and EXS_EXCLUDED only, no pairs; the
    workspace is four n0 x n1 tables and six ceil(n0/64) x n1 arrays, each
    rounded up to 256 bytes (host only)."""
    from paper_2106_00124_amd import _lib
    L = _lib.lib()
    n = ctypes.c_size_t()

    def ws(d, dims, box, dtype=_lib.F32, op=_lib.SUM, mode=_lib.EXCLUDED):
        j = _lib.make_job(d, dtype, op, mode, dims, box, None, None, None)
        return L.exs_corners_workspace_size(ctypes.byref(j), ctypes.byref(n))

    up = lambda b: (b + 255) // 256 * 256  # noqa: E731
    for (n0, n1), es, dt in (((64, 64), 4, _lib.F32), ((130, 77), 8, _lib.I64),
                             ((1, 1), 4, _lib.I32), ((1000, 3), 8, _lib.F64)):
        for op in (_lib.SUM, _lib.MAX, _lib.MIN):
            assert ws(2, [n0, n1], [1, 1], dt, op) == 0
            S = (n0 + 63) // 64
            assert n.value == 4 * up(n0 * n1 * es) + 6 * up(S * n1 * es)
    assert ws(3, [4, 4, 4], [2, 2, 2]) == _lib.EUNSUPPORTED
    assert ws(1, [8], [2]) == _lib.EUNSUPPORTED
    assert ws(2, [8, 8], [2, 2], mode=_lib.INCLUDED) == _lib.EINVAL
    assert ws(2, [8, 8], [2, 2], mode=_lib.INCLUDED | _lib.EXCLUDED) == _lib.EINVAL
    assert ws(2, [8, 8], [2, 2], mode=_lib.EXCLUDED | _lib.WEAK) == _lib.EINVAL
    assert ws(2, [8, 8], [9, 2]) == _lib.EINVAL
    assert ws(2, [8, 8], [2, 2], dtype=_lib.VALIDX, op=_lib.MAX) == _lib.EUNSUPPORTED
    # run: null pointers and a workspace over the input are refused on the host
    j = _lib.make_job(2, _lib.F32, _lib.SUM, _lib.EXCLUDED, [8, 8], [2, 2], None, None, None)
    assert L.exs_run_corners(ctypes.byref(j), None, 0, None) == _lib.EINVAL
    j = _lib.make_job(2, _lib.F32, _lib.SUM, _lib.EXCLUDED, [8, 8], [2, 2], 0x10000, None,
                      0x20000)
    assert ws(2, [8, 8], [2, 2]) == 0
    assert L.exs_run_corners(ctypes.byref(j), ctypes.c_void_p(0x10000), n.value,
                             None) == _lib.EINVAL
    assert L.exs_run_corners(ctypes.byref(j), ctypes.c_void_p(0x40000), 16,
                             None) == _lib.ENOMEM
