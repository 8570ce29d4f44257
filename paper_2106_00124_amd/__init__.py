"""MI355X-native multidimensional included and excluded sums (HIP for gfx950).

Paper: Xu, Fraser, Leiserson, "Multidimensional Included and Excluded Sums"
(SIAM ACDA 2021, arXiv 2106.00124).

Python binding of ``libexsum.so`` (C ABI in ``include/exsum.h``).  PyTorch is
used only for device memory and streams; every step of the computation runs
in the library's HIP kernels.  Nothing here computes on the host.

    inc, exc = run(x, box, op="sum", mode="both")
"""
from __future__ import annotations

import ctypes

from . import _lib
from ._lib import ExsError  # noqa: F401

_DTYPES = None


def _dtype_code(t):
    import torch
    global _DTYPES
    if _DTYPES is None:
        _DTYPES = {torch.float32: _lib.F32, torch.float64: _lib.F64,
                   torch.int32: _lib.I32, torch.int64: _lib.I64}
    try:
        return _DTYPES[t]
    except KeyError:
        raise ExsError(1, f"unsupported dtype {t}") from None


_OPS = {"sum": _lib.SUM, "+": _lib.SUM, "max": _lib.MAX, "min": _lib.MIN}
_MODES = {"inc": _lib.INCLUDED, "included": _lib.INCLUDED, "exc": _lib.EXCLUDED,
          "excluded": _lib.EXCLUDED, "both": _lib.INCLUDED | _lib.EXCLUDED,
          # weak excluded sums (total - included), + only
          "weak": _lib.EXCLUDED | _lib.WEAK,
          "both_weak": _lib.INCLUDED | _lib.EXCLUDED | _lib.WEAK}


def _mode_code(mode):
    if isinstance(mode, int):
        return mode
    return _MODES[mode]


def job_for(x, box, op="sum", mode="both", inc_out=None, exc_out=None, dtype_code=None):
    """Build an ``exs_job`` for device tensor ``x`` (outputs may be None).
    ``dtype_code`` overrides the element type taken from ``x.dtype`` (pairs:
    ``_lib.VALIDX`` on a packed int64 tensor)."""
    box = [int(v) for v in box]
    code = _dtype_code(x.dtype) if dtype_code is None else dtype_code
    return _lib.make_job(x.dim(), code, _OPS[op], _mode_code(mode),
                         list(x.shape), box, x.data_ptr(),
                         inc_out.data_ptr() if inc_out is not None else None,
                         exc_out.data_ptr() if exc_out is not None else None)


def workspace_size(shape, box, dtype, op="sum", mode="both") -> int:
    """Workspace bytes ``run`` needs (dtype: a torch dtype)."""
    j = _lib.make_job(len(shape), _dtype_code(dtype), _OPS[op], _mode_code(mode),
                      list(shape), list(box), None, None, None)
    n = ctypes.c_size_t()
    _lib.check(_lib.lib().exs_workspace_size(ctypes.byref(j), ctypes.byref(n)))
    return n.value


def _stream_ptr(stream):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def run(x, box, op="sum", mode="both", inc_out=None, exc_out=None, workspace=None,
        stream=None, dtype_code=None):
    """Included and/or excluded sums of the contiguous device tensor ``x``.

    Returns ``(inc, exc)`` (None for an output not requested).  The work is
    enqueued on ``stream`` (default: torch's current stream) without a host
    synchronisation.  ``workspace`` may be a preallocated uint8 device tensor.
    """
    import torch
    if not x.is_cuda:
        raise ExsError(1, "x must be a device tensor")
    if not x.is_contiguous():
        raise ExsError(1, "x must be contiguous")
    m = _mode_code(mode)
    if m & _lib.INCLUDED and inc_out is None:
        inc_out = torch.empty_like(x)
    if m & _lib.EXCLUDED and exc_out is None:
        exc_out = torch.empty_like(x)
    j = job_for(x, box, op, m, inc_out if m & _lib.INCLUDED else None,
                exc_out if m & _lib.EXCLUDED else None, dtype_code)
    n = ctypes.c_size_t()
    _lib.check(_lib.lib().exs_workspace_size(ctypes.byref(j), ctypes.byref(n)))
    if workspace is None or workspace.numel() < n.value:
        workspace = torch.empty(max(n.value, 1), dtype=torch.uint8, device=x.device)
    _lib.check(_lib.lib().exs_run(ctypes.byref(j), ctypes.c_void_p(workspace.data_ptr()),
                                  workspace.numel(), _stream_ptr(stream)))
    return (inc_out if m & _lib.INCLUDED else None, exc_out if m & _lib.EXCLUDED else None)


def run_corners(x, box, op="sum", exc_out=None, workspace=None, stream=None):
    """Strong excluded sums of the contiguous 2-D device tensor ``x`` by the
    corners algorithm, the paper's comparison system (``exs_run_corners``):
    the same results as ``run(x, box, op, "exc")``, by another method."""
    import torch
    if not x.is_cuda:
        raise ExsError(1, "x must be a device tensor")
    if not x.is_contiguous():
        raise ExsError(1, "x must be contiguous")
    if exc_out is None:
        exc_out = torch.empty_like(x)
    j = job_for(x, box, op, _lib.EXCLUDED, None, exc_out)
    n = ctypes.c_size_t()
    _lib.check(_lib.lib().exs_corners_workspace_size(ctypes.byref(j), ctypes.byref(n)))
    if workspace is None or workspace.numel() < n.value:
        workspace = torch.empty(max(n.value, 1), dtype=torch.uint8, device=x.device)
    _lib.check(_lib.lib().exs_run_corners(ctypes.byref(j), ctypes.c_void_p(workspace.data_ptr()),
                                          workspace.numel(), _stream_ptr(stream)))
    return exc_out


def corners_workspace_size(shape, box, dtype, op="sum") -> int:
    """Workspace bytes ``run_corners`` needs (dtype: a torch dtype)."""
    j = _lib.make_job(len(shape), _dtype_code(dtype), _OPS[op], _lib.EXCLUDED,
                      list(shape), list(box), None, None, None)
    n = ctypes.c_size_t()
    _lib.check(_lib.lib().exs_corners_workspace_size(ctypes.byref(j), ctypes.byref(n)))
    return n.value


def pack_pairs(values, index=None):
    """(value, index) pairs as one int64 tensor of the values' shape: each
    element holds the float32 value's bits in its low half and the int32
    index in its high half (the { float; int32; } layout of EXS_VALIDX).
    ``index`` defaults to the flat position."""
    import torch
    if values.dtype != torch.float32:
        raise ExsError(1, "pair values must be float32")
    if index is None:
        index = torch.arange(values.numel(), dtype=torch.int32,
                             device=values.device).reshape(values.shape)
    both = torch.stack([values.contiguous().view(torch.int32), index.to(torch.int32)], dim=-1)
    return both.contiguous().view(torch.int64).squeeze(-1)


def unpack_pairs(pairs):
    """The (values, index) tensors of packed pairs (views, no copy)."""
    import torch
    both = pairs.view(torch.int32).reshape(*pairs.shape, 2)
    return both[..., 0].view(torch.float32), both[..., 1]


def run_pairs(x, box, op="max", mode="both", inc_out=None, exc_out=None, workspace=None,
              stream=None):
    """Included and/or excluded "argmax" (``op="max"``) or "argmin"
    (``op="min"``) of packed (value, index) pairs (``pack_pairs``): per cell
    the best value over the box (or its complement) and, among equal values,
    the lowest index.  Returns packed pairs; ``unpack_pairs`` splits them."""
    import torch
    if x.dtype != torch.int64:
        raise ExsError(1, "pairs must be packed into an int64 tensor (pack_pairs)")
    return run(x, box, op, mode, inc_out, exc_out, workspace, stream, dtype_code=_lib.VALIDX)


FILL_NORMALISH, FILL_UNIFORM_INT, FILL_LOGMAG = 0, 1, 2


def fill(out, kind, seed, lo=-100, hi=100, stream=None):
    """Fill device tensor ``out`` with the counter-based generator (see exsum.h)."""
    _lib.check(_lib.lib().exs_fill(ctypes.c_void_p(out.data_ptr()), out.numel(),
                                   _dtype_code(out.dtype), kind, ctypes.c_uint64(seed),
                                   lo, hi, _stream_ptr(stream)))
    return out


def version() -> str:
    return _lib.lib().exs_version().decode()


class Batch:
    """Batched form: many jobs, one hipGraph launch (see exs_batch_* in exsum.h).

    ``items`` is a list of ``(x, box, op, mode)`` with ``x`` a contiguous
    device tensor.  Outputs are allocated here and exposed as ``outputs``
    (list of ``(inc, exc)``); they and the inputs must stay alive while the
    batch is used.  ``tune_cache`` is a JSON path for the autotuner (None:
    built-in settings).
    """

    def __init__(self, items, tune_cache=None):
        import torch
        self._keep = []
        self.outputs = []
        jobs = (_lib.ExsJob * len(items))()
        for i, (x, box, op, mode) in enumerate(items):
            if not x.is_cuda or not x.is_contiguous():
                raise ExsError(1, "batch inputs must be contiguous device tensors")
            m = _mode_code(mode)
            inc = torch.empty_like(x) if m & _lib.INCLUDED else None
            exc = torch.empty_like(x) if m & _lib.EXCLUDED else None
            jobs[i] = job_for(x, box, op, m, inc, exc)
            self._keep.append(x)
            self.outputs.append((inc, exc))
        h = ctypes.c_void_p()
        cache = tune_cache.encode() if tune_cache else None
        _lib.check(_lib.lib().exs_batch_create(jobs, len(items), cache, ctypes.byref(h)))
        self._h = h
        n = ctypes.c_size_t()
        _lib.check(_lib.lib().exs_batch_workspace_size(h, ctypes.byref(n)))
        self.workspace = torch.empty(max(n.value, 1), dtype=torch.uint8,
                                     device=items[0][0].device)

    def launch(self, stream=None):
        _lib.check(_lib.lib().exs_batch_launch(self._h, ctypes.c_void_p(self.workspace.data_ptr()),
                                               self.workspace.numel(), _stream_ptr(stream)))

    def launch_eager(self, stream=None):
        _lib.check(_lib.lib().exs_batch_launch_eager(
            self._h, ctypes.c_void_p(self.workspace.data_ptr()), self.workspace.numel(),
            _stream_ptr(stream)))

    def info(self):
        nodes = ctypes.c_int32()
        items = ctypes.c_int64()
        _lib.check(_lib.lib().exs_batch_info(self._h, ctypes.byref(nodes), ctypes.byref(items)))
        return {"graph_nodes": nodes.value, "work_items": items.value}

    def close(self):
        if getattr(self, "_h", None):
            _lib.lib().exs_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


_TYPESTR = {_lib.F32: "<f4", _lib.F64: "<f8", _lib.I32: "<i4", _lib.I64: "<i8"}


class _DeviceView:
    """A raw device buffer exposed through the CUDA array interface, so that
    torch can wrap it without a copy."""

    def __init__(self, ptr, shape, dtype_code):
        self.__cuda_array_interface__ = {"shape": tuple(int(v) for v in shape),
                                         "typestr": _TYPESTR[dtype_code],
                                         "data": (int(ptr), False), "version": 2,
                                         "strides": None}


class Server:
    """Serving form (see exs_server_* in exsum.h): requests are admitted in
    arrival order while their outputs and workspace fit ``hbm_budget`` bytes
    and one of ``max_inflight`` streams is idle; admitted requests run
    concurrently.

    ``submit`` returns a ticket; ``result`` returns ``(inc, exc)`` as torch
    views of the server's arena once the request completed (None before).
    The views are valid until ``release``; clone them to keep them longer
    (a clone enqueued on the stream passed to ``release`` is safe).
    """

    def __init__(self, hbm_budget, max_inflight=4):
        h = ctypes.c_void_p()
        _lib.check(_lib.lib().exs_server_create(int(hbm_budget), int(max_inflight),
                                                ctypes.byref(h)))
        self._h = h
        self._meta = {}
        self._keep = {}

    def submit(self, x, box, op="sum", mode="both", stream=None):
        """Queue a request on input ``x``; its work waits for what ``stream``
        (default: torch's current stream) has enqueued so far, so ``x`` may
        still be in production there."""
        if not x.is_cuda or not x.is_contiguous():
            raise ExsError(1, "server inputs must be contiguous device tensors")
        j = job_for(x, box, op, mode)
        t = ctypes.c_uint64()
        _lib.check(_lib.lib().exs_server_submit(self._h, ctypes.byref(j), _stream_ptr(stream),
                                                ctypes.byref(t)))
        self._meta[t.value] = (tuple(x.shape), j.dtype)
        self._keep[t.value] = x
        return t.value

    def submit_generated(self, shape, box, dtype, op="sum", mode="both", kind=0, seed=0,
                         lo=-100, hi=100):
        """Queue a request whose input the server fills itself (exs_fill)."""
        code = _dtype_code(dtype)
        j = _lib.make_job(len(shape), code, _OPS[op], _mode_code(mode), list(shape),
                          [int(v) for v in box], None, None, None)
        t = ctypes.c_uint64()
        _lib.check(_lib.lib().exs_server_submit_generated(
            self._h, ctypes.byref(j), int(kind), ctypes.c_uint64(seed), int(lo), int(hi),
            ctypes.byref(t)))
        self._meta[t.value] = (tuple(int(v) for v in shape), code)
        return t.value

    def _view(self, ptr, ticket):
        import torch
        if not ptr:
            return None
        shape, code = self._meta[ticket]
        return torch.as_tensor(_DeviceView(ptr, shape, code), device="cuda")

    def result(self, ticket):
        inc = ctypes.c_void_p()
        exc = ctypes.c_void_p()
        lat = ctypes.c_double()
        rc = _lib.lib().exs_server_poll(self._h, ctypes.c_uint64(ticket), ctypes.byref(inc),
                                        ctypes.byref(exc), ctypes.byref(lat))
        if rc == _lib.ENOTREADY:
            return None
        _lib.check(rc)
        return self._view(inc.value, ticket), self._view(exc.value, ticket), lat.value

    def done(self, ticket):
        """True once the request completed (no views are built)."""
        rc = _lib.lib().exs_server_poll(self._h, ctypes.c_uint64(ticket), None, None, None)
        if rc == _lib.ENOTREADY:
            return False
        _lib.check(rc)
        return True

    def input(self, ticket):
        p = ctypes.c_void_p()
        rc = _lib.lib().exs_server_input(self._h, ctypes.c_uint64(ticket), ctypes.byref(p))
        if rc == _lib.ENOTREADY:
            return None
        _lib.check(rc)
        return self._view(p.value, ticket)

    def drain(self):
        _lib.check(_lib.lib().exs_server_drain(self._h))

    def release(self, ticket, stream=None):
        """Forget ``ticket``; its memory is reused only after ``stream``
        (default: torch's current stream) has finished what it has enqueued so
        far, such as a copy of the result views."""
        _lib.check(_lib.lib().exs_server_release(self._h, ctypes.c_uint64(ticket),
                                                 _stream_ptr(stream)))
        self._meta.pop(ticket, None)
        self._keep.pop(ticket, None)

    def stats(self):
        d = [ctypes.c_double() for _ in range(4)]
        i = [ctypes.c_int64() for _ in range(3)]
        _lib.check(_lib.lib().exs_server_stats(self._h, *[ctypes.byref(v) for v in d],
                                               *[ctypes.byref(v) for v in i]))
        return {"p50_ms": d[0].value, "p99_ms": d[1].value, "req_per_s": d[2].value,
                "gelem_per_s": d[3].value, "completed": i[0].value,
                "max_queue": i[1].value, "peak_bytes": i[2].value}

    def close(self):
        if getattr(self, "_h", None):
            _lib.lib().exs_server_destroy(self._h)
            self._h = None
            self._keep.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
