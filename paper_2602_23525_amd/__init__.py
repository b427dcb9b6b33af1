"""Python binding of libmfft (ctypes): argument marshalling only.

Every step of a transform runs in the HIP kernels of libmfft.so; PyTorch is
used only to hold device memory and to name streams.  If the library has not
been built, loading fails loudly -- there is no fallback.

The functions keep the C names (``mfft_plan_dft``, ``mfft_execute``, ...) and
a small ``Plan`` class wraps them for tensors.
"""
from __future__ import annotations

import ctypes
import os
import re

__all__ = [
    "lib", "IoDim", "PlanInfo", "MfftError", "Plan", "mfft_problem_check", "mfft_plan_dft",
    "mfft_execute", "mfft_execute_scratch", "mfft_execute_static_scratch", "mfft_plan_dft_real", "mfft_problem_check_real", "mfft_plan_info", "mfft_plan_destroy",
    "mfft_wisdom_export", "mfft_wisdom_import", "mfft_wisdom_forget", "mfft_last_error",
    "mfft_version", "C32", "C64", "ESTIMATE", "MEASURE", "WISDOM_ONLY", "NO_WISDOM",
    "FP32_TWIDDLES", "NO_SCRATCH",
    "header_functions", "LIB_PATH", "HEADER_PATH", "Batch", "BATCH_GRAPH", "Server", "Request",
]

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmfft.so")
HEADER_PATH = os.path.join(os.path.dirname(HERE), "include", "mfft.h")

C32, C64 = 0, 1
ESTIMATE, MEASURE, WISDOM_ONLY, NO_WISDOM, FP32_TWIDDLES, NO_SCRATCH = 0, 1, 2, 4, 8, 16

STATUS = {0: "MFFT_OK", -1: "MFFT_EINVAL", -2: "MFFT_ENOTSUP", -3: "MFFT_ENOMEM",
          -4: "MFFT_EHIP", -5: "MFFT_EALIGN", -6: "MFFT_EBUDGET", -7: "MFFT_ESTATE",
          -8: "MFFT_ETIMEOUT", -9: "MFFT_ECANCELED", -10: "MFFT_ENOWISDOM"}


class MfftError(RuntimeError):
    def __init__(self, code: int, where: str, msg: str):
        super().__init__(f"{where}: {STATUS.get(code, code)} ({msg})")
        self.code = code


class IoDim(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("is_", ctypes.c_int64), ("os", ctypes.c_int64)]


class PlanInfo(ctypes.Structure):
    _fields_ = [("prec", ctypes.c_int), ("sign", ctypes.c_int), ("rank", ctypes.c_int),
                ("howmany_rank", ctypes.c_int), ("inplace", ctypes.c_int),
                ("n_passes", ctypes.c_int), ("n_total", ctypes.c_int64),
                ("howmany", ctypes.c_int64), ("flops", ctypes.c_double),
                ("bytes_compulsory", ctypes.c_double), ("bytes_passes", ctypes.c_double),
                ("scratch_bytes", ctypes.c_size_t), ("table_bytes", ctypes.c_size_t),
                ("desc", ctypes.c_char * 1024), ("n_radices", ctypes.c_int),
                ("radices", ctypes.c_int * 64)]


ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p, ctypes.c_void_p)
FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p)


class Allocator(ctypes.Structure):
    _fields_ = [("alloc", ALLOC_FN), ("free", FREE_FN), ("ctx", ctypes.c_void_p)]


_LIB = None


def lib():
    """Load libmfft.so (after torch, so both share one HIP runtime)."""
    global _LIB
    if _LIB is not None:
        return _LIB
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"libmfft.so is not built ({LIB_PATH}); run __graft_entry__.build()")
    try:
        import torch  # noqa: F401  (loads the HIP runtime first)
    except ImportError:  # pragma: no cover
        pass
    L = ctypes.CDLL(LIB_PATH, mode=ctypes.RTLD_GLOBAL)
    p = ctypes.c_void_p
    i64 = ctypes.c_int64
    dims_p = ctypes.POINTER(IoDim)
    L.mfft_problem_check.argtypes = [ctypes.c_int, dims_p, ctypes.c_int, dims_p, ctypes.c_int,
                                     ctypes.c_int, ctypes.c_int]
    L.mfft_plan_dft.argtypes = [ctypes.POINTER(p), ctypes.c_int, dims_p, ctypes.c_int, dims_p,
                                ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_uint,
                                ctypes.POINTER(Allocator), p]
    L.mfft_problem_check_real.argtypes = [ctypes.c_int, ctypes.c_int, dims_p, ctypes.c_int,
                                          dims_p, ctypes.c_int, ctypes.c_int]
    L.mfft_problem_check_real.restype = ctypes.c_int
    for name in ("mfft_plan_dft_r2c", "mfft_plan_dft_c2r"):
        f = getattr(L, name)
        f.argtypes = [ctypes.POINTER(p), ctypes.c_int, dims_p, ctypes.c_int, dims_p, ctypes.c_int,
                      ctypes.c_int, ctypes.c_uint, ctypes.POINTER(Allocator), p]
        f.restype = ctypes.c_int
    L.mfft_execute.argtypes = [p, p, p, p]
    L.mfft_execute_scratch.argtypes = [p, p, p, p, p]
    L.mfft_execute_static_scratch.argtypes = [p, p, p, p]
    L.mfft_plan_info.argtypes = [p, ctypes.POINTER(PlanInfo)]
    L.mfft_plan_destroy.argtypes = [p]
    L.mfft_wisdom_export.argtypes = [ctypes.POINTER(ctypes.c_char_p), ctypes.POINTER(ctypes.c_size_t)]
    L.mfft_wisdom_import.argtypes = [ctypes.c_char_p, ctypes.c_size_t]
    L.mfft_wisdom_forget.argtypes = []
    L.mfft_free.argtypes = [p]
    L.mfft_batch_create.argtypes = [ctypes.POINTER(p), ctypes.c_int, ctypes.POINTER(p),
                                    ctypes.POINTER(p), ctypes.POINTER(p), ctypes.c_uint, p]
    L.mfft_batch_execute.argtypes = [p, p]
    L.mfft_batch_info.argtypes = [p, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int64)]
    L.mfft_batch_destroy.argtypes = [p]
    for name in ("mfft_batch_create", "mfft_batch_execute", "mfft_batch_info",
                 "mfft_batch_destroy"):
        getattr(L, name).restype = ctypes.c_int
    u64 = ctypes.c_uint64
    L.mfft_server_create.argtypes = [ctypes.POINTER(p), ctypes.c_size_t, ctypes.c_int, ctypes.c_int, p]
    L.mfft_server_submit.argtypes = [p, p, ctypes.POINTER(u64)]
    L.mfft_server_wait.argtypes = [p, u64, ctypes.c_int, ctypes.POINTER(ctypes.c_int)]
    L.mfft_server_output.argtypes = [p, u64, ctypes.POINTER(p)]
    L.mfft_server_release.argtypes = [p, u64]
    L.mfft_server_cancel.argtypes = [p, u64]
    L.mfft_server_stats.argtypes = [p, p]
    L.mfft_server_destroy.argtypes = [p]
    L.mfft_server_reset_stats.argtypes = [p]
    for name in ("mfft_server_create", "mfft_server_submit", "mfft_server_wait",
                 "mfft_server_output", "mfft_server_release", "mfft_server_cancel",
                 "mfft_server_stats", "mfft_server_destroy", "mfft_server_reset_stats"):
        getattr(L, name).restype = ctypes.c_int
    L.mfft_last_error.restype = ctypes.c_char_p
    L.mfft_version.restype = ctypes.c_char_p
    for name in ("mfft_problem_check", "mfft_plan_dft", "mfft_execute", "mfft_execute_scratch",
                 "mfft_execute_static_scratch",
                 "mfft_plan_info", "mfft_plan_destroy", "mfft_wisdom_export",
                 "mfft_wisdom_import", "mfft_wisdom_forget"):
        getattr(L, name).restype = ctypes.c_int
    _LIB = L
    del i64
    return L


def header_functions(path: str = HEADER_PATH) -> list[str]:
    """Names of the functions include/mfft.h declares."""
    text = open(path).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(mfft_[a-z0-9_]+)\s*\(", text)))


def mfft_last_error() -> str:
    return lib().mfft_last_error().decode()


def mfft_version() -> str:
    return lib().mfft_version().decode()


def _check(rc: int, where: str):
    if rc != 0:
        raise MfftError(rc, where, mfft_last_error())


def _dims(dims):
    dims = [tuple(int(v) for v in d) for d in (dims or [])]
    arr = (IoDim * max(1, len(dims)))(*[IoDim(*d) for d in dims])
    return len(dims), arr


def _ptr(x) -> int:
    if x is None:
        return 0
    if isinstance(x, int):
        return x
    return int(x.data_ptr())


def _stream(stream) -> int:
    if stream is None:
        import torch
        return int(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, int):
        return stream
    return int(stream.cuda_stream)


def mfft_problem_check(dims, howmany_dims=(), inplace=0, sign=-1, prec=C32) -> int:
    """Host-only validation; returns the status code (0 = valid)."""
    nr, nd = _dims(dims)
    vr, vd = _dims(howmany_dims)
    return lib().mfft_problem_check(nr, nd, vr, vd, int(inplace), int(sign), int(prec))


def mfft_plan_dft(dims, howmany_dims=(), inplace=0, sign=-1, prec=C32, flags=ESTIMATE,
                  allocator=None, stream=None) -> int:
    """Returns a plan handle (int); raises MfftError on failure."""
    nr, nd = _dims(dims)
    vr, vd = _dims(howmany_dims)
    h = ctypes.c_void_p()
    rc = lib().mfft_plan_dft(ctypes.byref(h), nr, nd, vr, vd, int(inplace), int(sign),
                             int(prec), int(flags), allocator, _stream(stream))
    _check(rc, "mfft_plan_dft")
    return h.value


def mfft_problem_check_real(kind: str, dims, howmany_dims=(), inplace=0, prec=C32) -> int:
    """Host-only validation of an r2c / c2r problem; returns the status code."""
    nr, nd = _dims(dims)
    vr, vd = _dims(howmany_dims)
    return lib().mfft_problem_check_real(1 if kind == "c2r" else 0, nr, nd, vr, vd, int(inplace),
                                         int(prec))


def mfft_plan_dft_real(kind: str, dims, howmany_dims=(), inplace=0, prec=C32, flags=ESTIMATE,
                       allocator=None, stream=None) -> int:
    """kind "r2c" (real input, n/2+1 complex outputs) or "c2r" (the inverse);
    strides in elements of each side's type.  Returns a plan handle."""
    nr, nd = _dims(dims)
    vr, vd = _dims(howmany_dims)
    h = ctypes.c_void_p()
    fn = {"r2c": lib().mfft_plan_dft_r2c, "c2r": lib().mfft_plan_dft_c2r}[kind]
    rc = fn(ctypes.byref(h), nr, nd, vr, vd, int(inplace), int(prec), int(flags), allocator,
            _stream(stream))
    _check(rc, f"mfft_plan_dft_{kind}")
    return h.value


def mfft_execute(plan: int, x, y, stream=None):
    _check(lib().mfft_execute(plan, _ptr(x), _ptr(y), _stream(stream)), "mfft_execute")


def mfft_execute_scratch(plan: int, x, y, scratch, stream=None):
    _check(lib().mfft_execute_scratch(plan, _ptr(x), _ptr(y), _ptr(scratch), _stream(stream)),
           "mfft_execute_scratch")


def mfft_execute_static_scratch(plan: int, x, y, stream=None):
    _check(lib().mfft_execute_static_scratch(plan, _ptr(x), _ptr(y), _stream(stream)),
           "mfft_execute_static_scratch")


STATIC_SCRATCH_BYTES = 64 << 20


def mfft_plan_info(plan: int) -> dict:
    info = PlanInfo()
    _check(lib().mfft_plan_info(plan, ctypes.byref(info)), "mfft_plan_info")
    d = {k: getattr(info, k) for k, _ in PlanInfo._fields_ if k not in ("desc", "radices")}
    d["desc"] = info.desc.decode(errors="replace")
    # radices per pass (a pass without a transform: an empty list)
    passes, cur = [], []
    for r in info.radices[: info.n_radices]:
        if r == 0:
            passes.append(cur)
            cur = []
        else:
            cur.append(r)
    d["radices"] = passes
    return d


def mfft_plan_destroy(plan: int):
    _check(lib().mfft_plan_destroy(plan), "mfft_plan_destroy")


def mfft_wisdom_export() -> str:
    buf = ctypes.c_char_p()
    n = ctypes.c_size_t()
    _check(lib().mfft_wisdom_export(ctypes.byref(buf), ctypes.byref(n)), "mfft_wisdom_export")
    s = ctypes.string_at(buf, n.value).decode()
    lib().mfft_free(ctypes.cast(buf, ctypes.c_void_p))
    return s


def mfft_wisdom_import(text: str):
    b = text.encode()
    _check(lib().mfft_wisdom_import(b, len(b)), "mfft_wisdom_import")


def mfft_wisdom_forget():
    _check(lib().mfft_wisdom_forget(), "mfft_wisdom_forget")


def torch_allocator(device=None):
    """An mfft_allocator backed by torch's caching allocator (keeps the
    callbacks alive as attributes of the returned structure)."""
    import torch
    dev = torch.cuda.current_device() if device is None else device

    @ALLOC_FN
    def _alloc(nbytes, stream, ctx):
        try:
            return torch.cuda.caching_allocator_alloc(int(nbytes), dev, stream or 0)
        except Exception:  # pragma: no cover
            return None

    @FREE_FN
    def _free(ptr, stream, ctx):
        torch.cuda.caching_allocator_delete(ptr)

    a = Allocator(_alloc, _free, None)
    a._keep = (_alloc, _free)
    return a


class Plan:
    """A planned dft(N, V, I, O); strides in complex elements.  kind "r2c" /
    "c2r" plans the real-data transforms (strides in elements of each side's
    type, sign implied)."""

    def __init__(self, dims, howmany_dims=(), inplace=False, sign=-1, prec=C32,
                 flags=ESTIMATE, stream=None, allocator=None, kind="c2c"):
        self.dims = [tuple(d) for d in dims]
        self.howmany_dims = [tuple(d) for d in howmany_dims]
        self.inplace = bool(inplace)
        self.kind = kind
        self.sign = sign if kind == "c2c" else (-1 if kind == "r2c" else 1)
        self.prec = prec
        self._alloc = allocator
        al = ctypes.byref(allocator) if allocator is not None else None
        if kind == "c2c":
            self.handle = mfft_plan_dft(dims, howmany_dims, int(inplace), sign, prec, flags, al,
                                        stream)
        else:
            self.handle = mfft_plan_dft_real(kind, dims, howmany_dims, int(inplace), prec, flags,
                                             al, stream)

    def execute(self, x, y=None, stream=None):
        y = x if y is None else y
        mfft_execute(self.handle, x, y, stream)
        return y

    def execute_scratch(self, x, y, scratch, stream=None):
        mfft_execute_scratch(self.handle, x, y, scratch, stream)
        return y

    def execute_static_scratch(self, x, y=None, stream=None):
        y = x if y is None else y
        mfft_execute_static_scratch(self.handle, x, y, stream)
        return y

    def info(self) -> dict:
        return mfft_plan_info(self.handle)

    def destroy(self):
        if self.handle:
            mfft_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


BATCH_GRAPH = 1


class Batch:
    """Many (plan, in, out) triples executed as one workload (mfft_batch_*)."""

    def __init__(self, plans, ins, outs, graph=False, stream=None):
        n = len(plans)
        P = ctypes.c_void_p * max(1, n)
        self._plans = list(plans)          # keep the plans alive
        hp = P(*[pl.handle for pl in plans])
        hi = P(*[_ptr(x) for x in ins])
        ho = P(*[_ptr(y) for y in outs])
        h = ctypes.c_void_p()
        rc = lib().mfft_batch_create(ctypes.byref(h), n, hp, hi, ho,
                                     BATCH_GRAPH if graph else 0, _stream(stream))
        _check(rc, "mfft_batch_create")
        self.handle = h.value

    def execute(self, stream=None):
        _check(lib().mfft_batch_execute(self.handle, _stream(stream)), "mfft_batch_execute")

    def info(self):
        la = ctypes.c_int()
        ti = ctypes.c_int64()
        _check(lib().mfft_batch_info(self.handle, ctypes.byref(la), ctypes.byref(ti)),
               "mfft_batch_info")
        return {"launches": la.value, "tiles": ti.value}

    def destroy(self):
        if self.handle:
            lib().mfft_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


class Request(ctypes.Structure):
    _fields_ = [("rank", ctypes.c_int), ("dims", IoDim * 8), ("howmany_rank", ctypes.c_int),
                ("howmany_dims", IoDim * 8), ("sign", ctypes.c_int), ("prec", ctypes.c_int),
                ("in_", ctypes.c_void_p), ("out", ctypes.c_void_p), ("arrival", ctypes.c_double),
                ("in_stream", ctypes.c_void_p)]


class ServerStats(ctypes.Structure):
    _fields_ = [(k, ctypes.c_uint64) for k in ("submitted", "admitted", "completed", "rejected",
                                               "failed", "cancelled", "launches")] + \
               [(k, ctypes.c_double) for k in ("p50_ms", "p99_ms", "mean_ms", "max_ms", "busy_s",
                                               "flops", "bytes")] + \
               [("bytes_in_use", ctypes.c_size_t), ("peak_bytes", ctypes.c_size_t),
                ("plan_bytes", ctypes.c_size_t), ("plans_cached", ctypes.c_int),
                ("max_inflight_seen", ctypes.c_int), ("plans_evicted", ctypes.c_int)]


REQ_DONE, REQ_PENDING, REQ_RUNNING = 0, 1, 2


class Server:
    """Request server with continuous batching (mfft_server_*)."""

    def __init__(self, budget_bytes, max_inflight=64, n_streams=4, allocator=None):
        L = lib()
        h = ctypes.c_void_p()
        self._alloc = allocator      # keeps the callbacks alive
        al = ctypes.byref(allocator) if allocator is not None else None
        _check(L.mfft_server_create(ctypes.byref(h), int(budget_bytes), int(max_inflight),
                                    int(n_streams), al), "mfft_server_create")
        self.handle = h.value

    def submit(self, dims, howmany_dims=(), x=None, y=None, sign=-1, prec=C32, arrival=0.0,
               in_stream="current"):
        """in_stream: the stream whose work produces x ("current": torch's
        current stream; None: x is complete already)."""
        r = Request()
        r.rank = len(dims)
        for i, d in enumerate(dims):
            r.dims[i] = IoDim(*d)
        r.howmany_rank = len(howmany_dims)
        for i, d in enumerate(howmany_dims):
            r.howmany_dims[i] = IoDim(*d)
        r.sign, r.prec = int(sign), int(prec)
        r.in_ = _ptr(x)
        r.out = _ptr(y) if y is not None else None
        r.arrival = float(arrival)
        r.in_stream = None if in_stream is None else _stream(None if in_stream == "current"
                                                             else in_stream)
        t = ctypes.c_uint64()
        _check(lib().mfft_server_submit(self.handle, ctypes.byref(r), ctypes.byref(t)),
               "mfft_server_submit")
        return t.value

    def wait(self, ticket, timeout_ms=-1):
        st = ctypes.c_int()
        rc = lib().mfft_server_wait(self.handle, ctypes.c_uint64(ticket), int(timeout_ms),
                                    ctypes.byref(st))
        if rc not in (0, -8):
            _check(rc, "mfft_server_wait")
        return st.value

    def output(self, ticket) -> int:
        p = ctypes.c_void_p()
        _check(lib().mfft_server_output(self.handle, ctypes.c_uint64(ticket), ctypes.byref(p)),
               "mfft_server_output")
        return p.value or 0

    def release(self, ticket):
        _check(lib().mfft_server_release(self.handle, ctypes.c_uint64(ticket)),
               "mfft_server_release")

    def cancel(self, ticket):
        _check(lib().mfft_server_cancel(self.handle, ctypes.c_uint64(ticket)), "mfft_server_cancel")

    def reset_stats(self):
        _check(lib().mfft_server_reset_stats(self.handle), "mfft_server_reset_stats")

    def stats(self) -> dict:
        s = ServerStats()
        _check(lib().mfft_server_stats(self.handle, ctypes.byref(s)), "mfft_server_stats")
        return {k: getattr(s, k) for k, _ in ServerStats._fields_}

    def destroy(self):
        if self.handle:
            lib().mfft_server_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


def fft_plan_for(x_shape, axes=None, batch_axes=None, sign=-1, prec=C32, inplace=False,
                 out_strides=None):
    """Plan the DFT of a contiguous tensor of shape `x_shape` over `axes` (default:
    all), looping over the remaining axes.  Output strides default to the input's."""
    nd = len(x_shape)
    axes = list(range(nd)) if axes is None else [a % nd for a in axes]
    strides = [1] * nd
    for i in range(nd - 2, -1, -1):
        strides[i] = strides[i + 1] * x_shape[i + 1]
    ostr = strides if out_strides is None else out_strides
    dims = [(x_shape[a], strides[a], ostr[a]) for a in axes]
    hdims = [(x_shape[a], strides[a], ostr[a]) for a in range(nd) if a not in axes]
    return Plan(dims, hdims, inplace=inplace, sign=sign, prec=prec)
