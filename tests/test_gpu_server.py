"""GPU tests of the request server (continuous batching under an HBM budget):
every response matches the oracle, a request's result is identical alone and
in a mix, oversized requests are rejected, pending requests can be cancelled,
and the statistics are consistent."""
import time

import numpy as np
import pytest

import oracle
from synth import serve_trace, uniform_complex

pytestmark = pytest.mark.gpu


def _contig(dims):
    out, s = [], 1
    for n in reversed(dims):
        out.append((n, s, s))
        s *= n
    return list(reversed(out))


def _mk(req_dims, batch, prec, seed):
    import torch
    tot = int(np.prod(req_dims)) * batch
    cdt = np.complex64 if prec == 0 else np.complex128
    x = uniform_complex(tot, seed=seed, dtype=cdt)
    return x, torch.from_numpy(x).cuda()


def _problem(req_dims, batch):
    dims = _contig(req_dims)
    ntot = int(np.prod(req_dims))
    hd = [(batch, ntot, ntot)] if batch > 1 else []
    return dims, hd


def _read(ptr, count, prec):
    """Copy `count` elements of server-owned device memory to the host, with
    the hipMemcpy of the HIP runtime the library itself links."""
    import ctypes

    import torch

    import paper_2602_23525_amd as mfft
    dt = torch.complex64 if prec == 0 else torch.complex128
    t = torch.empty(count, dtype=dt, device="cuda")
    nbytes = count * (8 if prec == 0 else 16)
    hip_memcpy = mfft.lib().hipMemcpy
    hip_memcpy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int]
    hip_memcpy.restype = ctypes.c_int
    assert hip_memcpy(t.data_ptr(), ptr, nbytes, 3) == 0
    return t.cpu().numpy()


def test_server_mixed_requests_match_oracle():
    import paper_2602_23525_amd as mfft
    srv = mfft.Server(budget_bytes=2 << 30, max_inflight=32, n_streams=3)
    reqs = []
    specs = [((4096,), 8, 0, -1), ((1000,), 4, 0, 1), ((64, 64), 3, 1, -1), ((16, 12, 10), 2, 0, 1),
             ((65536,), 2, 0, -1), ((1009,), 5, 1, -1), ((256, 256), 1, 0, -1), ((97,), 30, 0, 1),
             ((2048,), 16, 1, 1), ((30, 42), 6, 0, -1)]
    for i, (shape, b, prec, sign) in enumerate(specs):
        x, xt = _mk(shape, b, prec, 900 + i)
        dims, hd = _problem(shape, b)
        t = srv.submit(dims, hd, xt, None, sign=sign, prec=prec)
        reqs.append((t, x, xt, dims, hd, prec, sign))
    for t, x, xt, dims, hd, prec, sign in reqs:
        assert srv.wait(t, 60000) == 0
        y = _read(srv.output(t), x.size, prec)
        ref = np.zeros(x.size, np.complex128)
        oracle.dft(x.astype(np.complex128), ref, dims, hd, sign=sign)
        assert oracle.rel_rms(y, ref) <= (2e-6 if prec == 0 else 1e-13)
        srv.release(t)
    st = srv.stats()
    assert st["completed"] == len(specs) and st["failed"] == 0
    assert st["launches"] >= 1 and st["p99_ms"] >= st["p50_ms"] > 0
    # what stays in use are the cached plans' tables, inside the budget
    assert st["bytes_in_use"] == st["plan_bytes"] > 0 and st["peak_bytes"] <= 2 << 30
    srv.destroy()


def test_result_same_alone_and_in_mix():
    import paper_2602_23525_amd as mfft
    shape, b, prec = (4096,), 4, 0
    x, xt = _mk(shape, b, prec, 77)
    dims, hd = _problem(shape, b)
    srv = mfft.Server(budget_bytes=1 << 30, max_inflight=64, n_streams=4)
    t = srv.submit(dims, hd, xt, None)
    assert srv.wait(t, 60000) == 0
    alone = _read(srv.output(t), x.size, prec)
    srv.release(t)
    # the same request among many others arriving together
    others = []
    for i in range(24):
        n = [128, 1000, 2187, 8192, 97][i % 5]
        xo, xot = _mk((n,), 3, 0, 1000 + i)
        d2, h2 = _problem((n,), 3)
        others.append((srv.submit(d2, h2, xot, None), xot))
        if i == 11:
            t = srv.submit(dims, hd, xt, None)
    assert srv.wait(t, 60000) == 0
    mixed = _read(srv.output(t), x.size, prec)
    srv.release(t)
    for to, _ in others:
        assert srv.wait(to, 60000) == 0
        srv.release(to)
    assert np.array_equal(alone, mixed)
    ref = oracle.fft(x.astype(np.complex128).reshape(b, 4096))
    assert oracle.rel_rms(mixed.reshape(b, 4096), ref) <= 2e-6
    srv.destroy()


def test_budget_rejection_and_cancel():
    import torch

    import paper_2602_23525_amd as mfft
    srv = mfft.Server(budget_bytes=10 << 20, max_inflight=1, n_streams=1)
    big = torch.zeros(1 << 21, dtype=torch.complex64, device="cuda")        # 16 MiB output
    with pytest.raises(mfft.MfftError) as e:
        srv.submit([(1 << 21, 1, 1)], [], big, None)
    assert e.value.code == -6
    # a queue of requests that each take most of the budget: later ones wait
    x = torch.zeros(1 << 19, dtype=torch.complex64, device="cuda")          # 4 MiB
    tickets = [srv.submit([(1 << 19, 1, 1)], [], x, None) for _ in range(6)]
    srv.cancel(tickets[-1])
    assert srv.wait(tickets[-1], 1000) == -9
    for t in tickets[:-1]:
        assert srv.wait(t, 60000) == 0
        srv.release(t)
    st = srv.stats()
    assert st["rejected"] == 1 and st["cancelled"] == 1 and st["completed"] == 5
    assert st["peak_bytes"] <= 10 << 20
    srv.destroy()


def test_poisson_trace_small():
    """A short seeded Poisson trace through the server, responses sampled
    against the oracle."""
    import torch

    import paper_2602_23525_amd as mfft
    trace = serve_trace(40, rate_hz=2000.0, seed=6, hi_exp=16, max_batch=4)
    srv = mfft.Server(budget_bytes=1 << 30, max_inflight=16, n_streams=4)
    pools = {0: torch.from_numpy(uniform_complex(1 << 19, seed=3, dtype=np.complex64)).cuda(),
             1: torch.from_numpy(uniform_complex(1 << 19, seed=4, dtype=np.complex128)).cuda()}
    t0 = time.monotonic()
    sub = []
    for r in trace:
        while time.monotonic() - t0 < r.arrival:
            pass
        prec = 0 if r.prec == "c32" else 1
        view = pools[prec]
        dims, hd = _problem(r.dims, r.batch)
        t = srv.submit(dims, hd, view, None, sign=r.sign, prec=prec, arrival=t0 + r.arrival)
        sub.append((t, r, prec, view, dims, hd))
    for k, (t, r, prec, view, dims, hd) in enumerate(sub):
        assert srv.wait(t, 60000) == 0
        if k % 5 == 0:
            cnt = int(np.prod(r.dims)) * r.batch
            y = _read(srv.output(t), cnt, prec)
            x = view[:cnt].cpu().numpy().astype(np.complex128)
            ref = np.zeros(cnt, np.complex128)
            oracle.dft(x, ref, dims, hd, sign=r.sign)
            assert oracle.rel_rms(y, ref) <= (2e-6 if prec == 0 else 1e-13)
        srv.release(t)
    st = srv.stats()
    assert st["completed"] == len(trace)
    srv.destroy()


def test_memory_blocked_head_waits_for_release():
    """The queue head waits for arena memory held by finished, unreleased
    outputs; a client's release admits it, and shutdown cancels a request
    still blocked (neither may stall the scheduler)."""
    import torch

    import paper_2602_23525_amd as mfft
    srv = mfft.Server(budget_bytes=10 << 20, max_inflight=8, n_streams=2)
    x = torch.zeros(1 << 19, dtype=torch.complex64, device="cuda")          # 4 MiB
    dims = [(1 << 19, 1, 1)]
    t = [srv.submit(dims, [], x, None) for _ in range(3)]
    assert srv.wait(t[0], 60000) == 0 and srv.wait(t[1], 60000) == 0
    assert srv.wait(t[2], 200) == mfft.REQ_PENDING        # two 4 MiB outputs held
    srv.release(t[0])
    assert srv.wait(t[2], 60000) == 0
    srv.release(t[1])
    srv.release(t[2])
    t2 = [srv.submit(dims, [], x, None) for _ in range(3)]
    assert srv.wait(t2[0], 60000) == 0 and srv.wait(t2[1], 60000) == 0
    st = srv.stats()
    assert st["completed"] == 5
    srv.destroy()                                           # t2[2] is cancelled


def _is_prime(n):
    return n > 1 and all(n % f for f in range(2, int(n ** 0.5) + 1))


def _check_output(srv, t, x, dims, hd, prec, sign, rows=None):
    """Compare a finished request's output with the oracle (whole, or the
    given transforms of its batch)."""
    ntot = int(np.prod([d[0] for d in dims]))
    y = _read(srv.output(t), x.size, prec).astype(np.complex128)
    if rows is None:
        ref = np.zeros(x.size, np.complex128)
        oracle.dft(x.astype(np.complex128), ref, dims, hd, sign=sign)
        got = y
    else:
        got = np.concatenate([y[v * ntot:(v + 1) * ntot] for v in rows])
        ref = np.concatenate([oracle.fft(x[v * ntot:(v + 1) * ntot].astype(np.complex128)[None],
                                         sign=sign)[0] for v in rows])
    rr = oracle.rel_rms(got, ref)
    assert rr <= (2e-6 if prec == 0 else 1e-13), rr


def test_cache_miss_planned_aside_does_not_delay_planned_requests():
    """Requests whose plan is cached complete while other requests' plans are
    still being made by the planner thread."""
    import paper_2602_23525_amd as mfft
    srv = mfft.Server(budget_bytes=4 << 30, max_inflight=32, n_streams=2)
    xw, xwt = _mk((4096,), 4, 0, 501)
    dw, hw = _problem((4096,), 4)
    t = srv.submit(dw, hw, xwt, None)                 # warm the cache
    assert srv.wait(t, 60000) == 0
    srv.release(t)
    cold = []
    # FP64 prime plans, made one after another by the planner thread: first
    # a 2097143-point one (Bluestein over 2^22 points: an FP64 transform of
    # that length and 200 MB of tables to make), then three of 65k points
    sizes = [(2097143, 1)] + [(p, 2) for p in range(65521, 60000, -1) if _is_prime(p)][:3]
    inputs = [(_mk((n,), b, 1, 510 + i), _problem((n,), b)) for i, (n, b) in enumerate(sizes)]
    import torch
    torch.cuda.synchronize()
    # the cold requests, then at once the cached one
    for (x, xt), (d, h) in inputs:
        cold.append((srv.submit(d, h, xt, None, prec=1), x, xt, d, h))
    t0 = time.monotonic()
    t = srv.submit(dw, hw, xwt, None)
    assert srv.wait(t, 60000) == 0
    t1 = time.monotonic()
    states = [srv.wait(c[0], 0) for c in cold]
    print(f"cached request done after {1e3 * (t1 - t0):.2f} ms; cold states {states}", flush=True)
    # the cached request finished while the first cold request's plan was
    # still being made
    assert states[0] == mfft.REQ_PENDING
    _check_output(srv, t, xw, dw, hw, 0, -1)
    srv.release(t)
    for tc, x, xt, d, h in cold:
        assert srv.wait(tc, 60000) == 0
        _check_output(srv, tc, x, d, h, 1, -1)
        srv.release(tc)
    st = srv.stats()
    assert st["completed"] == 6 and st["failed"] == 0 and st["plans_cached"] == 5
    srv.destroy()


def test_cancel_while_planning_never_runs_and_frees_everything():
    import paper_2602_23525_amd as mfft
    srv = mfft.Server(budget_bytes=1 << 30, max_inflight=8, n_streams=2)
    x, xt = _mk((65519,), 3, 1, 520)
    d, h = _problem((65519,), 3)
    tc = srv.submit(d, h, xt, None, prec=1)          # plan not cached: being planned
    srv.cancel(tc)
    assert srv.wait(tc, 0) == -9
    srv.release(tc)
    xw, xwt = _mk((1000,), 5, 0, 521)
    dw, hw = _problem((1000,), 5)
    t = srv.submit(dw, hw, xwt, None)
    assert srv.wait(t, 60000) == 0
    _check_output(srv, t, xw, dw, hw, 0, -1)
    srv.release(t)
    time.sleep(0.5)                                    # let the planner finish, if it started
    st = srv.stats()
    assert st["cancelled"] == 1 and st["failed"] == 0 and st["completed"] == 1
    assert st["admitted"] == 1
    assert st["bytes_in_use"] == st["plan_bytes"]       # only cached tables remain
    srv.destroy()


def test_plan_tables_count_against_the_budget_and_unused_plans_are_evicted():
    """A budget too small for every plan's tables at once: cached plans no
    request holds are evicted, every response still matches the oracle, and
    outputs, scratch, descriptors and tables together stay within the budget."""
    import paper_2602_23525_amd as mfft
    budget = 40 << 20
    srv = mfft.Server(budget_bytes=budget, max_inflight=4, n_streams=2)
    primes = [p for p in range(65521, 60000, -1) if _is_prime(p)][:18]
    for i, n in enumerate(primes):
        x, xt = _mk((n,), 4, 0, 530 + i)
        d, h = _problem((n,), 4)
        t = srv.submit(d, h, xt, None, sign=(-1 if i % 2 else 1))
        assert srv.wait(t, 60000) == 0
        if i % 4 == 0:
            _check_output(srv, t, x, d, h, 0, -1 if i % 2 else 1, rows=[0, 3])
        srv.release(t)
        st = srv.stats()
        assert st["bytes_in_use"] == st["plan_bytes"] <= budget
    st = srv.stats()
    assert st["plans_evicted"] > 0 and st["peak_bytes"] <= budget
    assert st["completed"] == len(primes) and st["failed"] == 0
    srv.destroy()


def test_budget_reserved_through_the_callers_allocator():
    import torch

    import paper_2602_23525_amd as mfft
    calls = {"alloc": 0, "free": 0}
    dev = torch.cuda.current_device()

    @mfft.ALLOC_FN
    def _alloc(nbytes, stream, ctx):
        calls["alloc"] += 1
        return torch.cuda.caching_allocator_alloc(int(nbytes), dev, stream or 0)

    @mfft.FREE_FN
    def _free(ptr, stream, ctx):
        calls["free"] += 1
        torch.cuda.caching_allocator_delete(ptr)

    al = mfft.Allocator(_alloc, _free, None)
    srv = mfft.Server(budget_bytes=256 << 20, max_inflight=4, n_streams=1, allocator=al)
    assert calls["alloc"] == 2                          # the budget: request memory + descriptors
    x, xt = _mk((4096,), 8, 0, 540)
    d, h = _problem((4096,), 8)
    t = srv.submit(d, h, xt, None)
    assert srv.wait(t, 60000) == 0
    _check_output(srv, t, x, d, h, 0, -1)
    srv.release(t)
    assert calls["alloc"] == 2                          # plans and outputs come from the budget
    srv.destroy()
    assert calls["free"] == 2


def test_input_written_on_another_stream_is_waited_for():
    """The request's input is produced by device work still queued on a side
    stream at submission; the server orders its launch after that work."""
    import torch

    import paper_2602_23525_amd as mfft
    n, b = 8192, 64
    x = uniform_complex(n * b, seed=550, dtype=np.complex64)
    src = torch.from_numpy(x).cuda()
    dst = torch.zeros_like(src)
    a = torch.randn(4096, 4096, device="cuda")
    torch.cuda.synchronize()
    side = torch.cuda.Stream()
    srv = mfft.Server(budget_bytes=1 << 30, max_inflight=4, n_streams=2)
    d, h = _problem((n,), b)
    with torch.cuda.stream(side):
        for _ in range(6):                             # milliseconds of work ahead of the copy
            a = torch.tanh(a @ a)
        dst.copy_(src)
        t = srv.submit(d, h, dst, None, in_stream=side)
    assert srv.wait(t, 60000) == 0
    _check_output(srv, t, x, d, h, 0, -1, rows=[0, 31, 63])
    srv.release(t)
    srv.destroy()
