"""Helpers for GPU parity tests: run a dft(N, V, I, O) problem through the HIP
library (via the C ABI binding) and the same problem through the FP64 oracle
on the same seeded input, then compare."""
from __future__ import annotations

import math
import sys

import numpy as np

import oracle
from synth import uniform_complex

TOL = {0: 2e-6, 1: 1e-13}          # relative RMS bounds, FP32 / FP64


def tol_for(prec: int, n_total: int) -> float:
    t = TOL[prec]
    if prec == 1 and n_total > (1 << 20):
        t *= math.log2(n_total) / 20.0
    return t


def span(dims, which):
    lo = hi = 0
    for d in dims:
        n, s = d[0], d[1 + which]
        if n <= 0:
            return 0, -1
        e = (n - 1) * s
        lo += min(e, 0)
        hi += max(e, 0)
    return lo, hi


def note(msg: str):
    print(msg, flush=True)
    sys.stdout.flush()


def run_case(dims, hdims=(), sign=-1, prec=0, inplace=False, seed=0, pad=3, check_guard=True,
             method="auto", sample=None, tol=None, name="", expect=None, flags=0,
             check_info=None):
    """Execute on the GPU and compare with the oracle; returns (relrms, maxerr).

    `sample`: list of vector multi-indices to compare (full-size runs); None =
    the whole problem.  `expect`: a substring the plan description must hold;
    `check_info`: a callable given the plan info; `flags`: planner flags.
    """
    import torch

    import paper_2602_23525_amd as mfft

    dims = [tuple(int(v) for v in d) for d in dims]
    hdims = [tuple(int(v) for v in d) for d in hdims]
    all_dims = dims + hdims
    ilo, ihi = span(all_dims, 0)
    olo, ohi = span(all_dims, 1)
    if inplace:
        lo, hi = min(ilo, olo), max(ihi, ohi)
        ilo = olo = lo
        ihi = ohi = hi
    in_len = ihi - ilo + 1 + 2 * pad
    out_len = ohi - olo + 1 + 2 * pad
    in_off = pad - ilo
    out_off = pad - olo
    cdt = np.complex64 if prec == 0 else np.complex128
    tdt = torch.complex64 if prec == 0 else torch.complex128
    note(f"[case] {name} dims={dims} hdims={hdims} sign={sign} prec={prec} inplace={inplace}")
    x = uniform_complex(max(in_len, 0), seed=seed, dtype=cdt)
    dev = torch.device("cuda", 0)
    xt = torch.from_numpy(x).to(dev)
    if inplace:
        yt = xt
    else:
        yt = torch.full((out_len,), complex(float("nan"), float("nan")), dtype=tdt, device=dev)
    plan = mfft.Plan(dims, hdims, inplace=inplace, sign=sign, prec=prec, flags=flags)
    eb = 8 if prec == 0 else 16
    plan.execute(xt.data_ptr() + eb * in_off, yt.data_ptr() + eb * out_off)
    torch.cuda.synchronize()
    y = yt.cpu().numpy().astype(np.complex128)
    info = plan.info()
    plan.destroy()
    if expect is not None:
        assert expect in info["desc"], f"plan lacks {expect!r}:\n{info['desc']}"
    if check_info is not None:
        check_info(info)

    x64 = x.astype(np.complex128)
    if not inplace:
        assert np.array_equal(xt.cpu().numpy(), x), "out-of-place transform modified its input"
    ref = np.full(out_len, np.nan + 0j)
    if sample is None:
        oracle.dft(x64, ref, dims, hdims, sign=sign, method=method, in_off=in_off,
                   out_off=out_off)
        mask = ~np.isnan(ref)
        got, want = y[mask], ref[mask]
        if check_guard and not inplace:
            assert np.all(np.isnan(y[~mask])), "library wrote outside the output tensor"
    else:
        # one transform at a time into a buffer spanning that transform's
        # outputs only
        tlo, thi = span(dims, 1)
        got_l, want_l = [], []
        for vidx in sample:
            ioff = in_off + sum(i * d[1] for i, d in zip(vidx, hdims))
            ooff = out_off + sum(i * d[2] for i, d in zip(vidx, hdims))
            r = np.full(thi - tlo + 1, np.nan + 0j)
            oracle.dft(x64, r, dims, [], sign=sign, method=method, in_off=ioff, out_off=-tlo)
            m = ~np.isnan(r)
            got_l.append(y[ooff + tlo:ooff + thi + 1][m])
            want_l.append(r[m])
        got, want = np.concatenate(got_l), np.concatenate(want_l)
    assert np.all(np.isfinite(got)), "non-finite output (unwritten element?)"
    rr = oracle.rel_rms(got, want)
    me = oracle.max_err(got, want)
    ntot = int(np.prod([d[0] for d in dims])) if dims else 1
    t = tol if tol is not None else tol_for(prec, ntot)
    note(f"    relrms={rr:.3e} maxerr={me:.3e} tol={t:.1e} passes={info['n_passes']}")
    assert rr <= t, f"relative RMS {rr} above {t}\n{info['desc']}"
    return rr, me
