"""GPU tests of batches across plans: uneven sizes in batched launches (with
and without a HIP graph) give, item by item, the transform of the oracle, and
the same result as each plan executed alone (within the precision's bound)."""
import numpy as np
import pytest

import oracle
from synth import uneven_batch, uniform_complex

pytestmark = pytest.mark.gpu

TOL = {0: 2e-6, 1: 1e-13}


def _items():
    # (dims, hdims, prec, sign, inplace)
    out = []
    for n, b, prec, sign in [(64, 9, 0, -1), (4096, 3, 0, 1), (1000, 4, 0, -1), (2187, 2, 1, -1),
                             (16384, 2, 0, -1), (65536, 1, 0, 1), (97, 7, 0, -1),
                             (1009, 3, 1, 1), (65537, 1, 0, -1), (65521, 1, 0, -1),
                             (8191, 2, 1, -1), (256, 31, 1, 1), (14175, 2, 0, -1),
                             (12, 50, 0, -1), (3125, 3, 0, 1),
                             # radices 17, 19, 23 (24 elements per thread), FP32 and FP64
                             (1088, 5, 0, -1), (7429, 2, 1, 1), (69632, 1, 0, -1)]:
        out.append(([(n, 1, 1)], [(b, n, n)] if b > 1 else [], prec, sign, False))
    out.append(([(24, 40, 40), (40, 1, 1)], [], 0, -1, True))            # 2-D in place
    out.append(([(32, 1, 32), (32, 32, 1)], [], 1, -1, False))            # transposed out
    # leaf-kernel passes with column and transposing tiles, both precisions
    out.append(([(65536, 1, 1)], [(2, 65536, 65536)], 1, -1, False))
    out.append(([(64, 4096, 4096), (64, 64, 64), (64, 1, 1)], [], 0, 1, True))   # 3-D in place
    out.append(([(256, 512, 1), (512, 1, 256)], [], 1, -1, False))        # transposed out
    return out


def _run_batch(graph):
    import torch

    import paper_2602_23525_amd as mfft
    specs = _items()
    plans, xs, ys, host = [], [], [], []
    for i, (dims, hd, prec, sign, ip) in enumerate(specs):
        tot = int(np.prod([d[0] for d in dims + hd]))
        cdt = np.complex64 if prec == 0 else np.complex128
        x = uniform_complex(tot, seed=500 + i, dtype=cdt)
        xt = torch.from_numpy(x).cuda()
        yt = xt if ip else torch.full_like(xt, float("nan"))
        plans.append(mfft.Plan(dims, hd, inplace=ip, sign=sign, prec=prec))
        xs.append(xt)
        ys.append(yt)
        host.append(x)
    b = mfft.Batch(plans, xs, ys, graph=graph)
    b.execute()
    torch.cuda.synchronize()
    outs = [y.cpu().numpy() for y in ys]
    for i, (dims, hd, prec, sign, ip) in enumerate(specs):
        ref = np.zeros(outs[i].size, np.complex128)
        oracle.dft(host[i].astype(np.complex128), ref, dims, hd, sign=sign)
        err = oracle.rel_rms(outs[i], ref)
        assert err <= TOL[prec], (i, dims, err)
    return plans, xs, ys, host, outs, b


def test_batch_matches_oracle_and_alone():
    import torch
    plans, xs, ys, host, outs, b = _run_batch(graph=False)
    info = b.info()
    assert info["tiles"] > 0 and info["launches"] >= 2
    # each plan alone
    for i, p in enumerate(plans):
        if p.inplace:
            continue
        y = torch.full_like(xs[i], float("nan"))
        p.execute(xs[i], y)
        torch.cuda.synchronize()
        a = y.cpu().numpy()
        tol = 2e-6 if a.dtype == np.complex64 else 1e-13
        assert oracle.rel_rms(a, outs[i]) <= 2 * tol
    b.destroy()


def test_batch_graph_replays_match_eager():
    import torch
    plans, xs, ys, host, outs, b = _run_batch(graph=True)
    for rep in range(3):
        # eager work between replays (restore in-place inputs first)
        for i, p in enumerate(plans):
            if p.inplace:
                xs[i].copy_(torch.from_numpy(host[i]).cuda())
            else:
                ys[i].fill_(float("nan"))
        torch.cuda.synchronize()
        b.execute()
        torch.cuda.synchronize()
        for i in range(len(plans)):
            assert np.array_equal(ys[i].cpu().numpy(), outs[i]), (rep, i)
    b.destroy()


def test_uneven_batch_sample_matches_oracle():
    """A seeded slice of the uneven-batch workload (sizes log-uniform 64..65536,
    60/30/10 power-of-two / smooth / prime), checked on every item."""
    import torch

    import paper_2602_23525_amd as mfft
    items = uneven_batch(count=60, seed=9)
    plans, xs, ys, host = [], [], [], []
    for it in items:
        x = uniform_complex(it.n * it.batch, seed=it.seed, dtype=np.complex64)
        xs.append(torch.from_numpy(x).cuda())
        ys.append(torch.empty_like(xs[-1]))
        host.append(x)
        plans.append(mfft.Plan([(it.n, 1, 1)], [(it.batch, it.n, it.n)] if it.batch > 1 else []))
    b = mfft.Batch(plans, xs, ys, graph=True)
    b.execute()
    torch.cuda.synchronize()
    for it, x, y in zip(items, host, ys):
        ref = oracle.fft(x.astype(np.complex128).reshape(it.batch, it.n))
        assert oracle.rel_rms(y.cpu().numpy().reshape(it.batch, it.n), ref) <= 2e-6, it
    b.destroy()


def test_batched_leaf_passes_bitwise_equal_alone():
    """Plans whose passes all run in the leaf kernel with full tiles (rows,
    columns, columns to rows with the twiddle) give the same bits in a batch
    (batched leaf launches) as alone."""
    import torch

    import paper_2602_23525_amd as mfft
    specs = [([(4096, 1, 1)], [(3, 4096, 4096)], 0), ([(1024, 1, 1)], [(40, 1024, 1024)], 1),
             ([(65536, 1, 1)], [(2, 65536, 65536)], 0), ([(65536, 1, 1)], [], 1),
             ([(256, 1, 16)], [(16, 256, 1)], 0)]
    plans, xs, ys = [], [], []
    for i, (dims, hd, prec) in enumerate(specs):
        tot = int(np.prod([d[0] for d in dims + hd]))
        cdt = np.complex64 if prec == 0 else np.complex128
        xs.append(torch.from_numpy(uniform_complex(tot, seed=700 + i, dtype=cdt)).cuda())
        ys.append(torch.full_like(xs[-1], float("nan")))
        plans.append(mfft.Plan(dims, hd, prec=prec))
        desc = plans[-1].info()["desc"]
        assert desc.count("leaf kernel") == plans[-1].info()["n_passes"], desc
    b = mfft.Batch(plans, xs, ys, graph=True)
    b.execute()
    torch.cuda.synchronize()
    for p, x, y in zip(plans, xs, ys):
        alone = torch.full_like(x, float("nan"))
        p.execute(x, alone)
        torch.cuda.synchronize()
        assert np.array_equal(alone.cpu().numpy(), y.cpu().numpy())
    b.destroy()
    for p in plans:
        p.destroy()
