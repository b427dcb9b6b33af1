"""GPU parity of the real-data transforms (r2c: real input, half spectrum out;
c2r: its unnormalized inverse) against the oracle's rfft / irfft, through the
C ABI: the packed half-length path (even n, unit real stride) and the general
path (odd n, strided real data), batches, both precisions, in place."""
import numpy as np
import pytest

import oracle
from synth import uniform_complex

pytestmark = pytest.mark.gpu
TOL = {0: 2e-6, 1: 1e-13}


def _real_seq(count, seed, prec):
    # U[-1, 1) reals from the seeded complex generator (real and imaginary parts)
    z = uniform_complex((count + 1) // 2, seed=seed, dtype=np.complex128)
    x = np.stack([z.real, z.imag], axis=-1).reshape(-1)[:count]
    return x.astype(np.float32 if prec == 0 else np.float64)


def _dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def r2c_case(n, b, prec, is_=1, dist_in=None, os_=1, dist_out=None, inplace=False, seed=1):
    import torch

    import paper_2602_23525_amd as mfft
    h = n // 2 + 1
    dist_in = dist_in if dist_in is not None else n * is_
    dist_out = dist_out if dist_out is not None else h * os_
    rdt = np.float32 if prec == 0 else np.float64
    cdt = np.complex64 if prec == 0 else np.complex128
    nin = (b - 1) * dist_in + (n - 1) * is_ + 1
    x = _real_seq(nin, seed, prec)
    xs = np.stack([x[v * dist_in:v * dist_in + (n - 1) * is_ + 1:is_] for v in range(b)])
    ref = oracle.rfft(xs.astype(np.float64))
    hd = [(b, dist_in, dist_out)] if b > 1 else []
    p = mfft.Plan([(n, is_, os_)], hd, inplace=inplace, prec=prec, kind="r2c")
    if inplace:
        # one buffer: real rows at dist_in reals, complex rows at dist_out
        nbytes = max(nin * x.itemsize, ((b - 1) * dist_out + (h - 1) * os_ + 1) * 2 * x.itemsize)
        nel = nbytes // x.itemsize + 2
        buf = torch.zeros(nel + nel % 2, dtype=torch.float32 if prec == 0 else torch.float64,
                          device="cuda")
        buf[:nin] = _dev(x)
        p.execute(buf, buf)
        torch.cuda.synchronize()
        y = buf.view(torch.complex64 if prec == 0 else torch.complex128).cpu().numpy()
    else:
        xt = _dev(x)
        nout = (b - 1) * dist_out + (h - 1) * os_ + 1
        yt = torch.full((nout,), float("nan"), dtype=torch.complex64 if prec == 0 else
                        torch.complex128, device="cuda")
        p.execute(xt, yt)
        torch.cuda.synchronize()
        assert np.array_equal(xt.cpu().numpy(), x)
        y = yt.cpu().numpy()
    p.destroy()
    ys = np.stack([y[v * dist_out:v * dist_out + (h - 1) * os_ + 1:os_] for v in range(b)])
    err = oracle.rel_rms(ys.astype(np.complex128), ref)
    assert err <= TOL[prec], (n, b, prec, err)
    return err


def c2r_case(n, b, prec, is_=1, dist_in=None, os_=1, dist_out=None, inplace=False, seed=2):
    import torch

    import paper_2602_23525_amd as mfft
    h = n // 2 + 1
    dist_in = dist_in if dist_in is not None else h * is_
    dist_out = dist_out if dist_out is not None else n * os_
    cdt = np.complex64 if prec == 0 else np.complex128
    nin = (b - 1) * dist_in + (h - 1) * is_ + 1
    X = uniform_complex(nin, seed=seed, dtype=cdt)
    Xs = np.stack([X[v * dist_in:v * dist_in + (h - 1) * is_ + 1:is_] for v in range(b)])
    ref = oracle.irfft(Xs.astype(np.complex128), n)
    hd = [(b, dist_in, dist_out)] if b > 1 else []
    p = mfft.Plan([(n, is_, os_)], hd, inplace=inplace, prec=prec, kind="c2r")
    rt = torch.float32 if prec == 0 else torch.float64
    if inplace:
        ncomplex = max(nin, ((b - 1) * dist_out + (n - 1) * os_ + 2) // 2 + 1)
        buf = torch.zeros(ncomplex, dtype=torch.complex64 if prec == 0 else torch.complex128,
                          device="cuda")
        buf[:nin] = _dev(X)
        p.execute(buf, buf)
        torch.cuda.synchronize()
        y = buf.view(rt).cpu().numpy()
    else:
        Xt = _dev(X)
        nout = (b - 1) * dist_out + (n - 1) * os_ + 1
        nout += nout % 2
        yt = torch.full((nout,), float("nan"), dtype=rt, device="cuda")
        p.execute(Xt, yt)
        torch.cuda.synchronize()
        assert np.array_equal(Xt.cpu().numpy(), X)
        y = yt.cpu().numpy()
    p.destroy()
    ys = np.stack([y[v * dist_out:v * dist_out + (n - 1) * os_ + 1:os_] for v in range(b)])
    err = oracle.rel_rms(ys.astype(np.float64), ref)
    assert err <= TOL[prec], (n, b, prec, err)
    return err


# 128 .. 8192 take the one-pass path (a specialized leaf of half the length)
SIZES = [1, 2, 3, 4, 5, 6, 8, 15, 16, 17, 30, 64, 100, 128, 243, 256, 512, 1000, 1009, 1024,
         2048, 2187, 4096, 8192, 14175, 65536, 65537]


@pytest.mark.parametrize("n", SIZES)
@pytest.mark.parametrize("prec", [0, 1])
def test_r2c_contiguous(n, prec):
    b = max(1, min(5, 100000 // n))
    r2c_case(n, b, prec, seed=n)


@pytest.mark.parametrize("n", SIZES)
@pytest.mark.parametrize("prec", [0, 1])
def test_c2r_contiguous(n, prec):
    b = max(1, min(5, 100000 // n))
    c2r_case(n, b, prec, seed=n + 1)


@pytest.mark.parametrize("n", [8, 9, 1000, 4096])
def test_strided_and_odd_distances(n):
    # real stride 2 and odd distances take the general path; complex side strided
    r2c_case(n, 3, 0, is_=2, dist_in=2 * n + 1, os_=3, dist_out=3 * (n // 2 + 1) + 2, seed=3)
    c2r_case(n, 3, 0, is_=2, dist_in=2 * (n // 2 + 1) + 1, os_=3, dist_out=3 * n + 1, seed=4)
    # packed path with padded even distances
    r2c_case(n, 4, 1, dist_in=n + 6, dist_out=n // 2 + 5, seed=5)
    c2r_case(n, 4, 1, dist_in=n // 2 + 3, dist_out=n + 2, seed=6)


@pytest.mark.parametrize("n", [16, 1000, 4096, 8192, 65536, 17])
@pytest.mark.parametrize("prec", [0, 1])
def test_in_place(n, prec):
    h = n // 2 + 1
    r2c_case(n, 3, prec, dist_in=2 * h, dist_out=h, inplace=True, seed=7)
    c2r_case(n, 3, prec, dist_in=h, dist_out=2 * h, inplace=True, seed=8)


@pytest.mark.parametrize("n", [4096, 1 << 20])
def test_round_trip(n):
    import torch

    import paper_2602_23525_amd as mfft
    b = 2
    x = _real_seq(n * b, 9, 0)
    xt = _dev(x)
    Xt = torch.empty(b * (n // 2 + 1), dtype=torch.complex64, device="cuda")
    zt = torch.empty_like(xt)
    f = mfft.Plan([(n, 1, 1)], [(b, n, n // 2 + 1)], kind="r2c")
    g = mfft.Plan([(n, 1, 1)], [(b, n // 2 + 1, n)], kind="c2r")
    f.execute(xt, Xt)
    g.execute(Xt, zt)
    torch.cuda.synchronize()
    z = zt.cpu().numpy() / n
    assert oracle.rel_rms(z.astype(np.float64), x.astype(np.float64)) <= 4e-6
    info = f.info()
    assert info["flops"] == pytest.approx(2.5 * n * np.log2(n) * b)
    f.destroy()
    g.destroy()


def test_real_plans_in_a_batch():
    """Real plans inside a batch across plans match the oracle, and graph
    replays repeat the same bits (the batch runs the generic tile kernel where
    a plan alone may use the specialized leaf, so alone vs batch agree within
    the tolerance, not bitwise)."""
    import torch

    import paper_2602_23525_amd as mfft
    shapes = [(4096, 8), (1000, 5), (17, 3), (65536, 2), (8192, 3)]
    plans, ins, outs, alone = [], [], [], []
    refs = []
    for i, (n, b) in enumerate(shapes):
        p = mfft.Plan([(n, 1, 1)], [(b, n, n // 2 + 1)], kind="r2c")
        xh = _real_seq(n * b, 20 + i, 0)
        refs.append(oracle.rfft(xh.astype(np.float64).reshape(b, n)))
        x = _dev(xh)
        y = torch.empty(b * (n // 2 + 1), dtype=torch.complex64, device="cuda")
        p.execute(x, y)
        torch.cuda.synchronize()
        alone.append(y.cpu().numpy())
        y.fill_(0)
        plans.append(p)
        ins.append(x)
        outs.append(y)
    bt = mfft.Batch(plans, [x.data_ptr() for x in ins], [y.data_ptr() for y in outs], graph=True)
    first = None
    for rep in range(3):
        bt.execute()
        torch.cuda.synchronize()
        got = [y.cpu().numpy() for y in outs]
        for g, a, r, (n, b) in zip(got, alone, refs, shapes):
            assert oracle.rel_rms(g.reshape(b, -1).astype(np.complex128), r) <= TOL[0]
            assert oracle.rel_rms(g, a) <= 2 * TOL[0]
        if first is None:
            first = got
        else:
            assert all(np.array_equal(g, f) for g, f in zip(got, first))
    bt.destroy()
    for p in plans:
        p.destroy()


def _row_major(shape):
    st, s = [], 1
    for n in reversed(shape):
        st.append(s)
        s *= n
    return list(reversed(st)), s


@pytest.mark.parametrize("shape", [(16, 32), (12, 10), (8, 6, 10), (3, 17), (256, 256),
                                   (32, 8192), (5, 7, 9)])
@pytest.mark.parametrize("prec", [0, 1])
def test_multidim(shape, prec):
    """Rank > 1: the last dimension halved (n/2+1 complex values), the others
    full; r2c against the oracle's rfftn, c2r of arbitrary half spectra
    against its irfftn (inverse along the leading axes, then the real inverse)."""
    import torch

    import paper_2602_23525_amd as mfft
    b = 2
    hshape = tuple(shape[:-1]) + (shape[-1] // 2 + 1,)
    rs, rtot = _row_major(shape)
    cs, ctot = _row_major(hshape)
    cdt = np.complex64 if prec == 0 else np.complex128
    # forward
    x = _real_seq(b * rtot, 40 + len(shape), prec)
    dims = [(n, rs[i], cs[i]) for i, n in enumerate(shape)]
    p = mfft.Plan(dims, [(b, rtot, ctot)], prec=prec, kind="r2c")
    yt = torch.full((b * ctot,), float("nan"), dtype=torch.complex64 if prec == 0 else
                    torch.complex128, device="cuda")
    p.execute(_dev(x), yt)
    torch.cuda.synchronize()
    p.destroy()
    ref = oracle.rfftn(x.astype(np.float64).reshape((b,) + shape), len(shape))
    assert oracle.rel_rms(yt.cpu().numpy().reshape(ref.shape).astype(np.complex128),
                          ref) <= TOL[prec]
    # inverse, from an arbitrary half spectrum (the input must stay intact)
    X = uniform_complex(b * ctot, seed=50 + len(shape), dtype=cdt)
    dims = [(n, cs[i], rs[i]) for i, n in enumerate(shape)]
    q = mfft.Plan(dims, [(b, ctot, rtot)], prec=prec, kind="c2r")
    Xt = _dev(X)
    zt = torch.full((b * rtot,), float("nan"), dtype=torch.float32 if prec == 0 else
                    torch.float64, device="cuda")
    q.execute(Xt, zt)
    torch.cuda.synchronize()
    q.destroy()
    assert np.array_equal(Xt.cpu().numpy(), X)
    ref = oracle.irfftn(X.astype(np.complex128).reshape((b,) + hshape), shape)
    assert oracle.rel_rms(zt.cpu().numpy().reshape(ref.shape).astype(np.float64),
                          ref) <= TOL[prec]


def test_multidim_in_place():
    """FFTW's in-place layout: real rows padded to 2(n/2+1) values."""
    import torch

    import paper_2602_23525_amd as mfft
    n0, n1 = 24, 40
    hc = n1 // 2 + 1
    x = _real_seq(n0 * n1, 61, 0).reshape(n0, n1)
    buf = torch.zeros(n0 * 2 * hc, dtype=torch.float32, device="cuda")
    buf.view(n0, 2 * hc)[:, :n1] = _dev(x)
    f = mfft.Plan([(n0, 2 * hc, hc), (n1, 1, 1)], [], inplace=True, kind="r2c")
    f.execute(buf, buf)
    torch.cuda.synchronize()
    y = buf.view(torch.complex64).cpu().numpy().reshape(n0, hc)
    assert oracle.rel_rms(y.astype(np.complex128), oracle.rfftn(x.astype(np.float64), 2)) <= 2e-6
    g = mfft.Plan([(n0, hc, 2 * hc), (n1, 1, 1)], [], inplace=True, kind="c2r")
    g.execute(buf, buf)
    torch.cuda.synchronize()
    z = buf.cpu().numpy().reshape(n0, 2 * hc)[:, :n1] / (n0 * n1)
    assert oracle.rel_rms(z.astype(np.float64), x.astype(np.float64)) <= 4e-6
    f.destroy()
    g.destroy()
