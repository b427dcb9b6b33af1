"""GPU tests of in-place plans without scratch (MFFT_NO_SCRATCH; Section
4.2's in-place plans): n = k*q*q as columns with the twiddle, rows, in-place
q x q transposes and (k > 1) an in-place transpose of the k x q matrix of
q-element runs, all in the caller's buffer, against the FP64 oracle; in-place
rank-0 transposes (Section 4.2, "Rank-0 plans") the same way; problems
without such a plan are refused."""
import numpy as np
import pytest

import oracle
from synth import uniform_complex
from tests.gpu_util import run_case

pytestmark = pytest.mark.gpu


def _no_scratch(passes):
    def check(info):
        assert info["scratch_bytes"] == 0, info
        assert info["n_passes"] == passes, info["desc"]
        assert "transpose" in info["desc"], info["desc"]
    return check


# lengths that do not fit one pass: 128^2 (FP64 only), 256^2, 512^2, 1024^2
@pytest.mark.parametrize("n,prec", [(65536, 0), (262144, 0), (1048576, 0), (16384, 1),
                                    (65536, 1), (1048576, 1)])
@pytest.mark.parametrize("sign", [-1, 1])
def test_square_inplace_without_scratch(n, prec, sign):
    import paper_2602_23525_amd as mfft
    b = 3 if n <= 65536 else 2
    run_case([(n, 1, 1)], [(b, n, n)], prec=prec, sign=sign, inplace=True, seed=n + b,
             name=f"noscratch {n}", flags=mfft.NO_SCRATCH, check_info=_no_scratch(3),
             expect="leaf kernel columns")


# n = 2*q*q: columns of 2q points, rows of q, the two q x q halves transposed,
# then their rows interleaved (an in-place perfect shuffle of 2q runs)
@pytest.mark.parametrize("n,b,prec", [(32768, 3, 0), (32768, 2, 1), (131072, 2, 0),
                                      (2097152, 1, 0), (20000, 3, 0), (131072, 1, 1)])
@pytest.mark.parametrize("sign", [-1, 1])
def test_double_square_inplace_without_scratch(n, b, prec, sign):
    import paper_2602_23525_amd as mfft

    def check(info):
        assert info["scratch_bytes"] == 0, info
        assert info["n_passes"] == 4, info["desc"]
        assert "transpose q=" in info["desc"] and "2x" in info["desc"], info["desc"]
    hd = [(b, n, n)] if b > 1 else []
    run_case([(n, 1, 1)], hd, prec=prec, sign=sign, inplace=True, seed=n + b + 1,
             name=f"noscratch 2q^2 {n}", flags=mfft.NO_SCRATCH, check_info=check)


def test_square_inplace_without_scratch_mixed_radix_and_strided():
    import paper_2602_23525_amd as mfft
    # 90000 = 300^2 (generic kernels), transforms at stride 2 interleaved with
    # a second batch dimension
    run_case([(90000, 1, 1)], [(2, 90000, 90000)], inplace=True, seed=5,
             name="noscratch 300^2", flags=mfft.NO_SCRATCH, check_info=_no_scratch(3))
    run_case([(65536, 2, 2)], [(2, 1, 1), (3, 131072, 131072)], inplace=True, seed=6,
             name="noscratch strided", flags=mfft.NO_SCRATCH, check_info=_no_scratch(3))


def test_multidim_inplace_without_scratch():
    import paper_2602_23525_amd as mfft
    # 2-D 5 x 65536 in place: the long dimension by the square plan, the other
    # as one leaf pass
    run_case([(5, 65536, 65536), (65536, 1, 1)], [], inplace=True, seed=7,
             name="noscratch 2d", flags=mfft.NO_SCRATCH, check_info=_no_scratch(4))


# n = k*q*q for k > 2: columns of k*q points, rows of q, k blocks of q x q
# transposed, then the k x q matrix of q-element runs transposed
@pytest.mark.parametrize("n,b,prec,k", [(49152, 2, 0, 3), (81920, 2, 0, 5), (12288, 3, 1, 3),
                                        (25088, 2, 0, 2), (57344, 1, 0, 14)])
@pytest.mark.parametrize("sign", [-1, 1])
def test_k_square_inplace_without_scratch(n, b, prec, k, sign):
    import paper_2602_23525_amd as mfft

    def check(info):
        assert info["scratch_bytes"] == 0, info
        assert info["n_passes"] == 4, info["desc"]
        assert f"transpose {k}x" in info["desc"], info["desc"]
    hd = [(b, n, n)] if b > 1 else []
    run_case([(n, 1, 1)], hd, prec=prec, sign=sign, inplace=True, seed=n + b + 2,
             name=f"noscratch {k}q^2 {n}", flags=mfft.NO_SCRATCH, check_info=check)


@pytest.mark.parametrize("R,C,outer,prec", [(24, 48, 1, 0), (48, 24, 1, 0), (96, 32, 3, 0),
                                            (32, 96, 2, 1), (64, 64, 2, 0), (7, 21, 1, 1),
                                            (2048, 4096, 1, 0), (1000, 10, 2, 0)])
def test_rank0_transpose_inplace_without_scratch(R, C, outer, prec):
    """An R x C matrix (optionally several) rewritten in place as its
    transpose, with no scratch: square blocks transposed in place, then the
    runs of the shorter side permuted along their cycles; the result is the
    exact transpose."""
    import torch

    import paper_2602_23525_amd as mfft
    cdt = np.complex64 if prec == 0 else np.complex128
    x = uniform_complex(outer * R * C, seed=R * 7 + C, dtype=cdt)
    hd = [(R, C, 1), (C, 1, R)] + ([(outer, R * C, R * C)] if outer > 1 else [])
    p = mfft.Plan([], hd, inplace=True, prec=prec, flags=mfft.NO_SCRATCH)
    info = p.info()
    assert info["scratch_bytes"] == 0, info
    t = torch.from_numpy(x).cuda()
    p.execute(t, t)
    torch.cuda.synchronize()
    want = x.reshape(outer, R, C).transpose(0, 2, 1).reshape(-1)
    assert np.array_equal(t.cpu().numpy(), want), info["desc"]
    p.destroy()


@pytest.mark.parametrize("dims,hdims", [
    ([(30030, 1, 1)], [(2, 30030, 30030)]),          # no k*q*q form with one-pass factors
    ([(65537, 1, 1)], [(2, 65537, 65537)]),          # Rader needs a convolution buffer
    ([(64, 1, 8)], [(8, 64, 1)]),                    # in place, different strides
])
def test_refused_without_scratch(dims, hdims):
    import paper_2602_23525_amd as mfft
    with pytest.raises(mfft.MfftError) as e:
        mfft.Plan(dims, hdims, inplace=True, flags=mfft.NO_SCRATCH)
    assert e.value.code == -2   # MFFT_ENOTSUP


def test_rank0_transpose_refused_without_scratch():
    import paper_2602_23525_amd as mfft
    # 24 x 40: neither side a multiple of the other
    with pytest.raises(mfft.MfftError) as e:
        mfft.Plan([], [(24, 40, 1), (40, 1, 24)], inplace=True, flags=mfft.NO_SCRATCH)
    assert e.value.code == -2


def test_out_of_place_needs_no_scratch():
    import paper_2602_23525_amd as mfft
    p = mfft.Plan([(65536, 1, 1)], [(2, 65536, 65536)], flags=mfft.NO_SCRATCH)
    assert p.info()["scratch_bytes"] == 0 and p.info()["n_passes"] == 2
    p.destroy()


def test_batch_with_a_plan_without_scratch():
    import torch

    import paper_2602_23525_amd as mfft
    n, b = 65536, 2
    x1 = uniform_complex(n * b, seed=21, dtype=np.complex64)
    x2 = uniform_complex(1000 * 3, seed=22, dtype=np.complex64)
    t1 = torch.from_numpy(x1).cuda()
    t2 = torch.from_numpy(x2).cuda()
    y2 = torch.empty_like(t2)
    p1 = mfft.Plan([(n, 1, 1)], [(b, n, n)], inplace=True, flags=mfft.NO_SCRATCH)
    p2 = mfft.Plan([(1000, 1, 1)], [(3, 1000, 1000)])
    bt = mfft.Batch([p1, p2], [t1, t2], [t1, y2], graph=True)
    bt.execute()
    torch.cuda.synchronize()
    r1 = oracle.fft(x1.astype(np.complex128).reshape(b, n))
    r2 = oracle.fft(x2.astype(np.complex128).reshape(3, 1000))
    assert oracle.rel_rms(t1.cpu().numpy().reshape(b, n), r1) <= 2e-6
    assert oracle.rel_rms(y2.cpu().numpy().reshape(3, 1000), r2) <= 2e-6
    bt.destroy()
    p1.destroy()
    p2.destroy()


def test_real_in_place_without_scratch():
    """r2c then c2r in place (rows padded to 2(n/2+1) reals) with the split and
    combine fused into the leaf kernel: no scratch either way."""
    import torch

    import paper_2602_23525_amd as mfft
    n, b = 8192, 3
    h = n // 2 + 1
    rng = np.random.default_rng(31)
    x = rng.uniform(-1, 1, (b, n)).astype(np.float32)
    buf = torch.zeros(b * 2 * h, dtype=torch.float32, device="cuda")
    buf.view(b, 2 * h)[:, :n] = torch.from_numpy(x).cuda()
    f = mfft.Plan([(n, 1, 1)], [(b, 2 * h, h)], inplace=True, kind="r2c", flags=mfft.NO_SCRATCH)
    g = mfft.Plan([(n, 1, 1)], [(b, h, 2 * h)], inplace=True, kind="c2r", flags=mfft.NO_SCRATCH)
    assert f.info()["scratch_bytes"] == 0 and g.info()["scratch_bytes"] == 0
    f.execute(buf, buf)
    torch.cuda.synchronize()
    y = buf.view(torch.complex64).cpu().numpy().reshape(b, h)
    assert oracle.rel_rms(y.astype(np.complex128), oracle.rfft(x.astype(np.float64))) <= 2e-6
    g.execute(buf, buf)
    torch.cuda.synchronize()
    z = buf.cpu().numpy().reshape(b, 2 * h)[:, :n] / n
    assert oracle.rel_rms(z.astype(np.float64), x.astype(np.float64)) <= 4e-6
    f.destroy()
    g.destroy()


def test_real_refused_without_scratch():
    import paper_2602_23525_amd as mfft
    # the inverse of a 2-D real transform runs its complex steps through a
    # packed copy (the input is not overwritten)
    with pytest.raises(mfft.MfftError) as e:
        mfft.Plan([(24, 21, 40), (40, 1, 1)], [], kind="c2r", flags=mfft.NO_SCRATCH)
    assert e.value.code == -2
