"""GPU tests of the planner modes (Section 4.3): estimate, measure, stored
plans ("wisdom"), and the plan description."""
import numpy as np
import pytest

import oracle
from synth import uniform_complex

pytestmark = pytest.mark.gpu


def _run(plan, x):
    import torch
    xt = torch.from_numpy(x).cuda()
    yt = torch.empty_like(xt)
    plan.execute(xt, yt)
    torch.cuda.synchronize()
    return yt.cpu().numpy()


def test_measure_wisdom_roundtrip():
    import paper_2602_23525_amd as mfft
    n, b = 1024, 2048
    x = uniform_complex(n * b, seed=41, dtype=np.complex64)
    ref = oracle.fft(x.astype(np.complex128).reshape(b, n))
    mfft.mfft_wisdom_forget()
    with pytest.raises(mfft.MfftError) as e:
        mfft.Plan([(n, 1, 1)], [(b, n, n)], flags=mfft.WISDOM_ONLY)
    assert e.value.code == -10
    pm = mfft.Plan([(n, 1, 1)], [(b, n, n)], flags=mfft.MEASURE)
    ym = _run(pm, x)
    assert oracle.rel_rms(ym.reshape(b, n), ref) <= 2e-6
    text = mfft.mfft_wisdom_export()
    assert "N:1024,1,1" in text
    mfft.mfft_wisdom_forget()
    mfft.mfft_wisdom_import(text)
    pw = mfft.Plan([(n, 1, 1)], [(b, n, n)], flags=mfft.WISDOM_ONLY)
    assert "choices from wisdom" in pw.info()["desc"]
    yw = _run(pw, x)
    assert np.array_equal(ym, yw), "same stored choices must give identical bits"
    pe = mfft.Plan([(n, 1, 1)], [(b, n, n)], flags=mfft.ESTIMATE | mfft.NO_WISDOM)
    ye = _run(pe, x)
    assert oracle.rel_rms(ye.reshape(b, n), ref) <= 2e-6
    for p in (pm, pw, pe):
        p.destroy()
    mfft.mfft_wisdom_forget()


def test_plan_info_counts():
    import paper_2602_23525_amd as mfft
    p = mfft.Plan([(4096, 1, 1)], [(64, 4096, 4096)])
    info = p.info()
    assert info["n_passes"] == 1 and info["howmany"] == 64 and info["n_total"] == 4096
    assert info["flops"] == pytest.approx(5 * 4096 * 12 * 64)
    assert info["bytes_compulsory"] == pytest.approx(2 * 8 * 4096 * 64)
    assert "leaf kernel" in info["desc"]
    p.destroy()
    p = mfft.Plan([(65536, 1, 1)], [(4, 65536, 65536)])
    assert p.info()["n_passes"] == 2
    p.destroy()


def test_execute_argument_checks():
    import torch

    import paper_2602_23525_amd as mfft
    p = mfft.Plan([(256, 1, 1)], [(4, 256, 256)])
    x = torch.zeros(1024, dtype=torch.complex64, device="cuda")
    with pytest.raises(mfft.MfftError) as e:
        p.execute(x, x)                       # out-of-place plan, in == out
    assert e.value.code == -5
    with pytest.raises(mfft.MfftError) as e:
        mfft.mfft_execute(p.handle, x.data_ptr() + 4, x.data_ptr() + 8192)   # misaligned
    assert e.value.code == -5
    p.destroy()
    q = mfft.Plan([(256, 1, 1)], [(4, 256, 256)], inplace=True)
    y = torch.zeros(1024, dtype=torch.complex64, device="cuda")
    with pytest.raises(mfft.MfftError):
        q.execute(x, y)                       # in-place plan, in != out
    q.destroy()


def test_torch_allocator_plan():
    import torch

    import paper_2602_23525_amd as mfft
    alloc = mfft.torch_allocator()
    n = 65536
    x = uniform_complex(n * 2, seed=43, dtype=np.complex64)
    p = mfft.Plan([(n, 1, 1)], [(2, n, n)], inplace=True, allocator=alloc)
    xt = torch.from_numpy(x).cuda()
    p.execute(xt, xt)
    torch.cuda.synchronize()
    ref = oracle.fft(x.astype(np.complex128).reshape(2, n))
    assert oracle.rel_rms(xt.cpu().numpy().reshape(2, n), ref) <= 2e-6
    assert p.info()["scratch_bytes"] > 0
    p.destroy()


def test_fp32_twiddle_ablation_is_less_accurate():
    """Section 6: twiddles must be accurate.  Stage tables evaluated in FP32
    arithmetic (the ablation flag) are no more accurate than FP64 tables
    rounded once, and both stay near FP32 precision."""
    import torch

    import paper_2602_23525_amd as mfft
    n, b = 4096, 64
    x = uniform_complex(n * b, seed=31, dtype=np.complex64)
    xt = torch.from_numpy(x).cuda()
    ref = oracle.fft(x.astype(np.complex128).reshape(b, n))
    errs = {}
    for flags in (mfft.NO_WISDOM, mfft.NO_WISDOM | mfft.FP32_TWIDDLES):
        yt = torch.empty_like(xt)
        p = mfft.Plan([(n, 1, 1)], [(b, n, n)], flags=flags)
        p.execute(xt, yt)
        torch.cuda.synchronize()
        p.destroy()
        errs[flags] = oracle.rel_rms(yt.cpu().numpy().reshape(b, n), ref)
    e64, e32 = errs[mfft.NO_WISDOM], errs[mfft.NO_WISDOM | mfft.FP32_TWIDDLES]
    print(f"relRMS FP64-generated twiddles {e64:.3e}, FP32-evaluated twiddles {e32:.3e}")
    assert e64 <= 2e-6 and e32 <= 1e-5
    assert e64 <= 1.05 * e32


# Every specialized leaf kernel variant (prefetch, occupancy floor of 2, 3 or 4
# waves, non-temporal access) and grid kind, forced through stored choices,
# on batches that leave a partial last tile and, with the persistent grid,
# give workgroups more than one tile.
LEAF_VARIANTS = [0, 1, 3, 5, 8, 9, 11, 13, 24, 25, 27, 29]


@pytest.mark.parametrize("n,b,prec", [(64, 1000, 0), (256, 999, 0), (1024, 1001, 0),
                                      (2048, 1003, 0), (4096, 1100, 0), (512, 777, 1),
                                      (4096, 1029, 1), (8192, 600, 0), (16384, 300, 0),
                                      (8192, 301, 1)])
def test_every_leaf_variant(n, b, prec):
    import paper_2602_23525_amd as mfft
    cdt = np.complex64 if prec == 0 else np.complex128
    x = uniform_complex(n * b, seed=n + b, dtype=cdt)
    ref = oracle.fft(x.astype(np.complex128).reshape(b, n))
    tol = 2e-6 if prec == 0 else 1e-13
    mfft.mfft_wisdom_forget()
    p = mfft.Plan([(n, 1, 1)], [(b, n, n)], prec=prec, flags=mfft.MEASURE)
    key = mfft.mfft_wisdom_export().strip().split("\n")[1].split(" => ")[0]
    p.destroy()
    for v in LEAF_VARIANTS:
        for pe in (0, 1):
            mfft.mfft_wisdom_forget()
            mfft.mfft_wisdom_import(f"mfft-wisdom 1 {mfft.mfft_version()}\n{key} => 0:v{v}p{pe}\n")
            p = mfft.Plan([(n, 1, 1)], [(b, n, n)], prec=prec, flags=mfft.WISDOM_ONLY)
            assert "choices from wisdom" in p.info()["desc"]
            y = _run(p, x)
            p.destroy()
            err = oracle.rel_rms(y.reshape(b, n), ref)
            assert err <= tol, (n, b, prec, v, pe, err)
    mfft.mfft_wisdom_forget()


def _wisdom_lines():
    import paper_2602_23525_amd as mfft
    return dict(line.split(" => ") for line in mfft.mfft_wisdom_export().strip().split("\n")[1:])


@pytest.mark.parametrize("n,b,prec,field", [(1000, 4096, 0, ":r="), (2187, 1024, 1, ":r="),
                                            (65537, 64, 0, ":a="), (4099, 256, 0, ":a="),
                                            (100000, 32, 0, ":s=")])
def test_measured_structure_is_stored_and_reused(n, b, prec, field):
    """Measure mode times structural alternatives (radix sequence and lines per
    tile of a generic leaf, Cooley-Tukey split, Rader or Bluestein and its
    length) and stores the winner per problem and per transform length; a
    wisdom-only plan rebuilt from the text gives identical bits, also for
    another batch count of the same length."""
    import paper_2602_23525_amd as mfft
    cdt = np.complex64 if prec == 0 else np.complex128
    tol = 2e-6 if prec == 0 else 1e-13
    x = uniform_complex(n * b, seed=n + 3, dtype=cdt)
    rows = [0, b - 1]
    ref = oracle.fft(x.astype(np.complex128).reshape(b, n)[rows])
    mfft.mfft_wisdom_forget()
    pm = mfft.Plan([(n, 1, 1)], [(b, n, n)], prec=prec, flags=mfft.MEASURE)
    ym = _run(pm, x)
    assert oracle.rel_rms(ym.reshape(b, n)[rows], ref) <= tol
    w = _wisdom_lines()
    line = [v for k, v in w.items() if k.startswith(f"line c{32 if prec == 0 else 64} n={n} ")]
    assert len(line) == 1 and line[0].startswith(f"n={n}") and field in line[0], w
    prob = [v for k, v in w.items() if not k.startswith("line ")]
    assert len(prob) == 1 and field in prob[0].split("|")[0], w
    text = mfft.mfft_wisdom_export()
    mfft.mfft_wisdom_forget()
    mfft.mfft_wisdom_import(text)
    pw = mfft.Plan([(n, 1, 1)], [(b, n, n)], prec=prec, flags=mfft.WISDOM_ONLY)
    assert "choices from wisdom" in pw.info()["desc"]
    assert pw.info()["desc"].replace("  (choices from wisdom)\n", "") == pm.info()["desc"]
    assert np.array_equal(_run(pw, x), ym), "stored structure must give identical bits"
    # the per-length entry plans the same length with another batch count
    b2 = 3
    pb = mfft.Plan([(n, 1, 1)], [(b2, n, n)], prec=prec, flags=mfft.WISDOM_ONLY)
    y2 = _run(pb, x[: n * b2])
    assert oracle.rel_rms(y2.reshape(b2, n)[:1], ref[:1]) <= tol
    for p in (pm, pw, pb):
        p.destroy()
    mfft.mfft_wisdom_forget()


def test_forced_radices_of_fig3_compute_the_dft():
    """The Fig. 3 plan of n = 30 (DIT radices 3, 2, 5; Stockham stages 5, 2, 3)
    given as a stored structural choice computes the DFT (FP64)."""
    import paper_2602_23525_amd as mfft
    n, b = 30, 7
    x = uniform_complex(n * b, seed=30, dtype=np.complex128)
    ref = oracle.fft(x.reshape(b, n))
    mfft.mfft_wisdom_forget()
    mfft.Plan([(n, 1, 1)], [(b, n, n)], prec=1, flags=mfft.MEASURE).destroy()
    key = [k for k in _wisdom_lines() if k.startswith("line c64 n=30 ")][0]
    mfft.mfft_wisdom_forget()
    mfft.mfft_wisdom_import(f"mfft-wisdom 1 {mfft.mfft_version()}\n{key} => n=30:r=5.2.3\n")
    p = mfft.Plan([(n, 1, 1)], [(b, n, n)], prec=1, flags=mfft.WISDOM_ONLY)
    assert "rad=5x2x3" in p.info()["desc"], p.info()["desc"]
    y = _run(p, x)
    assert oracle.rel_rms(y.reshape(b, n), ref) <= 1e-13
    p.destroy()
    mfft.mfft_wisdom_forget()


@pytest.mark.parametrize("emax,tpt", [(16, 1000), (24, 500)])
def test_forced_elements_per_thread_compute_the_dft(emax, tpt):
    """10000-point FP32 lines with 16 or 24 elements per thread (a structural
    choice stored as wisdom, ":e=16" / ":e=24") both compute the DFT."""
    import paper_2602_23525_amd as mfft
    n, b = 10000, 4
    x = uniform_complex(n * b, seed=77, dtype=np.complex64)
    ref = oracle.fft(x.astype(np.complex128).reshape(b, n))
    mfft.mfft_wisdom_forget()
    mfft.Plan([(n, 1, 1)], [(b, n, n)], flags=mfft.MEASURE).destroy()
    key = [k for k in _wisdom_lines() if k.startswith(f"line c32 n={n} ")][0]
    mfft.mfft_wisdom_forget()
    mfft.mfft_wisdom_import(f"mfft-wisdom 1 {mfft.mfft_version()}\n{key} => n={n}:e={emax}\n")
    p = mfft.Plan([(n, 1, 1)], [(b, n, n)], flags=mfft.WISDOM_ONLY)
    assert f"tpt={tpt} " in p.info()["desc"], p.info()["desc"]
    y = _run(p, x)
    assert oracle.rel_rms(y.reshape(b, n), ref) <= 2e-6
    p.destroy()
    mfft.mfft_wisdom_forget()


def test_plan_info_lists_each_pass_radices():
    """mfft_plan_info reports the radices each pass executes (Stockham stages in
    order; the leaf kernel's own sequence for its passes), one list per pass."""
    import paper_2602_23525_amd as mfft
    cases = [([(4096, 1, 1)], [(16, 4096, 4096)], 0, [[16, 16, 16]]),
             ([(8192, 1, 1)], [(4, 8192, 8192)], 0, [[16, 16, 16, 2]]),
             ([(1000, 1, 1)], [(8, 1000, 1000)], 0, [[10, 10, 10]]),
             ([(65536, 1, 1)], [(4, 65536, 65536)], 0, None)]
    for dims, hd, prec, want in cases:
        p = mfft.Plan(dims, hd, prec=prec)
        info = p.info()
        rad = info["radices"]
        assert len(rad) == info["n_passes"], (rad, info["desc"])
        for r in rad:
            assert r and all(x in (2, 3, 4, 5, 6, 7, 8, 9, 10, 11, 12, 13, 14, 15, 16, 17, 19, 23)
                             for x in r), rad
        # the passes' radices multiply to the transform length
        assert int(np.prod([int(np.prod(r)) for r in rad])) == dims[0][0], rad
        if want is not None:
            assert rad == want, (rad, info["desc"])
        p.destroy()
