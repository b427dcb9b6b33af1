"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle on the
same seeded inputs.  Bounds: relative RMS <= 2e-6 (FP32), <= 1e-13 (FP64,
n <= 2^20).  Output guard bands must stay untouched and out-of-place inputs
unmodified."""
import numpy as np
import pytest

from tests.gpu_util import run_case

pytestmark = pytest.mark.gpu


# ---------------------------------------------------------------- headline shapes

def test_single_1024_fp64_forward_and_roundtrip():
    run_case([(1024, 1, 1)], sign=-1, prec=1, seed=1, method="direct", name="n1024 c64")
    run_case([(1024, 1, 1)], sign=+1, prec=1, seed=2, method="direct", name="n1024 c64 inv")


@pytest.mark.parametrize("sign", [-1, 1])
def test_batched_4096_fp32_small_batch(sign):
    run_case([(4096, 1, 1)], [(64, 4096, 4096)], sign=sign, prec=0, seed=3, name="4096x64")


@pytest.mark.parametrize("sign", [-1, 1])
def test_batched_4096_fp64_small_batch(sign):
    run_case([(4096, 1, 1)], [(8, 4096, 4096)], sign=sign, prec=1, seed=4, name="4096x8 fp64")


@pytest.mark.parametrize("n", [2, 3, 4, 5, 7, 8, 16, 32, 64, 128, 256, 512, 1024, 2048, 4096,
                               6, 9, 10, 12, 14, 15, 21, 25, 27, 30, 35, 49, 60, 100, 210, 243,
                               343, 1000, 2187, 2401, 3125, 18, 36, 45, 63, 90, 126, 150, 225,
                               270, 441, 1008, 1050, 2025, 6144, 14175,
                               11, 13, 22, 26, 121, 143, 169, 1001, 2197, 2288, 3328])
@pytest.mark.parametrize("prec", [0, 1])
def test_leaf_sizes(n, prec):
    b = max(1, min(37, 20000 // n))
    run_case([(n, 1, 1)], [(b, n, n)], sign=-1, prec=prec, seed=n, name=f"leaf {n}")


def _has_wide_radix(info):
    import re
    rads = re.findall(r"rad=([0-9x]+)", info["desc"])
    assert any(int(r) in (17, 19, 23) for rs in rads for r in rs.split("x")), info["desc"]


# radices 17, 19, 23 (the butterflies by paired terms, in the kernel variant
# with 24 elements per thread): one-pass leaves, and two-pass Cooley-Tukey
# lengths whose factors need them
@pytest.mark.parametrize("n", [17, 19, 23, 34, 51, 289, 361, 529, 1088, 2432, 5888, 7429,
                               4 * 17 * 19, 69632, 12167])
@pytest.mark.parametrize("prec", [0, 1])
def test_radices_17_19_23(n, prec):
    b = max(1, min(19, 40000 // n))
    run_case([(n, 1, 1)], [(b, n, n)], sign=-1, prec=prec, seed=n + 5, name=f"wide {n}",
             check_info=_has_wide_radix)
    run_case([(n, 1, 1)], [(b, n, n)], sign=1, prec=prec, seed=n + 6, name=f"wide {n} inv")


def test_wide_radices_strided_and_in_place():
    # columns of a row-major 289 x 96 array (column tiles), a 2-D 19 x 23
    # transform in place, and a 1088-point batch in place
    run_case([(289, 96, 96)], [(96, 1, 1)], seed=71, name="wide columns", check_info=_has_wide_radix)
    run_case([(19, 23, 23), (23, 1, 1)], [(5, 437, 437)], inplace=True, prec=1, seed=72,
             name="wide 2d in place")
    run_case([(1088, 1, 1)], [(7, 1088, 1088)], inplace=True, seed=73, name="wide in place")


def _one_pass_24_per_thread(tpt):
    def check(info):
        d = info["desc"]
        assert info["n_passes"] == 1 and f"tpt={tpt} " in d, d
    return check


# 7-smooth lines of 4097..10240 points that may run with 24 elements per
# thread (512-thread workgroups): FP64 lengths whose 16-per-thread shape needs
# radix 3 (6561) or has no one-pass form (8000) take it always; FP32 lengths
# as the occupancy estimate decides (both forms are checked)
@pytest.mark.parametrize("n,prec,tpt", [(6561, 1, 365), (8000, 1, 400), (5000, 1, 250),
                                        (10000, 0, None), (8000, 0, None), (9000, 0, None),
                                        (4608, 0, None), (10240, 0, None), (6561, 0, None)])
def test_long_smooth_lines(n, prec, tpt):
    b = 4
    chk = _one_pass_24_per_thread(tpt) if tpt else None
    run_case([(n, 1, 1)], [(b, n, n)], sign=-1, prec=prec, seed=n + 11, name=f"long {n}",
             check_info=chk)
    run_case([(n, 1, 1)], [(b, n, n)], sign=1, prec=prec, seed=n + 12, name=f"long {n} inv")


def _smooth_in(lo, hi, count, seed):
    def smooth(v):
        for p in (2, 3, 5, 7):
            while v % p == 0:
                v //= p
        return v == 1
    pool = [v for v in range(lo, hi + 1) if smooth(v) and v & (v - 1)]
    rng = np.random.default_rng(seed)
    return sorted(int(v) for v in rng.choice(pool, count, replace=False))


# a seeded sample of the 7-smooth lengths in 4097..10240 (24 or 16 elements per
# thread as the planner decides, LDS padded once per 64 elements with 24)
@pytest.mark.parametrize("n", _smooth_in(4097, 10240, 12, 5))
@pytest.mark.parametrize("prec", [0, 1])
def test_long_smooth_sample(n, prec):
    run_case([(n, 1, 1)], [(3, n, n)], sign=-1 if n % 2 else 1, prec=prec, seed=n + 13,
             name=f"long sample {n}")


@pytest.mark.parametrize("n", [8192, 14175, 16384, 65536, 100000])
@pytest.mark.parametrize("prec", [0, 1])
def test_cooley_tukey_two_pass(n, prec):
    b = 3
    run_case([(n, 1, 1)], [(b, n, n)], sign=-1, prec=prec, seed=n + 7, name=f"ct {n}")
    run_case([(n, 1, 1)], [(b, n, n)], sign=1, prec=prec, seed=n + 8, name=f"ct {n} inv")


@pytest.mark.parametrize("n", [11, 13, 17, 29, 97, 113, 127, 193, 257, 1009, 2017,
                               23, 53, 79, 157, 859])
@pytest.mark.parametrize("prec", [0, 1])
def test_rader_single_kernel(n, prec):
    # 11, 13, 17, 19, 23 are radices (one butterfly); up to 257 points Rader
    # in one tile; above, Bluestein over a power of two in one leaf-kernel
    # tile is cheaper (same results)
    algo = None if n <= 23 else ("rader n=" if n <= 257 else "bluestein n=")
    run_case([(n, 1, 1)], [(5, n, n)], sign=-1, prec=prec, seed=n, name=f"rader {n}",
             expect=algo)
    run_case([(n, 1, 1)], [(5, n, n)], sign=1, prec=prec, seed=n + 1, name=f"rader {n} inv")


@pytest.mark.parametrize("n", [47, 59, 83, 683, 1013, 2039])   # p - 1 not 13-smooth
@pytest.mark.parametrize("prec", [0, 1])
def test_bluestein_single_kernel(n, prec):
    run_case([(n, 1, 1)], [(5, n, n)], sign=-1, prec=prec, seed=n, name=f"bluestein {n}")
    run_case([(n, 1, 1)], [(5, n, n)], sign=1, prec=prec, seed=n + 1, name=f"bluestein {n} inv")


@pytest.mark.parametrize("n,prec,algo", [
    (65537, 0, "raderA"), (65537, 1, "raderA"), (39937, 0, "raderA"),   # p-1 = 2^10*3*13
    (12289, 0, "rader n=12288"), (39937, 1, None), (65521, 0, None),
    # p-1 smooth but with costly radices (13, 11, 15): Bluestein is cheaper
    (5281, 0, "bluestein n=16384"), (8191, 0, "bluestein"), (8191, 1, "bluesteinA n=128"),
    (8009, 1, "bluesteinA n=128"), (65519, 0, "bluesteinA n=512")])
def test_prime_multi_pass(n, prec, algo):
    run_case([(n, 1, 1)], [(2, n, n)], sign=-1, prec=prec, seed=n, name=f"prime {n}",
             expect=algo)
    run_case([(n, 1, 1)], [(2, n, n)], sign=1, prec=prec, seed=n + 1, name=f"prime {n} inv")


@pytest.mark.parametrize("n,prec,algo", [(16633, 0, "raderB"), (8209, 0, "bluesteinB"),
                                         (10369, 1, "raderB")])
def test_three_pass_prime_with_partial_last_tile(n, prec, algo):
    # regression for the padding-line over-read of the generic tile kernel: the
    # middle pass tiles a column count that is not a multiple of its tile width
    # (16632 = 126 * 132, 132 lines by 16; 18432 = 128 * 144, 144 lines by 32;
    # 10368 = 96 * 108, 108 lines by 8, spectrum and twiddle tables), so the
    # last tile's padding lines take an in-range line's tables (table bounds
    # of every prime plan: the host planner test)
    for sign in (-1, 1):
        run_case([(n, 1, 1)], [(5, n, n)], sign=sign, prec=prec, seed=n + (sign > 0),
                 name=f"three-pass prime {n} partial tile", expect=algo)


@pytest.mark.parametrize("n,algo", [(4093, "bluestein n=8192"), (1213, "bluestein"),
                                    (3011, "bluestein")])
def test_bluestein_length_choice(n, algo):
    # the convolution length is the cheapest candidate, not the shortest:
    # 8190 = 15*14*13*3 loses to 8192
    run_case([(n, 1, 1)], [(3, n, n)], sign=-1, seed=n, name=f"bluestein {n}", expect=algo)


@pytest.mark.parametrize("n,prec,inplace,algo", [
    (37 * 4096, 0, False, "bluestein n=256"), (31 * 1024, 0, True, "rader n=30"),
    (1009 * 16, 0, False, "bluestein n=2048"), (41 * 2048, 1, False, "rader n=40"),
    (43 * 1024, 1, True, "rader n=42"), (47 * 2048, 0, False, "bluestein n=128"),
    (4099 * 8, 0, False, "bluesteinA")])   # second pass too long: Bluestein over n
def test_composite_with_one_large_prime(n, prec, inplace, algo):
    # one prime factor above 23: a Cooley-Tukey step whose second pass is a
    # one-tile prime-size plan (Rader, or Bluestein for 2*37 and 47), not
    # Bluestein over the whole length
    run_case([(n, 1, 1)], [(2, n, n)], prec=prec, inplace=inplace, seed=n, name=f"ct+prime {n}",
             expect=algo)
    run_case([(n, 1, 1)], [(2, n, n)], prec=prec, inplace=inplace, sign=1, seed=n + 1,
             name=f"ct+prime {n} inv")


@pytest.mark.parametrize("n,prec,inplace,hd,algo", [
    (4093, 0, True, (3, 4093, 4093), "bluestein n=8192"),        # one leaf tile, in place
    (4093, 0, False, (5, 4100, 4111), "bluestein n=8192"),       # padded distances
    (2039, 1, False, (7, 2047, 2040), "bluestein n=4096"),       # FP64, 3.5 lines per tile
    (65519, 1, False, (2, 65519, 65519), "bluesteinA n=512"),    # FP64, three leaf passes
    (65519, 0, True, (3, 65519, 65519), "bluesteinA n=512"),     # in place through scratch
    (50021, 0, False, (3, 50030, 50025), "bluesteinA n=512"),    # padded distances
])
def test_bluestein_in_leaf_kernel(n, prec, inplace, hd, algo):
    # Bluestein convolutions over a power of two run in the leaf kernel: the
    # chirp products with zero padding and truncation, the spectrum product
    # between two transforms, in one tile or three column-tile passes
    if inplace:
        hd = (hd[0], hd[1], hd[1])
    run_case([(n, 1, 1)], [hd], prec=prec, inplace=inplace, seed=n + hd[0], name=f"bl {n}",
             expect=algo)
    run_case([(n, 1, 1)], [hd], prec=prec, inplace=inplace, sign=1, seed=n + hd[0] + 1,
             name=f"bl {n} inv")


# ---------------------------------------------------------------- strides, ranks, in-place

def test_columns_and_rows_examples():
    n1, n2 = 48, 80
    # rows in place: dft({(n2,1,1)}, {(n1,n2,n2)}, X, X)
    run_case([(n2, 1, 1)], [(n1, n2, n2)], inplace=True, seed=11, name="rows ip")
    # columns in place: dft({(n1,n2,n2)}, {(n2,1,1)}, X, X)
    run_case([(n1, n2, n2)], [(n2, 1, 1)], inplace=True, seed=12, name="cols ip")
    run_case([(n1, n2, n2)], [(n2, 1, 1)], inplace=True, prec=1, seed=13, name="cols ip c64")


@pytest.mark.parametrize("n", [64, 128, 256, 512, 1024, 2048])
@pytest.mark.parametrize("prec", [0, 1])
def test_column_tiles(n, prec):
    # columns of a row-major array (element stride = row length, adjacent
    # lines): the leaf kernel with column tiles; row counts that leave a
    # partial last tile, an outer loop, in place, and a wider row than the
    # columns transformed
    C = 37
    run_case([(n, C, C)], [(C, 1, 1)], prec=prec, seed=n + 1, name=f"cols {n}",
             expect="leaf kernel columns")
    run_case([(n, C, C)], [(2, n * C, n * C), (C, 1, 1)], prec=prec, inplace=True,
             seed=n + 2, name=f"cols ip outer {n}", expect="leaf kernel columns")
    run_case([(n, 50, 40)], [(21, 1, 1)], prec=prec, sign=1, seed=n + 3,
             name=f"cols strided {n}", expect="leaf kernel columns")


@pytest.mark.parametrize("n", [256, 512, 1024, 2048])
@pytest.mark.parametrize("prec", [0, 1])
def test_transposing_column_tiles(n, prec):
    # one side adjacent lines, the other unit-stride lines: columns in and
    # rows out, rows in and columns out (partial last tiles: 37 lines)
    C = 37
    run_case([(n, C, 1)], [(C, 1, n)], prec=prec, seed=n + 4, name=f"cols->rows {n}",
             expect="leaf kernel columns->rows")
    run_case([(n, 1, C)], [(C, n, 1)], prec=prec, sign=1, seed=n + 5,
             name=f"rows->cols {n}", expect="leaf kernel rows->columns")


@pytest.mark.parametrize("n", [65536, 131072, 1048576])
@pytest.mark.parametrize("prec", [0, 1])
def test_two_pass_twiddled_column_tiles(n, prec):
    # first Cooley-Tukey pass: columns in, rows out, times w_N^(c*k)
    run_case([(n, 1, 1)], [(2, n, n)], prec=prec, seed=n + 6, name=f"ct {n}",
             expect="leaf kernel columns->rows")


def test_3d_inplace_small():
    n = 32
    dims = [(n, n * n, n * n), (n, n, n), (n, 1, 1)]
    run_case(dims, inplace=True, seed=14, name="3d ip")
    run_case(dims, inplace=True, sign=1, seed=15, name="3d ip inv")


def test_2d_transposed_output_fp64():
    n = 128
    run_case([(n, n, 1), (n, 1, n)], prec=1, seed=16, name="2d transposed")
    run_case([(n, n, 1), (n, 1, n)], prec=0, seed=17, name="2d transposed c32")


def test_2d_transposed_inplace_uses_snapshot():
    n = 64
    run_case([(n, n, 1), (n, 1, n)], prec=0, inplace=True, seed=18, name="2d transposed ip")


def test_general_strides_and_negative():
    run_case([(12, 3, -5)], [(4, 40, 1), (3, 7, 100)], seed=19, name="odd strides")
    run_case([(64, -1, 1)], [(5, 64, 64)], seed=20, name="negative input stride")
    run_case([(30, 2, 3)], [(7, 61, 97)], prec=1, seed=21, name="strided c64")


def test_rank0_copy_and_transpose():
    run_case([], [(1000, 1, 1)], seed=22, name="rank0 copy")
    run_case([], [(24, 40, 1), (40, 1, 24)], inplace=True, seed=23, name="rank0 ip transpose")


def test_degenerate_sizes():
    run_case([(1, 1, 1)], [(50, 1, 1)], seed=24, name="n=1")
    run_case([(0, 1, 1)], [(50, 1, 1)], seed=25, name="n=0", check_guard=True)
    run_case([(256, 1, 1)], [(0, 256, 256)], seed=26, name="empty vector")


def test_multidim_mixed_sizes():
    run_case([(12, 35, 35), (35, 1, 1)], [(3, 420, 420)], seed=27, name="12x35 batched")
    run_case([(7, 600, 600), (6, 100, 100), (100, 1, 1)], prec=1, seed=28, name="7x6x100")


def test_bitwise_determinism():
    import torch

    import paper_2602_23525_amd as mfft
    from synth import uniform_complex
    x = torch.from_numpy(uniform_complex(4096 * 32, seed=29, dtype=np.complex64)).cuda()
    y1 = torch.empty_like(x)
    y2 = torch.empty_like(x)
    p = mfft.Plan([(4096, 1, 1)], [(32, 4096, 4096)])
    p.execute(x, y1)
    p.execute(x, y2)
    torch.cuda.synchronize()
    assert torch.equal(y1, y2)
