"""CPU checks of the C-ABI library: it loads without a GPU, exports every
function include/mfft.h declares, and its host-only problem validation follows
the problem statement of Section 4.1 (non-negative lengths, integer strides)
plus the library's conventions (sign +-1, no aliasing outputs)."""


import pytest

import paper_2602_23525_amd as mfft

OK, EINVAL, ENOTSUP = 0, -1, -2


def test_library_exports_every_header_function():
    names = mfft.header_functions()
    assert "mfft_plan_dft" in names and "mfft_execute" in names
    L = mfft.lib()
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing
    assert mfft.mfft_version().startswith("mfft")


def test_header_declares_extern_c_block():
    text = open(mfft.HEADER_PATH).read()
    assert 'extern "C"' in text
    assert "typedef struct" in text and "mfft_iodim" in text


@pytest.mark.parametrize("dims,hdims,inplace,sign,prec,expect", [
    ([(1024, 1, 1)], [], 0, -1, 0, OK),
    ([(4096, 1, 1)], [(16384, 4096, 4096)], 0, -1, 0, OK),
    ([(256, 65536, 65536), (256, 256, 256), (256, 1, 1)], [], 1, 1, 0, OK),
    ([(2048, 2048, 1), (2048, 1, 2048)], [], 0, -1, 1, OK),
    ([(0, 1, 1)], [(5, 1, 1)], 0, -1, 0, OK),              # n = 0: valid no-op
    ([], [(10, 1, 1)], 0, -1, 0, OK),                      # rank 0: copy
    ([], [(6, 10, 1), (10, 1, 6)], 1, -1, 0, OK),          # in-place transpose
    ([(8, -1, 1)], [], 0, -1, 0, OK),                      # negative stride
    ([(-1, 1, 1)], [], 0, -1, 0, EINVAL),                  # negative length
    ([(8, 1, 1)], [], 0, 0, 0, EINVAL),                    # sign must be +-1
    ([(8, 1, 1)], [], 0, 2, 0, EINVAL),
    ([(8, 1, 1)], [], 0, -1, 7, EINVAL),                   # unknown precision
    ([(8, 1, 1)], [], 2, -1, 0, EINVAL),                   # inplace flag
    ([(8, 1, 0)], [], 0, -1, 0, EINVAL),                   # zero output stride aliases
    ([(8, 1, 1)], [(4, 8, 4)], 0, -1, 0, EINVAL),          # overlapping outputs
    ([(8, 0, 1)], [], 0, -1, 0, OK),                       # zero input stride: broadcast read
    ([(1 << 41, 1, 1)], [], 0, -1, 0, EINVAL),             # too large
    ([(1 << 30, 1 << 40, 1)], [], 0, -1, 0, EINVAL),       # stride * length overflows
    ([(2, 1, 1)] * 9, [], 0, -1, 0, EINVAL),               # rank above 8
    # above 2^22 elements, interleaved strides that fail the span test but
    # never collide (5a + 2b < 16 for a < 2, b < 5): legal
    ([(5, 2, 2), (2, 5, 5)], [(1 << 21, 16, 16)], 0, -1, 0, OK),
    # the same size with a collision (3*2 = 2*3): aliasing
    ([(4, 3, 3), (4, 2, 2)], [(1 << 20, 64, 64)], 0, -1, 0, EINVAL),
])
def test_problem_check(dims, hdims, inplace, sign, prec, expect):
    assert mfft.mfft_problem_check(dims, hdims, inplace, sign, prec) == expect


def test_problem_check_null_pointers():
    L = mfft.lib()
    assert L.mfft_problem_check(1, None, 0, None, 0, -1, 0) == EINVAL
    assert L.mfft_problem_check(0, None, 0, None, 0, -1, 0) == OK
    assert L.mfft_problem_check(0, None, 1, None, 0, -1, 0) == EINVAL


def test_error_text_is_thread_local_string():
    assert mfft.mfft_problem_check([(8, 1, 1)], [], 0, 3, 0) == EINVAL
    assert "sign" in mfft.mfft_last_error()


def test_plan_without_gpu_fails_cleanly():
    import torch
    if torch.cuda.is_available():
        pytest.skip("GPU present")
    with pytest.raises(mfft.MfftError) as e:
        mfft.mfft_plan_dft([(64, 1, 1)], stream=0)
    assert e.value.code == -4      # MFFT_EHIP


@pytest.mark.parametrize("flags,prec", [(32, 0), (1 << 31, 0), (8, 1)])
def test_plan_rejects_bad_flags_before_device_work(flags, prec):
    # unknown flag bits, and the FP32-twiddle ablation on an FP64 plan
    with pytest.raises(mfft.MfftError) as e:
        mfft.mfft_plan_dft([(64, 1, 1)], prec=prec, flags=flags, stream=0)
    assert e.value.code == EINVAL
    assert "flag" in mfft.mfft_last_error() or "FP32" in mfft.mfft_last_error()


def test_wisdom_roundtrip_text():
    mfft.mfft_wisdom_forget()
    text = mfft.mfft_wisdom_export()
    assert text.startswith("mfft-wisdom 1 ")
    mfft.mfft_wisdom_import(text + "c32 s-1 op N:64,1,1 V => emax=16 bt=4\n")
    assert "N:64,1,1" in mfft.mfft_wisdom_export()
    with pytest.raises(mfft.MfftError):
        mfft.mfft_wisdom_import("garbage")
    mfft.mfft_wisdom_forget()
    assert "N:64" not in mfft.mfft_wisdom_export()


@pytest.mark.parametrize("kind,dims,hdims,inplace,prec,expect", [
    ("r2c", [(16, 1, 1)], [(4, 16, 9)], 0, 0, 0),
    ("c2r", [(16, 1, 1)], [(4, 9, 16)], 0, 1, 0),
    ("r2c", [(17, 1, 1)], [], 0, 0, 0),
    ("r2c", [(8, 5, 5), (8, 1, 1)], [], 0, 0, 0),         # rank 2, last dim halved
    ("r2c", [(8, 5, 4), (8, 1, 1)], [], 0, 0, -1),        # 5 outputs per row at distance 4
    ("c2r", [], [], 0, 0, -1),                            # rank 0
    ("r2c", [(16, 1, 1)], [(4, 16, 4)], 0, 0, -1),        # 9 outputs per row at distance 4 alias
    ("c2r", [(16, 1, 1)], [(4, 9, 8)], 0, 0, -1),         # 16 real outputs at distance 8 alias
    ("r2c", [(-1, 1, 1)], [], 0, 0, -1),
    ("r2c", [(0, 1, 1)], [(3, 1, 1)], 0, 0, 0),           # empty
])
def test_problem_check_real(kind, dims, hdims, inplace, prec, expect):
    assert mfft.mfft_problem_check_real(kind, dims, hdims, inplace, prec) == expect


def test_flag_constants_match_header():
    import re
    text = open(mfft.HEADER_PATH).read()
    for name in ("MEASURE", "WISDOM_ONLY", "NO_WISDOM", "FP32_TWIDDLES", "NO_SCRATCH"):
        m = re.search(r"#define MFFT_%s +(\d+)u" % name, text)
        assert m, name
        assert int(m.group(1)) == getattr(mfft, name), name


def _collides(dims):
    seen = set()
    idx = [0] * len(dims)
    while True:
        off = sum(i * d[2] for i, d in zip(idx, dims))
        if off in seen:
            return True
        seen.add(off)
        j = 0
        while j < len(dims):
            idx[j] += 1
            if idx[j] < dims[j][0]:
                break
            idx[j] = 0
            j += 1
        if j == len(dims):
            return False


def test_aliasing_check_is_exact_on_random_layouts():
    # small output layouts with arbitrary strides: the library's answer equals
    # brute-force enumeration of every output address
    import random
    rng = random.Random(5)
    seen_ok = seen_bad = 0
    for _ in range(600):
        k = rng.randint(1, 4)
        dims = [(rng.randint(2, 6), 1, rng.choice([-1, 1]) * rng.randint(1, 12)) for _ in range(k)]
        want = EINVAL if _collides(dims) else OK
        got = mfft.mfft_problem_check(dims[:1], dims[1:], 0, -1, 0)
        assert got == want, (dims, got, want)
        seen_ok += want == OK
        seen_bad += want == EINVAL
    assert seen_ok > 100 and seen_bad > 100


def test_plan_info_struct_matches_header(tmp_path):
    """The binding's PlanInfo has the header's mfft_plan_info_t layout: size and
    the offsets of the last fields, from a C program built against the header."""
    import ctypes
    import os
    import shutil
    import subprocess
    if shutil.which("gcc") is None:
        pytest.skip("no gcc")
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    src = tmp_path / "info.c"
    src.write_text(
        "#include <stddef.h>\n#include <stdio.h>\n#include \"mfft.h\"\n"
        "int main(void){printf(\"%zu %zu %zu %zu\\n\", sizeof(mfft_plan_info_t),"
        " offsetof(mfft_plan_info_t, desc), offsetof(mfft_plan_info_t, n_radices),"
        " offsetof(mfft_plan_info_t, radices));return 0;}\n")
    exe = str(tmp_path / "info")
    subprocess.run(["gcc", "-I", os.path.join(root, "include"), str(src), "-o", exe], check=True)
    size, desc, nrad, rad = map(int, subprocess.run([exe], capture_output=True, text=True,
                                                    check=True).stdout.split())
    P = mfft.PlanInfo
    assert (ctypes.sizeof(P), P.desc.offset, P.n_radices.offset, P.radices.offset) == \
        (size, desc, nrad, rad)
