"""The planner and the problem canonicalization compiled for the host with g++
(tests/host_stub stands in for the HIP runtime: tables are address ranges,
launches do nothing), so that every plan the library would make can be
inspected on the CPU:

  * table bounds: for each pass, the largest index any lane forms in each table
    (gather/scatter, pre/post multipliers, convolution spectrum, two-level
    twiddles, stage twiddles, Rader's per-transform terms), padding lines of a
    partial last tile included, lies inside the table
    (tests/plan_host_check.cpp), for every prime from 67 to 65521 in both
    precisions -- the three-pass Rader / Bluestein plans whose column count is
    not a multiple of the tile width among them, the case of the padding-line
    over-read fixed in the generic tile kernel -- and for every length up to
    4096 and sampled composite lengths above;
  * every structural alternative measure mode would time plans and stays in
    bounds, and its wisdom text reads back unchanged;
  * the same planner (and the oracle's C code) under AddressSanitizer and
    UndefinedBehaviorSanitizer, on prime ranges, measure candidates and seeded
    random problems (strided, transposed, reversed, in place, aliasing)."""
import os
import re
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(ROOT, "paper_2602_23525_amd", "csrc")
SOURCES = [os.path.join(HERE, "plan_host_check.cpp"), os.path.join(CSRC, "plan.cpp"),
           os.path.join(CSRC, "problem.cpp")]
INC = ["-I", os.path.join(HERE, "host_stub"), "-I", CSRC, "-I", os.path.join(ROOT, "include")]
SAN = ["-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all"]

pytestmark = pytest.mark.skipif(shutil.which("g++") is None, reason="no host C++ compiler")


@pytest.fixture(scope="module")
def checker(tmp_path_factory):
    exe = str(tmp_path_factory.mktemp("planhost") / "plan_host_check")
    subprocess.run(["g++", "-std=c++17", "-O2", *INC, *SOURCES, "-o", exe], check=True)
    return exe


@pytest.fixture(scope="module")
def checker_san(tmp_path_factory):
    exe = str(tmp_path_factory.mktemp("planhost_san") / "plan_host_check")
    subprocess.run(["g++", "-std=c++17", *SAN, *INC, *SOURCES, "-o", exe], check=True)
    return exe


def _run(exe, *args, env=None):
    r = subprocess.run([exe, *map(str, args)], capture_output=True, text=True, env=env)
    summary = r.stdout.strip().splitlines()[-1] if r.stdout.strip() else ""
    print(summary)
    assert r.returncode == 0, (r.stdout[-4000:], r.stderr[-4000:])
    assert "VIOLATION" not in r.stdout and "runtime error" not in r.stderr, r.stderr[-4000:]
    return r.stdout, dict((k, int(v)) for k, v in re.findall(r"(\w+)=(\d+)", summary))


@pytest.mark.parametrize("prec", [0, 1])
def test_prime_plans_stay_inside_their_tables(checker, prec):
    out, s = _run(checker, "bounds", prec, 67, 65521, 2, "primes")
    assert s["plans"] == 6524 and s["violations"] == 0 and s["failed"] == 0
    # multi-pass prime plans with a partial last column tile exist, and their
    # padding lines would read past the spectrum without the clamp
    assert s["partial"] > 50 and s["guarded"] > 20
    if prec == 0:
        # p = 16633: Rader, L = 16632 = 126 * 132, the middle pass tiles 132
        # lines by 16
        assert re.search(r"GUARDED n=16633 c32: conv .*raderB", out)
        # p = 8209: Bluestein, M = 18432 = 128 * 144, 144 lines by 32
        assert re.search(r"GUARDED n=8209 c32: conv .*bluesteinB", out)
    else:
        # p = 10369: Rader, L = 10368 = 96 * 108, 108 lines by 8 (spectrum and
        # two-level twiddles)
        assert re.search(r"GUARDED n=10369 c64: tw4_hi .*raderB", out)


@pytest.mark.parametrize("prec", [0, 1])
def test_every_length_to_4096_stays_inside_its_tables(checker, prec):
    _, s = _run(checker, "bounds", prec, 1, 4096, 3, "all")
    assert s["violations"] == 0 and s["failed"] == 0 and s["plans"] == 4096


def test_sampled_composite_lengths_stay_inside_their_tables(checker):
    for lo in (4097, 16000, 40000, 65530):
        _, s = _run(checker, "bounds", 0, lo, lo + 400, 2, "composite")
        assert s["violations"] == 0 and s["failed"] == 0


@pytest.mark.parametrize("prec,lo,hi", [(0, 2, 4096), (1, 2, 4096), (0, 60000, 65536)])
def test_measure_candidates_plan_and_stay_inside_their_tables(checker, prec, lo, hi):
    # every structural alternative measure mode times (radix sequences, lines
    # per tile, Cooley-Tukey splits, Rader or Bluestein and its length) plans,
    # keeps its table reads in bounds, and its wisdom text reads back the same
    _, s = _run(checker, "cands", prec, lo, hi, 3)
    assert s["violations"] == 0 and s["failed"] == 0 and s["candidates"] > s["lengths"]


@pytest.mark.parametrize("prec,n,rad", [(0, 8192, "16.8.8.8"), (0, 16384, "4.16.16.16"),
                                         (1, 8192, "8.8.8.16"), (0, 1024, "4.4.4.4.4"),
                                         (0, 2048, "2.16.4.16")])
def test_forced_radices_keep_the_leaf_kernels_table(checker, prec, n, rad):
    """A power-of-two length runs in the specialized leaf kernel, whose stage
    twiddle table is laid out for its own radix sequence (radix-16 stages,
    then 2^(e mod 4)).  A structure imported as wisdom that names another
    sequence for the length changes the generic shape only: the leaf kernel's
    table still covers what the kernel reads (a table laid out for 16.8.8.8
    holds 9360 entries where the kernel reads up to index 12559)."""
    r = subprocess.run([checker, "forced", str(prec), str(n), "r=" + rad, "4"],
                       capture_output=True, text=True)
    print(r.stdout[-2000:])
    assert r.returncode == 0 and "VIOLATION" not in r.stdout, r.stdout + r.stderr
    assert "kernel=1" in r.stdout   # the specialized leaf kernel runs it


@pytest.mark.parametrize("prec,n,batch,bt", [(0, 98, 65536, 36), (0, 1000, 16384, 5),
                                              (0, 60, 131072, 64), (0, 144, 65536, 21),
                                              (1, 1000, 8192, 2)])
def test_lines_per_row_tile_keep_most_lanes_resident(checker, prec, n, batch, bt):
    """Lines per row tile come from the 256/512/1024-thread class that keeps the
    most working lanes resident per CU (lines x threads x workgroups per CU;
    here the checker's model of the occupancy query: registers of the plain
    FP32 kernel allow 6 waves per SIMD, FP64 3, and 160 KB of LDS per CU).
    98 points: 36 lines (252 of 256 threads, five per CU) rather than 73 (511
    of 512, two per CU); 1000 points FP32: 5 lines of 100 threads (512-thread
    class, three per CU) rather than 2 or 10."""
    r = subprocess.run([checker, "plan", str(prec), str(n), str(batch)],
                       capture_output=True, text=True)
    print(r.stdout)
    assert r.returncode == 0, r.stdout + r.stderr
    assert f" bt={bt} " in r.stdout, r.stdout


def test_fig3_plan_of_30_with_radices_3_2_5(checker):
    """Fig. 3 (Section 4.2, "Discussion"): n = 30 planned by DIT steps of radix
    3, then 2, then 5.  Here the steps are Stockham stages, executed innermost
    first (radix 5, then 2, then 3); forced through the planner's structural
    choice, the stage descriptors and the steps they execute must be the
    figure's: the size-5 DFTs without twiddles (vector 2, loop 3), the size-2
    twiddle step (vector 5, loop 3), the size-3 twiddle step (vector 10) --
    the breadth-first list, and grouped under the shared loop of 3, the
    depth-first one."""
    r = subprocess.run([checker, "steps", "30", "5.2.3"], capture_output=True, text=True)
    assert r.returncode == 0, r.stdout + r.stderr
    lines = r.stdout.strip().splitlines()
    stages = [tuple(int(v) for v in re.findall(r"=(\d+)", ln)) for ln in lines if ln.startswith("stage")]
    assert stages == [(5, 1, 6), (2, 5, 15), (3, 10, 10)]          # (R, Ns, butterflies)
    steps = dict(ln.split(": ", 1) for ln in lines if ": " in ln)

    def parse(text):
        # "loop L {a ; b} ; c" -> [("loop", L, [a, b]), c] with a = (kind, R, vector)
        out = []
        for m in re.finditer(r"loop (\d+) \{([^}]*)\}|(direct|twiddle) (\d+) x(\d+)", text):
            if m.group(1):
                body = [(k, int(a), int(v)) for k, a, v in
                        re.findall(r"(direct|twiddle) (\d+) x(\d+)", m.group(2))]
                out.append(("loop", int(m.group(1)), body))
            else:
                out.append((m.group(3), int(m.group(4)), int(m.group(5))))
        return out

    # the figure's two step lists (tests/golden/fig3_plan_n30.txt)
    with open(os.path.join(HERE, "golden", "fig3_plan_n30.txt")) as fh:
        fig = dict(ln.strip().split(": ", 1) for ln in fh if ln.strip() and not ln.startswith("#"))
    assert parse(fig["breadth"]) == [("loop", 3, [("direct", 5, 2)]),
                                     ("loop", 3, [("twiddle", 2, 5)]), ("twiddle", 3, 10)]
    assert parse(steps["breadth"]) == parse(fig["breadth"])
    assert parse(steps["depth"]) == parse(fig["depth"])


def test_planner_under_address_and_ub_sanitizers(checker_san):
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    _, s = _run(checker_san, "bounds", 0, 67, 12000, 2, "primes", env=env)
    assert s["violations"] == 0 and s["guarded"] > 0
    _, s = _run(checker_san, "bounds", 1, 1, 2100, 3, "all", env=env)
    assert s["violations"] == 0
    _, s = _run(checker_san, "random", 3000, 11, env=env)
    assert s["violations"] == 0 and s["planned"] > 1000
    _, s = _run(checker_san, "cands", 0, 2, 1200, 2, env=env)
    assert s["violations"] == 0 and s["failed"] == 0


def test_oracle_under_address_and_ub_sanitizers(tmp_path):
    if shutil.which("gcc") is None:
        pytest.skip("no gcc")
    exe = str(tmp_path / "oracle_san")
    subprocess.run(["gcc", "-std=gnu11", *SAN, "-pthread", os.path.join(ROOT, "oracle", "oracle.c"),
                    os.path.join(HERE, "oracle_sanitize_check.c"), "-o", exe, "-lm"], check=True)
    r = subprocess.run([exe], capture_output=True, text=True,
                       env=dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1"))
    print(r.stdout)
    assert r.returncode == 0 and "check ok" in r.stdout, (r.stdout, r.stderr[-4000:])
