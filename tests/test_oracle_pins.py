"""Pins for the FP64 CPU oracle, independent of the oracle itself.

Each check ties the oracle to something the paper or mathematics fixes:
hand-expanded small DFTs, an arbitrary-precision evaluation of eq. (dft)
(Section 6 measures accuracy against an arbitrary-precision slow FFT), closed
forms and invariants of the DFT, the I/O-tensor examples of Section 4.1, and an
independent library FFT (numpy) as a tertiary cross-check.
"""
import cmath
import math

import mpmath
import numpy as np
import pytest

import oracle
from synth import uniform_complex

METHODS_1D = [oracle.dft_direct_1d, oracle.fft_rec_1d, oracle.fft_bluestein_1d,
              lambda x, sign=-1: oracle.fft(x, sign=sign)]


def mp_dft(x, sign=-1, dps=40):
    """eq. (dft) evaluated at `dps` decimal digits with mpmath."""
    with mpmath.workdps(dps):
        n = len(x)
        xs = [mpmath.mpc(complex(v)) for v in x]
        out = []
        for k in range(n):
            s = mpmath.mpc(0)
            for l in range(n):
                s += xs[l] * mpmath.expjpi(mpmath.mpf(2 * sign * ((l * k) % n)) / n)
            out.append(complex(s))
    return np.array(out)


# ------------------------------------------------------------ hand expansions

@pytest.mark.parametrize("f", METHODS_1D)
def test_hand_expanded_small_sizes(f):
    a, b, c, d = 0.3 - 0.7j, -1.1 + 0.2j, 0.5 + 0.25j, -0.125 - 0.9j
    # n = 1: identity
    assert np.allclose(f(np.array([a])), [a], atol=0, rtol=0)
    # n = 2: [a + b, a - b]
    assert np.allclose(f(np.array([a, b])), [a + b, a - b], atol=1e-15)
    # n = 4, forward (w = -i): Y1 = x0 - i x1 - x2 + i x3
    y = f(np.array([a, b, c, d]))
    exp = [a + b + c + d, a - 1j * b - c + 1j * d, a - b + c - d, a + 1j * b - c - 1j * d]
    assert np.allclose(y, exp, atol=1e-15)
    # n = 4, sign +1 (w = +i)
    y = f(np.array([a, b, c, d]), sign=1)
    exp = [a + b + c + d, a + 1j * b - c - 1j * d, a - b + c - d, a - 1j * b - c + 1j * d]
    assert np.allclose(y, exp, atol=1e-15)
    # n = 3: w = exp(-2 pi i/3)
    w = complex(-0.5, -math.sqrt(3) / 2)
    y = f(np.array([a, b, c]))
    exp = [a + b + c, a + w * b + w * w * c, a + w * w * b + w * c]
    assert np.allclose(y, exp, atol=1e-15)


# ------------------------------------------------------------ arbitrary precision

@pytest.mark.parametrize("n", list(range(1, 33)) + [48, 60, 64, 97, 100, 128])
def test_mpmath_definition(n):
    x = uniform_complex(n, seed=1000 + n)
    ref = mp_dft(x)
    for f in METHODS_1D:
        assert oracle.rel_rms(f(x), ref) <= 1e-15, f
    refp = mp_dft(x, sign=1)
    for f in METHODS_1D:
        assert oracle.rel_rms(f(x, sign=1), refp) <= 1e-15, f


@pytest.mark.parametrize("n", [243, 256, 257])
def test_mpmath_definition_larger(n):
    x = uniform_complex(n, seed=2000 + n)
    ref = mp_dft(x, dps=30)
    for f in METHODS_1D:
        assert oracle.rel_rms(f(x), ref) <= 1e-15


def test_roots_exact_and_accurate():
    for n in [1, 2, 3, 4, 5, 8, 12, 16, 24, 100, 1000, 4096, 65537, 1 << 22]:
        assert oracle.root(0, n) == 1 + 0j
        if n % 2 == 0:
            assert oracle.root(n // 2, n) == -1 + 0j or oracle.root(n // 2, n) == complex(-1, -0.0)
        if n % 4 == 0:
            assert oracle.root(n // 4, n, -1) == complex(0.0, -1.0) or \
                oracle.root(n // 4, n, -1).real == 0 and oracle.root(n // 4, n, -1).imag == -1
            assert abs(oracle.root(n // 4, n, +1) - 1j) == 0
        if n % 8 == 0:
            r = oracle.root(n // 8, n, -1)
            assert abs(r.real - math.sqrt(0.5)) <= 1.2e-16 and abs(r.imag + math.sqrt(0.5)) <= 1.2e-16
        for m in list(range(0, min(n, 40))) + [n - 1, n // 3, (7 * n) // 9]:
            if not 0 <= m < n:
                continue
            w = oracle.root(m, n)
            if m:
                assert oracle.root(n - m, n) == w.conjugate()
            with mpmath.workdps(30):
                ref = complex(mpmath.expjpi(mpmath.mpf(-2 * m) / n))
            assert abs(w - ref) <= 1.2e-16


# ------------------------------------------------------------ closed forms

SIZES = [1, 2, 3, 5, 6, 7, 8, 12, 16, 30, 64, 97, 100, 210, 256, 1000, 1009]


@pytest.mark.parametrize("n", SIZES)
def test_closed_forms(n):
    rng = np.random.default_rng(n)
    x = uniform_complex(n, seed=3000 + n)
    for f in METHODS_1D:
        # impulse at l0 -> w^(l0 k)
        l0 = int(rng.integers(0, n))
        d = np.zeros(n, complex)
        d[l0] = 1
        k = np.arange(n)
        assert np.allclose(f(d), np.exp(-2j * np.pi * ((l0 * k) % n) / n), atol=1e-13)
        # constant -> n delta
        e = np.zeros(n, complex)
        e[0] = n
        assert np.allclose(f(np.ones(n, complex)), e, atol=1e-12 * n)
        # tone exp(+2 pi i k0 l/n) -> n delta[k - k0] under the forward transform
        k0 = int(rng.integers(0, n))
        tone = np.exp(2j * np.pi * ((k0 * k) % n) / n)
        e = np.zeros(n, complex)
        e[k0] = n
        assert np.allclose(f(tone), e, atol=1e-12 * n)
        y = f(x)
        # shift: x[l - s] -> w^(s k) Y[k]
        s = int(rng.integers(0, n))
        assert np.allclose(f(np.roll(x, s)), np.exp(-2j * np.pi * ((s * k) % n) / n) * y,
                           atol=1e-12 * n)
        # modulation: x[l] w^(-m l) -> Y[k - m]
        m = int(rng.integers(0, n))
        assert np.allclose(f(x * np.exp(2j * np.pi * ((m * k) % n) / n)), np.roll(y, m),
                           atol=1e-12 * n)
        # Parseval
        assert abs(np.sum(abs(y) ** 2) - n * np.sum(abs(x) ** 2)) <= 1e-12 * n * n
        # linearity
        z = uniform_complex(n, seed=4000 + n)
        al, be = 0.3 - 1.7j, -2.2 + 0.4j
        assert np.allclose(f(al * x + be * z), al * y + be * f(z), atol=1e-12 * n)
        # forward then sign +1 = n * identity
        assert np.allclose(f(y, sign=1), n * x, atol=1e-12 * n)
        # F^4 = n^2 I
        assert np.allclose(f(f(f(y))), n * n * x, atol=1e-11 * n * n)
        # conjugation: F(conj x)[k] = conj(F(x)[-k])
        assert np.allclose(f(np.conj(x)), np.conj(y[(-k) % n]), atol=1e-12 * n)
        # real input -> Hermitian output
        yr = f(x.real.astype(complex))
        assert np.allclose(yr, np.conj(yr[(-k) % n]), atol=1e-12 * n)


@pytest.mark.parametrize("n", [5, 12, 31, 64])
def test_convolution_theorem(n):
    x = uniform_complex(n, seed=5000 + n)
    h = uniform_complex(n, seed=6000 + n)
    conv = np.array([sum(x[j] * h[(k - j) % n] for j in range(n)) for k in range(n)])
    for f in METHODS_1D:
        assert np.allclose(f(conv), f(x) * f(h), atol=1e-12 * n)


# ------------------------------------------------------------ algorithms agree

def test_recursion_and_bluestein_match_direct_exhaustive():
    for n in range(1, 513):
        x = uniform_complex(n, seed=7000 + n)
        d = oracle.dft_direct_1d(x)
        assert oracle.rel_rms(oracle.fft_rec_1d(x), d) <= 1e-15, n
        assert oracle.rel_rms(oracle.fft_bluestein_1d(x), d) <= 2e-15, n


@pytest.mark.parametrize("n", [1000, 2187, 4096, 14175, 65537])
def test_large_sizes_against_numpy_and_sampled_direct(n):
    x = uniform_complex(n, seed=8000 + n)
    y = oracle.fft(x)
    assert oracle.rel_rms(y, np.fft.fft(x)) <= 1e-14
    # sampled outputs against eq. (dft) with exact index reduction
    for k in (0, 1, n // 3, n - 1):
        e = (np.arange(n, dtype=np.int64) * k) % n
        ref = np.sum(x * np.exp(-2j * np.pi * e / n))
        assert abs(y[k] - ref) <= 1e-9 * math.sqrt(n)


# ------------------------------------------------------------ multi-dim, strides

@pytest.mark.parametrize("shape", [(2, 3, 5), (4, 4), (7, 3), (3, 1, 4), (2, 2, 2, 3)])
def test_multidim_separable_equals_definition(shape):
    x = uniform_complex(int(np.prod(shape)), seed=sum(shape)).reshape(shape)
    a = oracle.fftn(x, len(shape))
    b = oracle.fftn(x, len(shape), method="md_direct")
    assert oracle.rel_rms(a, b) <= 1e-15
    assert oracle.rel_rms(a, np.fft.fftn(x)) <= 1e-15
    # the multi-dimensional definition at arbitrary precision on one output
    idx = tuple(s // 2 for s in shape)
    with mpmath.workdps(30):
        s = mpmath.mpc(0)
        for l in np.ndindex(*shape):
            ph = sum(mpmath.mpf(li * ki) / ni for li, ki, ni in zip(l, idx, shape))
            s += mpmath.mpc(complex(x[l])) * mpmath.expjpi(-2 * ph)
    assert abs(complex(s) - b[idx]) <= 1e-14


def test_paper_examples_rows_columns_copy_transpose():
    """The I/O-tensor examples of Section 4.1 ("DFT problem examples")."""
    n1, n2 = 6, 10
    X = uniform_complex(n1 * n2, seed=11)
    # single 1D DFT dft({(n,1,1)}, {}, X, Y)
    Y = np.zeros_like(X)
    oracle.dft(X, Y, [(n1 * n2, 1, 1)])
    assert oracle.rel_rms(Y, np.fft.fft(X)) <= 1e-15
    # in-place DFTs of all rows: dft({(n2,1,1)}, {(n1,n2,n2)}, X, X)
    A = X.copy()
    oracle.dft(A, A, [(n2, 1, 1)], [(n1, n2, n2)])
    assert oracle.rel_rms(A.reshape(n1, n2), np.fft.fft(X.reshape(n1, n2), axis=1)) <= 1e-15
    # in-place DFTs of all columns: dft({(n1,n2,n2)}, {(n2,1,1)}, X, X)
    A = X.copy()
    oracle.dft(A, A, [(n1, n2, n2)], [(n2, 1, 1)])
    assert oracle.rel_rms(A.reshape(n1, n2), np.fft.fft(X.reshape(n1, n2), axis=0)) <= 1e-15
    # rank-0 copy dft({}, {(n,1,1)}, I, O)
    O = np.zeros_like(X)
    oracle.dft(X, O, [], [(n1 * n2, 1, 1)])
    assert np.array_equal(O, X)
    # rank-0 in-place transpose dft({}, {(n1,n2,1),(n2,1,n1)}, X, X)
    A = X.copy()
    oracle.dft(A, A, [], [(n1, n2, 1), (n2, 1, n1)])
    assert np.array_equal(A.reshape(n2, n1), X.reshape(n1, n2).T)


def test_strided_vector_problem_equals_gather_scatter():
    rng = np.random.default_rng(3)
    buf = uniform_complex(4000, seed=12)
    out = np.full(4000, np.nan + 0j)
    # N = {(12, is=3, os=-5)}, V = {(4, 40, 1), (3, 7, 100)}, base offsets
    dims = [(12, 3, -5)]
    vdims = [(4, 40, 1), (3, 7, 100)]
    in_off, out_off = 100, 2000
    oracle.dft(buf, out, dims, vdims, in_off=in_off, out_off=out_off)
    for a in range(4):
        for b in range(3):
            src = buf[in_off + a * 40 + b * 7 + 3 * np.arange(12)]
            ref = np.fft.fft(src)
            got = out[out_off + a * 1 + b * 100 - 5 * np.arange(12)]
            assert oracle.rel_rms(got, ref) <= 1e-15
    written = np.zeros(4000, bool)
    for a in range(4):
        for b in range(3):
            written[out_off + a + b * 100 - 5 * np.arange(12)] = True
    assert np.all(np.isnan(out[~written]))
    assert rng is not None


def test_inplace_snapshot_semantics():
    """In-place problems whose input and output strides differ read the
    pre-call input (the 2-D transform with transposed output)."""
    n = 8
    X = uniform_complex(n * n, seed=13)
    A = X.copy()
    oracle.dft(A, A, [(n, n, 1), (n, 1, n)])
    ref = np.fft.fft2(X.reshape(n, n)).T
    assert oracle.rel_rms(A.reshape(n, n), ref) <= 1e-15


def test_empty_and_degenerate():
    X = uniform_complex(10, seed=14)
    O = np.full(10, 7 + 7j)
    oracle.dft(X, O, [(0, 1, 1)], [(10, 1, 1)])          # n = 0: no-op
    assert np.all(O == 7 + 7j)
    oracle.dft(X, O, [(5, 1, 1)], [(0, 5, 5)])           # empty vector loop
    assert np.all(O == 7 + 7j)
    oracle.dft(X, O, [(1, 1, 1)], [(10, 1, 1)])          # size-1 DFT is a copy
    assert np.array_equal(O, X)


# ------------------------------------------------------------ plan algebra

@pytest.mark.parametrize("n", [6, 12, 30, 64, 100, 210, 256])
def test_dit_rule_reproduces_whole_transform(n):
    """The decimation-in-time step of Section 4.2 ("Cooley-Tukey plans"):
    dft({(m, r is, os)}, V u {(r, is, m os)}, I, O), then twiddles
    w_n^(l2 k1) on O, then dft({(r, m os, m os)}, V u {(m, os, os)}, O, O)
    equals dft({(n, is, os)}, V, I, O) for every factor r of n.  The last step
    works on O alone, so its vector loops V run with their output strides
    (copy-o(V)); the paper writes V there, which only matches when is = os."""
    B = 3
    is_, os_ = 2, 3
    X = uniform_complex(is_ * n * B + 5, seed=15 + n)
    V = [(B, is_ * n, os_ * n)]
    ref = np.zeros(os_ * n * B + 5, complex)
    oracle.dft(X, ref, [(n, is_, os_)], V)
    for r in [d for d in range(2, n) if n % d == 0]:
        m = n // r
        O = np.zeros_like(ref)
        oracle.dft(X, O, [(m, r * is_, os_)], V + [(r, is_, m * os_)])
        for b in range(B):
            for l2 in range(r):
                for k1 in range(m):
                    O[b * os_ * n + (l2 * m + k1) * os_] *= oracle.root(l2 * k1, n)
        Vo = [(d[0], d[2], d[2]) for d in V]
        oracle.dft(O, O, [(r, m * os_, m * os_)], Vo + [(m, os_, os_)])
        assert oracle.rel_rms(O, ref) <= 1e-14, r


@pytest.mark.parametrize("n", [8, 15, 36])
def test_indirect_rule(n):
    """Indirect plans (Section 4.2): dft({}, N u V, I, O) then
    dft(copy-o(N), copy-o(V), O, O) equals dft(N, V, I, O)."""
    X = uniform_complex(4 * n * 7, seed=16 + n)
    N = [(n, 3, 7)]
    V = [(4, 1, 1)]
    ref = np.zeros(7 * n + 10, complex)
    oracle.dft(X, ref, N, V)
    O = np.zeros_like(ref)
    oracle.dft(X, O, [], N + V)
    copy_o = lambda t: [(d[0], d[2], d[2]) for d in t]
    oracle.dft(O, O, copy_o(N), copy_o(V))
    assert oracle.rel_rms(O, ref) <= 1e-15


def test_error_growth_is_small():
    """Section 6: Cooley-Tukey error grows like sqrt(log n) at most; the FP64
    oracle stays within a few ulps of numpy across a wide size range."""
    for e in range(4, 21, 4):
        n = 1 << e
        x = uniform_complex(n, seed=e)
        assert oracle.rel_rms(oracle.fft(x), np.fft.fft(x)) <= 4e-16 * math.sqrt(e)
