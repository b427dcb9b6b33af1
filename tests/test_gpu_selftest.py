"""Large-size checks where the O(n^2) definition is out of reach.

Section 6 names an O(n log n) randomized self-test (Ergun) for correctness at
any size; its ingredients -- linearity, the impulse response and the time-shift
rule -- are checked here on the GPU output itself, together with Parseval and
sampled outputs against the oracle.  The error-growth check follows the same
section: with accurate twiddles the mean error grows like sqrt(log n)."""
import math

import numpy as np
import pytest

import oracle
from synth import uniform_complex

pytestmark = pytest.mark.gpu


def _fft(x, sign=-1, prec=0):
    import torch

    import paper_2602_23525_amd as mfft
    n = x.size
    xt = torch.from_numpy(x).cuda()
    yt = torch.empty_like(xt)
    p = mfft.Plan([(n, 1, 1)], [], sign=sign, prec=prec)
    p.execute(xt, yt)
    torch.cuda.synchronize()
    p.destroy()
    return yt.cpu().numpy().astype(np.complex128)


@pytest.mark.parametrize("n,prec", [(65537, 0), (131220, 0), (1 << 22, 0), (65537, 1),
                                    (1 << 20, 1), (999983, 0)])
def test_ergun_style_self_test(n, prec):
    cdt = np.complex64 if prec == 0 else np.complex128
    tol = 2e-6 if prec == 0 else 1e-13 * max(1.0, math.log2(n) / 20)
    rng = np.random.default_rng(n)
    x = uniform_complex(n, seed=n + 1, dtype=cdt)
    z = uniform_complex(n, seed=n + 2, dtype=cdt)
    X, Z = _fft(x, prec=prec), _fft(z, prec=prec)
    # linearity with random complex coefficients
    a, b = complex(rng.uniform(-1, 1), rng.uniform(-1, 1)), complex(rng.uniform(-1, 1), 0.5)
    comb = (a * x.astype(np.complex128) + b * z.astype(np.complex128)).astype(cdt)
    ref = a * X + b * Z
    assert oracle.rel_rms(_fft(comb, prec=prec), ref) <= 3 * tol
    # impulse at l0: Y[k] = w^(l0 k)
    l0 = int(rng.integers(1, n))
    d = np.zeros(n, cdt)
    d[l0] = 1
    k = np.arange(n, dtype=np.int64)
    e = (l0 * k) % n
    w = np.exp(-2j * np.pi * e / n)
    assert oracle.rel_rms(_fft(d, prec=prec), w) <= tol
    # time shift: x[l - s] -> w^(s k) X[k]
    s = int(rng.integers(1, n))
    ws = np.exp(-2j * np.pi * ((s * k) % n) / n)
    assert oracle.rel_rms(_fft(np.roll(x, s), prec=prec), ws * X) <= 3 * tol
    # Parseval
    xx = x.astype(np.complex128)
    assert abs(np.sum(abs(X) ** 2) / (n * np.sum(abs(xx) ** 2)) - 1) <= 20 * tol
    # sampled outputs against the definition (exact index reduction)
    for kk in (0, 1, n // 2, n - 1, int(rng.integers(0, n))):
        ref_k = np.sum(xx * np.exp(-2j * np.pi * ((k * kk) % n) / n))
        assert abs(X[kk] - ref_k) <= 50 * tol * math.sqrt(n)


def test_error_growth_is_logarithmic():
    """FP32 relative RMS error divided by 2^-24 sqrt(log2 n) stays bounded from
    n = 2^4 to 2^22 (no O(sqrt n) growth from the twiddles)."""
    ratios = []
    for e in range(4, 23, 2):
        n = 1 << e
        b = max(1, (1 << 20) // n)
        x = uniform_complex(n * b, seed=e, dtype=np.complex64)
        import torch

        import paper_2602_23525_amd as mfft
        xt = torch.from_numpy(x).cuda()
        yt = torch.empty_like(xt)
        p = mfft.Plan([(n, 1, 1)], [(b, n, n)] if b > 1 else [])
        p.execute(xt, yt)
        torch.cuda.synchronize()
        p.destroy()
        y = yt.cpu().numpy().reshape(b, n)
        ref = oracle.fft(x.astype(np.complex128).reshape(b, n))
        err = oracle.rel_rms(y, ref)
        ratios.append(err / (2.0 ** -24 * math.sqrt(e)))
    assert max(ratios) <= 4.0, ratios
    # no systematic growth: the last ratio is not far above the first
    assert ratios[-1] <= 3.0 * ratios[0] + 0.5, ratios
