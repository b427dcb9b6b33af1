"""Pins of the oracle's real-input transforms (rfft / irfft) against facts fixed
outside the oracle: hand-expanded tiny cases, closed forms, numpy's real FFT as a
tertiary library check, and the inverse relation."""
import numpy as np
import pytest

import oracle


def test_tiny_by_hand():
    a, b = 0.75, -0.25
    y = oracle.rfft(np.array([a, b]))
    assert np.allclose(y, [a + b, a - b], atol=1e-15)
    y = oracle.rfft(np.array([1.0, 2.0, 3.0, 4.0]))
    # Y0 = 10, Y1 = (1-3) + (4-2)i... = -2 + 2i, Y2 = 1 - 2 + 3 - 4 = -2
    assert np.allclose(y, [10, -2 + 2j, -2], atol=1e-14)
    assert np.allclose(oracle.rfft(np.array([5.0])), [5.0])


@pytest.mark.parametrize("n", [1, 2, 3, 4, 5, 8, 15, 16, 100, 243, 1009, 1024])
def test_matches_numpy_rfft(n):
    rng = np.random.default_rng(n)
    x = rng.uniform(-1, 1, (3, n))
    y = oracle.rfft(x)
    assert y.shape == (3, n // 2 + 1)
    assert oracle.rel_rms(y, np.fft.rfft(x)) < 1e-14
    z = oracle.irfft(y, n)
    assert np.allclose(z, np.fft.irfft(np.fft.rfft(x), n) * n, atol=1e-11 * n)


@pytest.mark.parametrize("n,k0", [(16, 3), (17, 5), (1000, 1), (1000, 499), (33, 16)])
def test_cosine_tone_closed_form(n, k0):
    l = np.arange(n)
    y = oracle.rfft(np.cos(2 * np.pi * k0 * l / n))
    ref = np.zeros(n // 2 + 1, complex)
    ref[k0] = n / 2
    assert np.max(np.abs(y - ref)) < 1e-11 * n


def test_constant_and_alternating():
    n = 64
    assert np.allclose(oracle.rfft(np.ones(n)), np.r_[n, np.zeros(n // 2)], atol=1e-12)
    alt = (-1.0) ** np.arange(n)
    ref = np.zeros(n // 2 + 1)
    ref[-1] = n
    assert np.allclose(oracle.rfft(alt), ref, atol=1e-12)


@pytest.mark.parametrize("n", [2, 7, 64, 1000, 4097])
def test_round_trip_is_n_times_identity(n):
    x = np.random.default_rng(n + 1).uniform(-1, 1, (2, n))
    assert np.max(np.abs(oracle.irfft(oracle.rfft(x), n) - n * x)) < 1e-12 * n


@pytest.mark.parametrize("n", [8, 9])
def test_irfft_ignores_imaginary_parts_of_self_conjugate_bins(n):
    y = oracle.rfft(np.random.default_rng(3).uniform(-1, 1, n))
    y2 = y.copy()
    y2[0] += 0.5j
    if n % 2 == 0:
        y2[-1] -= 0.25j
    assert np.array_equal(oracle.irfft(y, n), oracle.irfft(y2, n))


@pytest.mark.parametrize("shape", [(4, 6), (3, 5, 8), (7, 9)])
def test_multidim_matches_numpy(shape):
    x = np.random.default_rng(len(shape)).uniform(-1, 1, (2,) + shape)
    axes = tuple(range(1, len(shape) + 1))
    y = oracle.rfftn(x, len(shape))
    assert oracle.rel_rms(y, np.fft.rfftn(x, axes=axes)) < 1e-14
    z = oracle.irfftn(y, shape)
    assert np.allclose(z, np.prod(shape) * x, atol=1e-11 * np.prod(shape))
    # the inverse of an arbitrary (non-symmetric) half spectrum follows numpy's
    # convention: inverse DFTs along the leading axes, then the real inverse
    w = (np.random.default_rng(5).uniform(-1, 1, y.shape)
         + 1j * np.random.default_rng(6).uniform(-1, 1, y.shape))
    ref = np.fft.irfftn(w, s=shape, axes=axes) * np.prod(shape)
    assert np.allclose(oracle.irfftn(w, shape), ref, atol=1e-11 * np.prod(shape))
