"""FP64 CPU oracle for dft(N, V, I, O) -- test infrastructure.

Only the tests, the smoke check and the benchmark's CPU-baseline leg may import
this package.  The GPU library never imports, links or runs it, and it shares no
code with the library: the arithmetic lives in ``oracle.c`` (plain C, gcc), this
file only marshals numpy buffers.

Functions follow Johnson & Frigo, "Implementing FFTs in Practice":
  * ``dft``  -- the problem dft(N, V, I, O) of Section 4.1 over strided buffers;
  * ``fft``  -- convenience: DFT along the last axis of a numpy array;
  * ``fftn`` -- convenience: multi-dimensional DFT over the trailing axes;
  * ``dft_direct_1d`` / ``fft_rec_1d`` / ``fft_bluestein_1d`` -- the single
    algorithms O1 (eq. dft, Section 2), O2 (eq. ct, Section 2, decimation in time
    by the smallest prime factor; Algorithm 1 is its radix-2 case) and O3
    (Bluestein's chirp-z, Section 4.2 "Plans for prime sizes");
  * ``root`` -- exp(sign 2 pi i m / n) from the oracle's own octant-reduced table;
  * ``rfft`` / ``irfft`` -- real-input DFTs (the conjugate-symmetric case of
    eq. dft that Sections 5 and 7 single out): the forward DFT of real data keeping
    outputs 0 .. n//2, and its unnormalized inverse from such a half spectrum;
    ``rfftn`` / ``irfftn`` the same over the trailing axes, the last one halved.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None

METHODS = {"auto": 0, "direct": 1, "recursive": 2, "bluestein": 3, "md_direct": 4}


class _IoDim(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("is_", ctypes.c_int64), ("os", ctypes.c_int64)]


def _lib():
    global _LIB
    if _LIB is None:
        path = os.path.join(_HERE, "liboracle.so")
        if not os.path.exists(path):
            from . import build as _b
            _b.build()
        lib = ctypes.CDLL(path)
        dp = ctypes.POINTER(ctypes.c_double)
        lib.oracle_dft.argtypes = [ctypes.c_int, ctypes.POINTER(_IoDim), ctypes.c_int,
                                   ctypes.POINTER(_IoDim), dp, dp, ctypes.c_int, ctypes.c_int,
                                   ctypes.c_int]
        lib.oracle_dft.restype = ctypes.c_int
        for name in ("oracle_dft_direct_1d",):
            f = getattr(lib, name)
            f.argtypes = [ctypes.c_int64, ctypes.c_int, dp, ctypes.c_int64, dp, ctypes.c_int64]
            f.restype = None
        for name in ("oracle_fft_rec_1d", "oracle_fft_bluestein_1d"):
            f = getattr(lib, name)
            f.argtypes = [ctypes.c_int64, ctypes.c_int, dp, ctypes.c_int64, dp]
            f.restype = None
        lib.oracle_root.argtypes = [ctypes.c_int64, ctypes.c_int64, ctypes.c_int, dp]
        lib.oracle_root.restype = None
        _LIB = lib
    return _LIB


def default_threads() -> int:
    try:
        return max(1, len(os.sched_getaffinity(0)))
    except AttributeError:  # pragma: no cover
        return os.cpu_count() or 1


def _dptr(a: np.ndarray, offset: int = 0):
    assert a.dtype == np.complex128 and a.flags["C_CONTIGUOUS"]
    return ctypes.cast(a.ctypes.data + 16 * offset, ctypes.POINTER(ctypes.c_double))


def _span(dims, vdims, which):
    lo = hi = 0
    for (n, is_, os_) in list(dims) + list(vdims):
        if n <= 0:
            return None
        s = is_ if which == 0 else os_
        ext = (n - 1) * s
        if ext < 0:
            lo += ext
        else:
            hi += ext
    return lo, hi


def dft(inbuf: np.ndarray, outbuf: np.ndarray, dims, vdims=(), sign: int = -1,
        method: str = "auto", in_off: int = 0, out_off: int = 0, nthreads: int | None = None):
    """Solve dft(N=dims, V=vdims, I=inbuf+in_off, O=outbuf+out_off) in FP64.

    ``dims``/``vdims`` are sequences of (n, is, os) with strides in complex
    elements.  ``inbuf`` and ``outbuf`` are flat complex128 arrays and may be the
    same array (in-place); the input is snapshotted before any write.
    """
    dims = [tuple(int(v) for v in d) for d in dims]
    vdims = [tuple(int(v) for v in d) for d in vdims]
    if any(d[0] == 0 for d in dims + vdims):
        return outbuf
    for which, buf, off in ((0, inbuf, in_off), (1, outbuf, out_off)):
        lo, hi = _span(dims, vdims, which)
        if off + lo < 0 or off + hi >= buf.size:
            raise IndexError("tensor reaches outside its buffer")
    nd = len(dims)
    nv = len(vdims)
    cd = (_IoDim * max(1, nd))(*[_IoDim(*d) for d in dims])
    cv = (_IoDim * max(1, nv))(*[_IoDim(*d) for d in vdims])
    rc = _lib().oracle_dft(nd, cd, nv, cv, _dptr(inbuf, in_off), _dptr(outbuf, out_off),
                           int(sign), METHODS[method], int(nthreads or default_threads()))
    if rc != 0:
        raise ValueError("oracle_dft rejected the problem")
    return outbuf


def fft(x, sign: int = -1, method: str = "auto", nthreads: int | None = None) -> np.ndarray:
    """DFT along the last axis of ``x`` (any leading batch shape), FP64."""
    x = np.ascontiguousarray(np.asarray(x, dtype=np.complex128))
    n = x.shape[-1]
    b = x.size // n if n else 0
    out = np.empty_like(x)
    if x.size == 0:
        return out
    dft(x.reshape(-1), out.reshape(-1), [(n, 1, 1)], [(b, n, n)] if b > 1 else [],
        sign=sign, method=method, nthreads=nthreads)
    return out


def fftn(x, ndim: int, sign: int = -1, method: str = "auto", nthreads: int | None = None):
    """Separable DFT over the trailing ``ndim`` axes of ``x``, FP64."""
    x = np.ascontiguousarray(np.asarray(x, dtype=np.complex128))
    shape = x.shape[x.ndim - ndim:]
    ntot = int(np.prod(shape))
    b = x.size // ntot if ntot else 0
    dims = []
    stride = 1
    for n in reversed(shape):
        dims.append((n, stride, stride))
        stride *= n
    dims.reverse()
    out = np.empty_like(x)
    if x.size == 0:
        return out
    dft(x.reshape(-1), out.reshape(-1), dims, [(b, ntot, ntot)] if b > 1 else [],
        sign=sign, method=method, nthreads=nthreads)
    return out


def _one(fname, n, sign, x, xs=1):
    x = np.ascontiguousarray(np.asarray(x, dtype=np.complex128))
    y = np.empty(n, dtype=np.complex128)
    f = getattr(_lib(), fname)
    if fname == "oracle_dft_direct_1d":
        f(n, sign, _dptr(x), xs, _dptr(y), 1)
    else:
        f(n, sign, _dptr(x), xs, _dptr(y))
    return y


def dft_direct_1d(x, sign: int = -1):
    """O1: eq. (dft) summed directly (long double accumulation)."""
    return _one("oracle_dft_direct_1d", len(x), sign, x)


def fft_rec_1d(x, sign: int = -1):
    """O2: decimation-in-time recursion by the smallest prime factor (eq. ct)."""
    return _one("oracle_fft_rec_1d", len(x), sign, x)


def fft_bluestein_1d(x, sign: int = -1):
    """O3: Bluestein's chirp-z algorithm over a power-of-two convolution."""
    return _one("oracle_fft_bluestein_1d", len(x), sign, x)


def root(m: int, n: int, sign: int = -1) -> complex:
    out = (ctypes.c_double * 2)()
    _lib().oracle_root(int(m), int(n), int(sign), out)
    return complex(out[0], out[1])


def rel_rms(y, yref) -> float:
    """||y - yref||_2 / ||yref||_2 over all elements."""
    y = np.asarray(y, dtype=np.complex128).ravel()
    yref = np.asarray(yref, dtype=np.complex128).ravel()
    den = np.linalg.norm(yref)
    return float(np.linalg.norm(y - yref) / den) if den > 0 else float(np.linalg.norm(y))


def max_err(y, yref) -> float:
    """max_k |y_k - yref_k| / rms(yref)."""
    y = np.asarray(y, dtype=np.complex128).ravel()
    yref = np.asarray(yref, dtype=np.complex128).ravel()
    rms = np.sqrt(np.mean(np.abs(yref) ** 2)) if yref.size else 0.0
    d = np.max(np.abs(y - yref)) if y.size else 0.0
    return float(d / rms) if rms > 0 else float(d)


def rfft(x, nthreads: int | None = None) -> np.ndarray:
    """Forward DFT (eq. dft, sign -1) of real data along the last axis, outputs
    k = 0 .. n//2.  The others follow from conjugate symmetry, Y[n-k] = conj(Y[k]),
    which holds for every real input (Section 5 notes the factor of two this
    redundancy saves)."""
    x = np.asarray(x, np.float64)
    n = x.shape[-1]
    y = fft(x.astype(np.complex128), sign=-1, nthreads=nthreads)
    return y[..., : n // 2 + 1]


def irfft(y, n: int, nthreads: int | None = None) -> np.ndarray:
    """Inverse of ``rfft`` without normalization (irfft(rfft(x), n) = n x): the half
    spectrum k = 0 .. n//2 is extended by Y[n-k] = conj(Y[k]), the imaginary parts of
    Y[0] and (n even) Y[n/2] are dropped -- a conjugate-symmetric spectrum has them
    zero -- and the sign +1 DFT of the extension is real; its real part is returned."""
    y = np.asarray(y, np.complex128)
    h = n // 2 + 1
    full = np.zeros(y.shape[:-1] + (n,), np.complex128)
    full[..., :h] = y[..., :h]
    full[..., 0] = full[..., 0].real
    if n % 2 == 0:
        full[..., n // 2] = full[..., n // 2].real
    k = np.arange(h, n)
    full[..., h:] = np.conj(y[..., n - k])
    return fft(full, sign=+1, nthreads=nthreads).real


def rfftn(x, ndim: int, nthreads: int | None = None) -> np.ndarray:
    """Multi-dimensional forward DFT of real data over the trailing ``ndim`` axes
    (the separable product of eq. dft), keeping indices 0 .. n//2 of the last axis."""
    x = np.asarray(x, np.float64)
    n = x.shape[-1]
    y = fftn(x.astype(np.complex128), ndim, sign=-1, nthreads=nthreads)
    return y[..., : n // 2 + 1]


def irfftn(y, shape, nthreads: int | None = None) -> np.ndarray:
    """Inverse of ``rfftn`` without normalization over the trailing axes of real
    lengths ``shape``: sign +1 DFTs along all but the last axis, then ``irfft``
    along the last (whose bins 0 and n/2 keep only their real parts)."""
    y = np.asarray(y, np.complex128)
    z = y
    if len(shape) > 1:
        # move the halved axis out of the way, transform the others, move it back
        z = np.moveaxis(z, -1, 0)
        z = fftn(z, len(shape) - 1, sign=+1, nthreads=nthreads)
        z = np.moveaxis(z, 0, -1)
    return irfft(z, shape[-1], nthreads=nthreads)
