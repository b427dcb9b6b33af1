"""Seeded synthetic workloads shared by the tests, the benchmark and the oracle checks.

This module only draws random numbers and picks sizes; it holds none of the
transform's arithmetic, so the GPU library and the CPU oracle can both be fed
from it without sharing any part of the method.

Workload recipes (all synthetic; the paper measures no public dataset):
  * values: real and imaginary parts i.i.d. uniform on [-1, 1), drawn in FP64
    with numpy's PCG64 from a recorded seed and rounded to nearest for FP32;
  * uneven batch: sizes log-uniform on [64, 65536], 60% powers of two, 30%
    7-smooth non-powers of two, 10% primes, each with a batch of 1..32;
  * serving trace: Poisson arrivals, rank 1..3, total points log-uniform on
    [2^8, 2^22] rounded to 7-smooth, batch 1..64, FP32/FP64 80/20,
    forward/inverse 50/50.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "uniform_complex", "is_prime", "is_smooth", "smooth_numbers", "nearest_smooth",
    "nearest_prime", "uneven_batch", "UnevenItem", "serve_trace", "Request",
    "split_smooth",
]


def uniform_complex(count: int, seed: int, dtype=np.complex128) -> np.ndarray:
    """`count` complex values with re, im i.i.d. U[-1, 1) (PCG64, FP64, then cast)."""
    rng = np.random.default_rng(seed)
    re = rng.uniform(-1.0, 1.0, int(count))
    im = rng.uniform(-1.0, 1.0, int(count))
    z = re + 1j * im
    return z.astype(dtype)


def is_prime(n: int) -> bool:
    if n < 2:
        return False
    if n % 2 == 0:
        return n == 2
    f = 3
    while f * f <= n:
        if n % f == 0:
            return False
        f += 2
    return True


def is_smooth(n: int, bound: int = 7) -> bool:
    if n < 1:
        return False
    for p in (2, 3, 5, 7):
        if p > bound:
            break
        while n % p == 0:
            n //= p
    return n == 1


def smooth_numbers(lo: int, hi: int, bound: int = 7) -> list[int]:
    return [n for n in range(max(1, lo), hi + 1) if is_smooth(n, bound)]


def nearest_smooth(x: float, candidates: list[int]) -> int:
    """Candidate nearest to x in log distance."""
    lx = math.log(x)
    return min(candidates, key=lambda c: (abs(math.log(c) - lx), c))


def nearest_prime(x: float, lo: int, hi: int) -> int:
    c = int(round(x))
    for d in range(0, hi):
        for cand in (c - d, c + d):
            if lo <= cand <= hi and is_prime(cand):
                return cand
    raise ValueError("no prime in range")


@dataclass
class UnevenItem:
    n: int
    batch: int
    cls: str          # "pow2" | "smooth" | "prime"
    seed: int


def uneven_batch(count: int = 10000, seed: int = 4, lo: int = 64, hi: int = 65536) -> list[UnevenItem]:
    """Uneven batch of 1D transforms: log-uniform sizes, class mix 60/30/10."""
    rng = np.random.default_rng(seed)
    smooth = [n for n in smooth_numbers(lo, hi) if n & (n - 1)]
    pmax = max(p for p in range(hi - 20, hi) if is_prime(p))
    items = []
    for i in range(count):
        u = rng.uniform()
        x = math.exp(rng.uniform(math.log(lo), math.log(hi)))
        if u < 0.6:
            n = 1 << int(round(math.log2(x)))
            n = min(max(n, lo), hi)
            cls = "pow2"
        elif u < 0.9:
            n = nearest_smooth(x, smooth)
            cls = "smooth"
        else:
            n = nearest_prime(x, 67, pmax)
            cls = "prime"
        b = int(rng.integers(1, 33))
        items.append(UnevenItem(n=n, batch=b, cls=cls, seed=seed * 1000003 + i))
    return items


def split_smooth(total: int, rank: int) -> list[int]:
    """Split a 7-smooth `total` into `rank` near-equal 7-smooth factors."""
    f = []
    m = total
    for p in (2, 3, 5, 7):
        while m % p == 0:
            f.append(p)
            m //= p
    assert m == 1
    dims = [1] * rank
    for p in sorted(f, reverse=True):
        i = min(range(rank), key=lambda j: dims[j])
        dims[i] *= p
    return sorted(dims, reverse=True)


@dataclass
class Request:
    arrival: float               # seconds since trace start
    dims: list[int]              # transform shape (row-major, contiguous)
    batch: int
    prec: str                    # "c32" | "c64"
    sign: int
    seed: int
    meta: dict = field(default_factory=dict)

    @property
    def points(self) -> int:
        return int(np.prod(self.dims)) * self.batch


def serve_trace(count: int, rate_hz: float, seed: int = 5, lo_exp: int = 8, hi_exp: int = 22,
                max_batch: int = 64) -> list[Request]:
    """Poisson arrivals of FFT requests (the serving workload recipe)."""
    rng = np.random.default_rng(seed)
    smooth = smooth_numbers(1 << lo_exp, 1 << hi_exp)
    t = 0.0
    out = []
    for i in range(count):
        t += rng.exponential(1.0 / rate_hz)
        rank = int(rng.integers(1, 4))
        x = math.exp(rng.uniform(math.log(2.0 ** lo_exp), math.log(2.0 ** hi_exp)))
        total = nearest_smooth(x, smooth)
        dims = split_smooth(total, rank)
        batch = int(rng.integers(1, max_batch + 1))
        # keep one request's input under 2^22 points * batch budget used by the recipe
        prec = "c32" if rng.uniform() < 0.8 else "c64"
        sign = -1 if rng.uniform() < 0.5 else 1
        out.append(Request(arrival=t, dims=dims, batch=batch, prec=prec, sign=sign,
                           seed=seed * 7919 + i))
    return out
