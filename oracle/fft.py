"""Naive recursive mixed-radix DFT (test infrastructure only).

Convention (plane-wave expansion on the periodic grid):
  forward   X~(m) = (1/M) sum_r X(r) exp(-i G_m . r)
  inverse   X(r)  = sum_m X~(m) exp(+i G_m . r)

Along one axis of length N = p*m (p the smallest prime factor, p in
{2, 3, 5}): decimate in time into p interleaved sub-sequences, transform
each recursively, multiply by twiddles exp(-+2 pi i r k / N) and combine
with a plain size-p DFT. No blocking, no reordering tricks: every step is
the textbook Cooley-Tukey identity. Pinned against a direct O(N^2) DFT on
8^3 grids and against an independent library FFT in the tests.
"""
from __future__ import annotations

import numpy as np


def _smallest_factor(n: int) -> int:
    for p in (2, 3, 5):
        if n % p == 0:
            return p
    raise ValueError(f"size {n} is not 5-smooth")


def dft1(x: np.ndarray, axis: int, sign: int) -> np.ndarray:
    """Unnormalised DFT along `axis` with kernel exp(sign * 2 pi i j k / N)."""
    x = np.moveaxis(np.asarray(x, dtype=np.complex128), axis, -1)
    y = _dft_last(x, sign)
    return np.moveaxis(y, -1, axis)


def _dft_last(x: np.ndarray, sign: int) -> np.ndarray:
    N = x.shape[-1]
    if N == 1:
        return x.copy()
    p = _smallest_factor(N)
    m = N // p
    # sub-sequences x[r::p], each transformed with length m
    subs = [_dft_last(x[..., r::p], sign) for r in range(p)]
    k = np.arange(m)
    out = np.empty(x.shape, dtype=np.complex128)
    for q in range(p):
        acc = np.zeros(x.shape[:-1] + (m,), dtype=np.complex128)
        for r in range(p):
            # exp(sign 2 pi i r (k + m q) / N)
            ang = sign * 2.0 * np.pi * (r * (k + m * q) % N) / N
            acc = acc + subs[r] * np.exp(1j * ang)
        out[..., q * m:(q + 1) * m] = acc
    return out


def fft3(x: np.ndarray) -> np.ndarray:
    """Forward 3D transform, normalised by 1/M (plane-wave coefficients)."""
    y = np.asarray(x, dtype=np.complex128)
    for ax in range(3):
        y = dft1(y, ax, -1)
    return y / y.size


def ifft3(x: np.ndarray) -> np.ndarray:
    """Inverse 3D transform (sum over plane waves, no normalisation)."""
    y = np.asarray(x, dtype=np.complex128)
    for ax in range(3):
        y = dft1(y, ax, +1)
    return y


def direct_dft3(x: np.ndarray, sign: int = -1) -> np.ndarray:
    """O(M^2) textbook DFT, used only as a pin for the fast transform."""
    n1, n2, n3 = x.shape
    out = np.zeros(x.shape, dtype=np.complex128)
    idx = np.indices(x.shape).reshape(3, -1)
    flat = x.reshape(-1)
    for a in range(n1):
        for b in range(n2):
            for c in range(n3):
                ph = (a * idx[0] / n1 + b * idx[1] / n2 + c * idx[2] / n3)
                out[a, b, c] = np.sum(flat * np.exp(sign * 2j * np.pi * ph))
    return out
