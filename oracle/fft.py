"""Naive FP64 transforms for the oracle (test infrastructure only).

* ``dft_axis``   -- the discrete Fourier transform written out as a matrix
                    product (definition; O(n^2)); used only to pin ``fft_axis``.
* ``fft_axis``   -- recursive decimation-in-time mixed-radix FFT (radix = the
                    largest divisor <= 16; the definition for short or prime
                    lengths).  Unnormalised:
                    X_j = sum_a x_a exp(sign * 2 pi i j a / n).
* ``forward3`` / ``inverse3`` -- the half-integer-shifted 3D transforms of the
  section "Numerical procedure" (k grid at half-integer points, r grid at
  integer points, which keeps k = 0 off the grid):

      X(k_j) = dV * sum_a x_a exp(-2 pi i (j + 1/2) . a / n)
      x_a    = (N dV)^-1 * sum_j X_j exp(+2 pi i (j + 1/2) . a / n)

  with the product taken over the three axes.  Writing
  exp(-2 pi i (j+1/2) a / n) = exp(-i pi a / n) exp(-2 pi i j a / n) lets the
  unshifted FFT do the sum; that factorisation is exact.
"""
from __future__ import annotations

import numpy as np


SMALL = 16   # lengths up to this are transformed by the definition (a matrix product)


def _radix(n: int) -> int:
    """Largest divisor of n not exceeding SMALL (n itself when n is prime)."""
    for p in range(min(SMALL, n - 1), 1, -1):
        if n % p == 0:
            return p
    return n


def dft_axis(x, axis: int = -1, sign: int = -1, shift: float = 0.0):
    """Brute-force DFT along ``axis``: X_j = sum_a x_a exp(sign 2 pi i (j+shift) a / n)."""
    x = np.moveaxis(np.asarray(x, dtype=np.complex128), axis, -1)
    n = x.shape[-1]
    j = np.arange(n) + shift
    a = np.arange(n)
    w = np.exp(sign * 2j * np.pi * np.outer(j, a) / n)
    return np.moveaxis(x @ w.T, -1, axis)


def _fft_rows(x: np.ndarray, sign: int) -> np.ndarray:
    """DFT of every row of a contiguous [B, n] array, by decimation in time.
    With n = p m (p the radix chosen by ``_radix``) write a = r + p s and
    k = k1 + m k2; then
        X[k1 + m k2] = sum_r exp(sign 2 pi i r k2 / p)
                             * exp(sign 2 pi i r k1 / n) * Y_r[k1],
    where Y_r is the length-m DFT of the subsequence x[r::p].  The p
    subsequences of all rows are transformed together (one recursive call)."""
    b, n = x.shape
    p = _radix(n)
    if n <= SMALL or p == n:   # short or prime length: the definition
        a = np.arange(n)
        return x @ np.exp(sign * 2j * np.pi * np.outer(a, a) / n).T
    m = n // p
    sub = np.ascontiguousarray(x.reshape(b, m, p).transpose(0, 2, 1)).reshape(b * p, m)
    y = _fft_rows(sub, sign).reshape(b, p, m)                              # [b, r, k1]
    r = np.arange(p)[:, None]
    k1 = np.arange(m)[None, :]
    y = y * np.exp(sign * 2j * np.pi * r * k1 / n)
    wp = np.exp(sign * 2j * np.pi * np.outer(np.arange(p), np.arange(p)) / p)   # [k2, r]
    return np.einsum("qr,brk->bqk", wp, y).reshape(b, n)                         # [b, k2, k1]


def _fft_last(x: np.ndarray, sign: int) -> np.ndarray:
    shape = x.shape
    return _fft_rows(np.ascontiguousarray(x).reshape(-1, shape[-1]), sign).reshape(shape)


def fft_axis(x, axis: int = -1, sign: int = -1):
    """Unnormalised FFT along ``axis`` (sign -1 forward, +1 backward)."""
    x = np.moveaxis(np.asarray(x, dtype=np.complex128), axis, -1)
    return np.moveaxis(_fft_last(np.ascontiguousarray(x), sign), -1, axis)


def _half_phase(n: int, sign: int) -> np.ndarray:
    return np.exp(sign * 1j * np.pi * np.arange(n) / n)


def forward3(x, dv: float):
    """Shifted forward transform of a real or complex field [..., nz, ny, nx]."""
    y = np.asarray(x, dtype=np.complex128)
    for axis in (-1, -2, -3):
        n = y.shape[axis]
        shape = [1] * y.ndim
        shape[axis] = n
        y = fft_axis(y * _half_phase(n, -1).reshape(shape), axis=axis, sign=-1)
    return dv * y


def inverse3(X, dv: float):
    """Shifted inverse transform; returns complex [..., nz, ny, nx]."""
    y = np.asarray(X, dtype=np.complex128)
    n_tot = 1
    for axis in (-1, -2, -3):
        n = y.shape[axis]
        n_tot *= n
        shape = [1] * y.ndim
        shape[axis] = n
        y = fft_axis(y, axis=axis, sign=+1) * _half_phase(n, +1).reshape(shape)
    return y / (n_tot * dv)


def forward3_bruteforce(x, dv: float):
    """Shifted forward transform by direct summation along each axis (pins only)."""
    y = np.asarray(x, dtype=np.complex128)
    for axis in (-1, -2, -3):
        y = dft_axis(y, axis=axis, sign=-1, shift=0.5)
    return dv * y


def inverse3_bruteforce(X, dv: float):
    y = np.asarray(X, dtype=np.complex128)
    n_tot = 1
    for axis in (-1, -2, -3):
        n = y.shape[axis]
        n_tot *= n
        # x_a = sum_j X_j exp(+2 pi i (j+1/2) a / n): the transpose of the shifted matrix
        ym = np.moveaxis(y, axis, -1)
        a = np.arange(n)
        j = np.arange(n) + 0.5
        w = np.exp(+2j * np.pi * np.outer(a, j) / n)
        y = np.moveaxis(ym @ w.T, -1, axis)
    return y / (n_tot * dv)
