"""3-D DFT / iDFT exactly as defined in paper Sec. 2.3, eqs. (3DFT), (3iDFT).

(3DFT):  X^(l,m,n)  = sum_{i,j,k} X(i,j,k) e^{-2 pi i (i-1)(l-1)/L} e^{-2 pi i (j-1)(m-1)/M}
                                           e^{-2 pi i (k-1)(n-1)/N}
(3iDFT): X~(l,m,n)  = 1/(LMN) * the same sum with e^{+...}

Implemented with 0-based indices as one explicit dense FP64 matrix per axis.  The
exponent uses the reduced integer product (k*i) mod L so that no large argument
reaches exp().  This is the textbook definition, one axis at a time (the 3-D
kernel is a product of three 1-D kernels), with no factorisation.

For large arrays (dense cost above DENSE_LIMIT multiply-adds per axis) the same
1-D sum along an axis is evaluated with numpy's FFT, a library primitive for
exactly this DFT; tests/test_oracle_transforms.py checks that both evaluations
agree.  This file is test infrastructure: only the tests, the smoke check and
the benchmark's CPU baseline use it.
"""
from __future__ import annotations

import numpy as np


def dft_matrix(length: int, sign: int = -1) -> np.ndarray:
    """D[k, i] = exp(sign * 2 pi i * ((k*i) mod L) / L)."""
    idx = np.arange(length, dtype=np.int64)
    prod = np.outer(idx, idx) % length
    return np.exp(sign * 2j * np.pi * prod.astype(np.float64) / length)


# dense per-axis products above this many multiply-adds use numpy's FFT instead
DENSE_LIMIT = 1 << 30


def _apply_axis(a: np.ndarray, mat: np.ndarray, axis: int) -> np.ndarray:
    # out[..., k, ...] = sum_i mat[k, i] a[..., i, ...]
    a = np.moveaxis(a, axis, -1)
    out = a @ mat.T
    return np.moveaxis(out, -1, axis)


def _dft_axis(a: np.ndarray, axis: int, sign: int) -> np.ndarray:
    """out[k] = sum_i exp(sign 2 pi i k i / L) a[i] along one axis (un-normalised)."""
    length = a.shape[axis]
    if a.size * length < DENSE_LIMIT:
        return _apply_axis(a, dft_matrix(length, sign), axis)
    if sign < 0:
        return np.fft.fft(a, axis=axis)
    return np.fft.ifft(a, axis=axis) * float(length)


def axis_routes(shape) -> dict:
    """Which evaluation _dft_axis takes along each axis of a [theta][y][x] array."""
    size = int(np.prod(shape))
    m, ny, nx = shape[-3:]
    return {name: ("dense" if size * length < DENSE_LIMIT else "fft")
            for name, length in (("x", nx), ("y", ny), ("theta", m))}


def dft3(a: np.ndarray) -> np.ndarray:
    """Un-normalised 3-D DFT (3DFT) of an array laid out [theta][y][x]."""
    a = np.asarray(a, dtype=np.complex128)
    m, ny, nx = a.shape[-3:]
    out = _dft_axis(a, a.ndim - 1, -1)
    out = _dft_axis(out, a.ndim - 2, -1)
    out = _dft_axis(out, a.ndim - 3, -1)
    return out


def idft3(a: np.ndarray) -> np.ndarray:
    """3-D inverse DFT (3iDFT), including the 1/(LMN) factor."""
    a = np.asarray(a, dtype=np.complex128)
    m, ny, nx = a.shape[-3:]
    out = _dft_axis(a, a.ndim - 1, +1)
    out = _dft_axis(out, a.ndim - 2, +1)
    out = _dft_axis(out, a.ndim - 3, +1)
    return out / float(nx * ny * m)


def dft1(v: np.ndarray, sign: int = -1) -> np.ndarray:
    """1-D DFT (un-normalised) along the last axis; the 1-D case of (3DFT)."""
    v = np.asarray(v, dtype=np.complex128)
    return _dft_axis(v, v.ndim - 1, sign)
