"""Finite Fourier coefficients and finite Fourier series on the grid Omega_L.

Paper Sec. 3.2: the FFC (eq. (fkLvMain)) is
    f^[k; L] = 1/|Omega_L| * sum_{w in Omega_L} f(w) * conj(phi_k(w)),
with phi_k(x, y, theta) = exp(2 pi i (k1 x + k2 y)) exp(i k3 theta) (eq. (phik)).
Sec. 4.1, eq. (FkLv) rewrites it through the DFT of the samples:
    f^[k; L] = (-1)^(k1+k2) / (Lx Ly Lr) * F^(tau(k1), tau(k2), tau(k3)),
with tau_L(k) = k mod L (Sec. 2.1 item 3; Annex eq. (tauKk)).

Signed frequencies: array index t in [0, L) stands for k = t if t <= (L-1)//2,
else t - L.  For odd L = 2K+1 this is the paper's set |k| <= K.  For even L
(every size used here) it is {-L/2, ..., L/2-1}; on the grid both (-1)^k and
phi_k(w) are L-periodic in k when L is even, so the choice of representative does
not change any on-grid value.

The finite Fourier series is evaluated by explicit synthesis
    S(w) = sum_k c[k] phi_k(w),
with phi_k at x = -1/2 + a/G written exactly as (-1)^k * exp(2 pi i ((k a) mod G)/G).
G may exceed L: that is the evaluation of S_K on a finer grid (Sec. 4.1, eq.
(MatSKfonG)).  The paper states it for odd L only.  For even L the index L/2 holds
both frequencies +-L/2 (they coincide on Omega_L); off the grid this oracle splits
it in halves between phi_{-L/2} and phi_{+L/2}, so that a real field stays real.
On Omega_L itself the split changes nothing.
"""
from __future__ import annotations

import numpy as np

from .transforms import dft3


def signed_freqs(length: int) -> np.ndarray:
    t = np.arange(length, dtype=np.int64)
    return np.where(t <= (length - 1) // 2, t, t - length)


def tau(k, length: int):
    """tau_L(k) = k mod L (non-negative remainder)."""
    return np.mod(k, length)


def sign_w(nx: int, ny: int, m: int) -> np.ndarray:
    """W[t3, t2, t1] = (-1)^(k1 + k2) with k the signed frequency of the index."""
    k1 = signed_freqs(nx)
    k2 = signed_freqs(ny)
    s1 = np.where(k1 % 2 == 0, 1.0, -1.0)
    s2 = np.where(k2 % 2 == 0, 1.0, -1.0)
    w2 = np.outer(s2, s1)
    return np.broadcast_to(w2[None, :, :], (m, ny, nx)).copy()


def ffc(samples: np.ndarray) -> np.ndarray:
    """All FFCs f^[k; L] (eq. (FkLv)), stored at array index tau(k)."""
    m, ny, nx = samples.shape[-3:]
    fh = dft3(samples)
    return sign_w(nx, ny, m) * fh / float(nx * ny * m)


def ffc_direct(samples: np.ndarray, k: tuple[int, int, int]) -> complex:
    """One FFC by the literal grid sum of eq. (fkLvMain); for tiny grids only."""
    m, ny, nx = samples.shape
    x = -0.5 + np.arange(nx) / nx
    y = -0.5 + np.arange(ny) / ny
    t = 2.0 * np.pi * np.arange(m) / m
    phase = np.exp(-2j * np.pi * (k[0] * x[None, None, :] + k[1] * y[None, :, None])) * \
        np.exp(-1j * k[2] * t[:, None, None])
    return complex(np.sum(samples * phase) / (nx * ny * m))


def _phi_axis(length: int, points: np.ndarray, grid: int, spatial: bool) -> np.ndarray:
    """E[a, t] = value of the 1-D factor of phi_k at point index a of a G-grid.

    spatial axis: x_a = -1/2 + a/G, factor exp(2 pi i k x_a) = (-1)^k exp(2 pi i (k a mod G)/G)
    angular axis: theta_a = 2 pi a / G, factor exp(i k theta_a) = exp(2 pi i (k a mod G)/G)
    """
    k = signed_freqs(length)
    a = np.asarray(points, dtype=np.int64)
    red = np.mod(np.outer(a, k), grid).astype(np.float64)
    e = np.exp(2j * np.pi * red / grid)
    if length % 2 == 0:
        # Nyquist index: average of the factors of k = -L/2 and k = +L/2
        h = length // 2
        plus = np.exp(2j * np.pi * np.mod(a * h, grid).astype(np.float64) / grid)
        e[:, h] = 0.5 * (e[:, h] + plus)
    if spatial:
        e = e * np.where(k % 2 == 0, 1.0, -1.0)[None, :]
    return e


def synthesize(coeffs: np.ndarray, grid=None, points=None) -> np.ndarray:
    """S(w) = sum_k c[k] phi_k(w) on a tensor-product set of grid points.

    grid   = (Gx, Gy, Gm) sizes of the evaluation grid (default: the coefficient grid).
    points = (ax, ay, at) index lists on that grid (default: all points).
    """
    m, ny, nx = coeffs.shape[-3:]
    if grid is None:
        grid = (nx, ny, m)
    gx, gy, gm = grid
    if points is None:
        points = (np.arange(gx), np.arange(gy), np.arange(gm))
    ax, ay, at = points
    ex = _phi_axis(nx, ax, gx, True)
    ey = _phi_axis(ny, ay, gy, True)
    et = _phi_axis(m, at, gm, False)
    c = np.asarray(coeffs, dtype=np.complex128)
    out = np.moveaxis(np.moveaxis(c, -1, -1) @ ex.T, -1, -1)          # x
    out = np.moveaxis(np.moveaxis(out, -2, -1) @ ey.T, -1, -2)        # y
    out = np.moveaxis(np.moveaxis(out, -3, -1) @ et.T, -1, -3)        # theta
    return out
