"""Route 2 of the oracle: direct quadrature of the SE(2) coset convolution.

Paper Sec. 5.1: (f1 * f2)(x, R) = int int f1(y, S) f2(S^{-1}(x - y), S^{-1} R) dy dS
(eq. (f*g)) with the Haar measure dg = dx dtheta / 2pi (eq. (dg)); on the coset
space the field is periodized and the kernel is summed over lattice images
(eqs. (oslash), (Tf*g)).  Nothing here assumes the kernel is radial: the
rotation R_{-theta_l} is applied explicitly, so a non-radial kernel gives a
different answer from the Fourier route.

The image-summed kernel is tabulated in numpy (explicit rotation, images
l in {-R..R}^2); the O(n^2) rectangle-rule sum runs in plain C (csrc/quad.c).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "csrc", "quad.c")
_LIB = os.path.join(_HERE, "csrc", "libquad.so")
_lib = None


def build(force: bool = False) -> str:
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", _SRC, "-o", _LIB])
    return _LIB


def _load():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(_LIB)
        lib.quad_sum.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                 ctypes.c_void_p, ctypes.c_void_p]
        lib.quad_sum.restype = None
        _lib = lib
    return _lib


def kernel_table(rho, nx, ny, m, images=2):
    """K[l][dc][dj][di] = sum_images rho(R_{-theta_l}(di/nx - l1, dj/ny - l2), 2 pi dc/m)."""
    di = np.arange(-(nx - 1), nx) / nx
    dj = np.arange(-(ny - 1), ny) / ny
    tab = np.zeros((m, m, 2 * ny - 1, 2 * nx - 1))
    dth = 2.0 * np.pi * np.arange(m) / m
    for l in range(m):
        a = 2.0 * np.pi * l / m
        ca, sa = np.cos(a), np.sin(a)
        for l1 in range(-images, images + 1):
            for l2 in range(-images, images + 1):
                vx = di[None, :] - l1
                vy = dj[:, None] - l2
                # R_{-a} v = (cos a vx + sin a vy, -sin a vx + cos a vy)
                rx = ca * vx + sa * vy
                ry = -sa * vx + ca * vy
                tab[l] += rho(rx[None, :, :], ry[None, :, :], dth[:, None, None])
    return tab


def quadrature_conv(f: np.ndarray, rho, images=2) -> np.ndarray:
    """Rectangle-rule value of (f~ (/) rho) at every point of Omega_L."""
    f = np.ascontiguousarray(f, dtype=np.float64)
    m, ny, nx = f.shape
    tab = np.ascontiguousarray(kernel_table(rho, nx, ny, m, images))
    out = np.empty_like(f)
    _load().quad_sum(f.ctypes.data, nx, ny, m, tab.ctypes.data, out.ctypes.data)
    return out


def quadrature_chain(f: np.ndarray, rhos, images=2) -> np.ndarray:
    """(...((f * rho_1) * rho_2) ...) applied one kernel at a time on the grid."""
    out = f
    for rho in rhos:
        out = quadrature_conv(out, rho, images)
    return out
