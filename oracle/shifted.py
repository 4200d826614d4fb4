"""Kernels that are sums of SE(2)-shifts of one kernel radial in translations.

Test infrastructure only (see the package docstring).

Sec. 1 proposes approximating a general kernel f2 by sum_k a_k rho_k, where the rho_k are
SE(2)-shifts of one rho that is radial in translations, so that f * f2 ~ sum_k a_k f * rho_k.
A shift is read as the left action of s_k = (t_k, R_phi_k) (group law eq. (SE2law)):
    rho_k(g) = rho(s_k^{-1} o g).
A shifted rho is no longer radial, so the product of coefficients (Thm. f*gP) does not
apply to rho_k itself.  It applies after moving the shift onto the field: with
h = (y, alpha), g = (x, theta),
    rho_k(h^{-1} o g) = rho(R_{-phi}(R_{-alpha}(x - y) - t), theta - alpha - phi)
                      = rho(x - y - R_alpha t, theta - alpha - phi)
since rho ignores rotations of its translation part (twice).  Hence
    f * rho_k = f_k * rho  (the reduced convolution of eq. (f*gRadialMain)),
    f_k(y, alpha) = f(y - R_{alpha - phi} t, alpha - phi):
every theta-slice alpha of f translated by R_alpha t, then the whole field shifted by phi
in theta.  On the finite Fourier series of f this is, per term,
 1. the spatial FFC of every theta-slice, F2[k1, k2, alpha] (eq. (fkLvMain) in x, y);
 2. times the translation phase e^{-2 pi i (k1, k2) . R_alpha t} (exact for the
    trigonometric polynomial in x, y);
 3. the FFC in theta (eq. (fkLvMain) in theta), times the shift phase e^{-i k3 phi};
and then, summed over the terms with weights a_k, times rho^[k; L] and synthesised
(eq. (SKfg)).  For even grid lengths the Nyquist index stands for +-L/2 in halves (the
reading used for evaluation off the grid), so its phase is the real cos(pi L tau): a real
field stays real.  When every R_alpha t_k is a grid vector and every phi_k a grid angle
(M = 4 with square grids, for instance) the shifts are exact index rolls and the result
equals the direct quadrature of f with the shifted kernel sum.
"""
from __future__ import annotations

import numpy as np

from .ffc import signed_freqs, synthesize, ffc
from .transforms import dft_matrix


def axis_phase(length: int, tau: np.ndarray) -> np.ndarray:
    """E[a, t] = e^{-2 pi i k_t tau_a} for signed frequency k_t of index t, and the real
    cos(pi L tau_a) at the Nyquist index of an even length (the two signs in halves)."""
    k = signed_freqs(length).astype(np.float64)
    tau = np.asarray(tau, dtype=np.float64)
    e = np.exp(-2j * np.pi * np.outer(tau, k))
    if length % 2 == 0:
        e[:, length // 2] = np.cos(np.pi * length * tau)
    return e


def slice_translation(alpha: np.ndarray, tx: float, ty: float):
    """R_alpha t: the translation of the theta-slice alpha under the shift by t."""
    return np.cos(alpha) * tx - np.sin(alpha) * ty, np.sin(alpha) * tx + np.cos(alpha) * ty


def shift_coeffs(f: np.ndarray, shifts, weights) -> np.ndarray:
    """FFCs of sum_k a_k f_k, f_k the field moved by the shift s_k = (tx, ty, phi):
    steps 1-3 of the module docstring, stored at array index tau(k) like ffc()."""
    f = np.asarray(f, dtype=np.complex128)
    m, ny, nx = f.shape
    # 1. spatial FFC of every theta-slice: (-1)^{k1+k2}/(Nx Ny) DFT_xy (eq. (FkLv) in x, y)
    dx = dft_matrix(nx, -1)
    dy = dft_matrix(ny, -1)
    f2 = f @ dx.T                                # x: f2[t, j, k1] = sum_i D[k1, i] f[t, j, i]
    f2 = np.matmul(dy, f2)                       # y: sum_j D[k2, j] f2[t, j, k1]
    sx = np.where(signed_freqs(nx) % 2 == 0, 1.0, -1.0)
    sy = np.where(signed_freqs(ny) % 2 == 0, 1.0, -1.0)
    f2 = f2 * (sy[:, None] * sx[None, :])[None] / float(nx * ny)
    alpha = 2.0 * np.pi * np.arange(m) / m
    k3 = signed_freqs(m).astype(np.float64)
    dt = dft_matrix(m, -1) / float(m)            # theta FFC: (1/M) sum_alpha e^{-i k3 alpha}
    out = np.zeros((m, ny, nx), np.complex128)
    for (tx, ty, phi), a in zip(shifts, weights):
        # 2. translation of slice alpha by R_alpha t
        ux, uy = slice_translation(alpha, tx, ty)
        ph = axis_phase(ny, uy)[:, :, None] * axis_phase(nx, ux)[:, None, :]   # [alpha][k2][k1]
        g = f2 * ph
        # 3. FFC in theta, shift by phi
        gh = (dt @ g.reshape(m, -1)).reshape(m, ny, nx)
        sh = np.exp(-1j * k3 * phi)
        if m % 2 == 0:
            sh[m // 2] = np.cos(0.5 * m * phi)
        out += a * sh[:, None, None] * gh
    return out


def shifted_sum_conv(f: np.ndarray, p: np.ndarray, shifts, weights, return_complex: bool = False):
    """S_K[f, sum_k a_k rho_k] on Omega_L: the shifted field coefficients times the FFCs of
    the radial kernel samples p (Thm. f*gP), synthesised on the grid (eq. (SKfg))."""
    h = shift_coeffs(f, shifts, weights) * ffc(p)
    out = synthesize(h)
    return out if return_complex else out.real


def shifted_kernel_function(rho, shifts, weights):
    """The kernel sum_k a_k rho(s_k^{-1} o (x, theta)) as a plain function, with the
    explicit rotation R_{-phi} (eq. (SE2law): s^{-1} o (x, R) = (R_{-phi}(x - t), R_{-phi} R))."""
    def kern(x, y, t):
        acc = 0.0
        for (tx, ty, phi), a in zip(shifts, weights):
            c, s = np.cos(phi), np.sin(phi)
            ux, uy = x - tx, y - ty
            acc = acc + a * rho(c * ux + s * uy, -s * ux + c * uy, t - phi)
        return acc
    return kern
