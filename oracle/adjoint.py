"""Gradients of the convolutional FFS (FP64 oracle).

For out = S_K[f, rho] on the grid and a loss with dL/dout = g (real):

* w.r.t. the field samples F: the transpose of F -> out, i.e. the same series
  with conjugated kernel coefficients (correlation with the kernel).
* w.r.t. the kernel samples P: out depends linearly on P through
  rho^[k; L] = (-1)^{k1+k2} P^[k] / n (eq. (FkLv)); differentiating
  out(w_a) = sum_k f^[k] rho^[k] phi_k(w_a) gives
      dL/dP = Re S_K[g, conj(f^)],
  the series of g with the conjugated FFCs of the field as coefficients.
* w.r.t. a radial profile prof[q][l] (P = sum_q prof[q][l] H_q, with H_q the
  lattice-periodized hat basis in r = |x|): dL/dprof[q][l] = sum_ji H_q[j,i] dL/dP[l,j,i].

`grad_kernel_direct` evaluates dL/dP from the grid form of the convolution for
even sizes, out[a] = (1/n) sum_i F[i] P[a - i + (Nx/2, Ny/2, 0)] (all indices mod
the grid), with explicit loops: tiny grids only.
"""
from __future__ import annotations

import numpy as np

from .conv import conv_chain, conv_with_coeffs
from .ffc import ffc
from .kernels import hat_weights


def grad_field(g, kernels):
    """dL/dF for dL/dout = g."""
    return conv_chain(g, kernels, adjoint=True)


def grad_kernel_samples(f, g, other_kernels=()):
    """dL/dP_j for out = S_K[f, rho_j, others], dL/dout = g."""
    table = np.conj(ffc(f))
    for p in other_kernels:
        table = table * np.conj(ffc(p))
    return conv_with_coeffs(g, table)


def grad_kernel_direct(f, g):
    """Explicit-loop dL/dP from the grid form of the convolution (even Nx, Ny; tiny grids)."""
    m, ny, nx = f.shape
    n = nx * ny * m
    out = np.zeros_like(f)
    for c in range(m):
        for b in range(ny):
            for a in range(nx):
                # P index (c, b, a) is hit by out[l', j', i'] with input F[(l'-c), (j'-b+ny/2), (i'-a+nx/2)]
                acc = 0.0
                for l2 in range(m):
                    for j2 in range(ny):
                        for i2 in range(nx):
                            acc += g[l2, j2, i2] * f[(l2 - c) % m, (j2 - b + ny // 2) % ny, (i2 - a + nx // 2) % nx]
                out[c, b, a] = acc / n
    return out


def profile_basis(nx, ny, n_knots, r_max, images=2):
    """H[q, j, i] = sum_images hat_q(|x_ij + image|) on the spatial grid."""
    x = -0.5 + np.arange(nx) / nx
    y = -0.5 + np.arange(ny) / ny
    basis = np.zeros((n_knots, ny, nx))
    for l1 in range(-images, images + 1):
        for l2 in range(-images, images + 1):
            r = np.sqrt((x[None, :] + l1) ** 2 + (y[:, None] + l2) ** 2)
            basis += hat_weights(r, n_knots, r_max)
    return basis


def grad_profile(grad_p_samples, n_knots, r_max):
    """dL/dprof[q][l] from dL/dP[l][j][i] (one field or summed over a batch)."""
    gp = np.asarray(grad_p_samples)
    if gp.ndim == 4:
        gp = gp.sum(axis=0)
    m, ny, nx = gp.shape
    basis = profile_basis(nx, ny, n_knots, r_max)
    return np.einsum("qji,lji->ql", basis, gp)
