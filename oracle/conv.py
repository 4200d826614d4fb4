"""Convolutional finite Fourier series (paper Secs. 5.2 and 6), FP64.

Route 1 of the oracle.  Steps, in the paper's order:
 1. FFCs f^[k; L] and rho^_j[k; L] of the samples (eq. (FkLv)).
 2. Product H[k] = f^[k; L] * prod_j rho^_j[k; L]  (eq. (SKfg); for a chain the
    kernels are applied on the right, f * rho_1 * ... * rho_q, and by Thm. f*gP(2)
    their coefficients multiply, Sec. 6.3).
 3. S_K[f, rho](w) = sum_k H[k] phi_k(w), evaluated on the grid (eq. (SKfg)).
 4. Real part (the paper plots Re S_K, Sec. 6.2).

Also: the closed matrix form of Algorithm 3 with N = L (end of Sec. 6.1),
the power form of Algorithm 4 (eq. (MatSqKfgG)) and the all-powers loop of
Algorithm 7 (Sec. 6.3).
"""
from __future__ import annotations

import numpy as np

from .ffc import ffc, sign_w, signed_freqs, synthesize
from .transforms import dft3, idft3


def conv_chain(f: np.ndarray, kernels, return_complex: bool = False,
               adjoint: bool = False) -> np.ndarray:
    """S_K[f, rho_1, ..., rho_q] on Omega_L from samples f and kernel samples rho_j.

    adjoint=True applies the transpose operator (conjugated coefficients), i.e.
    the correlation with the kernels.
    """
    h = ffc(f)
    for p in kernels:
        c = ffc(p)
        h = h * (np.conj(c) if adjoint else c)
    out = synthesize(h)
    return out if return_complex else out.real


def coeff_product(kernels) -> np.ndarray:
    """prod_j rho^_j[k; L] for a chain (the folded coefficient table)."""
    t = None
    for p in kernels:
        c = ffc(p)
        t = c if t is None else t * c
    return t


def conv_with_coeffs(f: np.ndarray, table: np.ndarray, points=None) -> np.ndarray:
    """Re S_K with a given coefficient table, optionally only at some grid points."""
    h = ffc(f) * table
    return synthesize(h, points=points).real


def conv_on_grid(f: np.ndarray, kernels, grid, adjoint: bool = False) -> np.ndarray:
    """Re S_K[f, rho_1, ...] evaluated on a finer (Gx, Gy, Gm) grid, G >= L per axis.

    The coefficients are those of the sampling grid Omega_L; only the evaluation
    points change (Sec. 4.1 eq. (MatSKfonG), Sec. 6.1 eq. (MatSKfgonG)).
    """
    h = ffc(f)
    for p in kernels:
        c = ffc(p)
        h = h * (np.conj(c) if adjoint else c)
    return synthesize(h, grid=grid).real


def _pad_axis(length: int, grid: int) -> np.ndarray:
    """Q[g, t]: weight of L-grid index t at N-grid index g in the zero-padded spectrum.

    Prop. LtoN1D: coefficient k (|k| <= K, L = 2K+1) moves from index tau_L(k) to
    tau_N(k); the rest of the N-spectrum is zero.  Even L: the index L/2 is split in
    halves between tau_N(-L/2) and tau_N(+L/2) (the same index when N = L).
    """
    q = np.zeros((grid, length))
    for t, k in enumerate(signed_freqs(length)):
        if length % 2 == 0 and t == length // 2:
            q[np.mod(-k, grid), t] += 0.5
            q[np.mod(k, grid), t] += 0.5
        else:
            q[np.mod(k, grid), t] = 1.0
    return q


def padded_matrix_form(f: np.ndarray, kernels, grid) -> np.ndarray:
    """Algorithm 3 with N > L: (N_prod / n^2) iDFT_N(W . Q_f . Q_rho), eq. (MatSKfgonG).

    Q is the zero-padded DFT (eq. (Qf)); W = (-1)^{k1+k2} of the signed frequency
    on the N-grid (eq. (W)).  A chain of q kernels multiplies their DFTs, each with
    a factor 1/n, and W enters q times (W . W = 1), as in the power form of Alg. 4.
    """
    m, ny, nx = f.shape
    gx, gy, gm = grid
    n = float(nx * ny * m)
    h = dft3(f)
    for p in kernels:
        h = h * dft3(p) / n
    qx, qy, qt = _pad_axis(nx, gx), _pad_axis(ny, gy), _pad_axis(m, gm)
    big = np.einsum("ct,bs,ar,tsr->cba", qt, qy, qx, h)
    if len(kernels) % 2 == 1:
        big = big * sign_w(gx, gy, gm)
    return (float(gx * gy * gm) / n * idft3(big)).real


def alg3_matrix_form(f: np.ndarray, p: np.ndarray) -> np.ndarray:
    """Algorithm 3 with N = L: S_K[f, rho] = 1/(Lx Ly Lr) * iDFT(W . F^ . P^)."""
    m, ny, nx = f.shape
    w = sign_w(nx, ny, m)
    return (idft3(w * dft3(f) * dft3(p)) / float(nx * ny * m)).real


def alg4_power(f: np.ndarray, p: np.ndarray, q: int) -> np.ndarray:
    """Algorithm 4 with N = L: S^q_K[f, rho] = n/n^(q+1) iDFT(W^q . F^ . P^^q).

    W enters only when q is odd (W . W = 1).
    """
    m, ny, nx = f.shape
    n = float(nx * ny * m)
    h = dft3(f) * dft3(p) ** q
    if q % 2 == 1:
        h = sign_w(nx, ny, m) * h
    return (n / n ** (q + 1) * idft3(h)).real


def alg7_all_powers(f: np.ndarray, p: np.ndarray, q: int) -> list[np.ndarray]:
    """Algorithm 7: one forward DFT, running Hadamard product, q inverse DFTs.

    V := F^; for p = 1..q: H := W . V . P^ ; V_p := iDFT(H) / n^p ; V := H.
    """
    m, ny, nx = f.shape
    n = float(nx * ny * m)
    w = sign_w(nx, ny, m)
    ph = dft3(p)
    v = dft3(f)
    outs = []
    for k in range(1, q + 1):
        h = w * v * ph
        outs.append((idft3(h) / n ** k).real)
        v = h
    return outs


def alg6_naive_recursive(f: np.ndarray, p: np.ndarray, q: int) -> list[np.ndarray]:
    """Algorithm 6: V := f; repeat V_p := S_K[V, rho] on the sampling grid."""
    outs = []
    v = f
    for _ in range(q):
        v = conv_chain(v, [p])
        outs.append(v)
    return outs
