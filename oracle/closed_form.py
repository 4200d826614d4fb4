"""Continuous closed form of (bump field) * (chain of Gaussian x von Mises kernels).

Derivation from the convolution integral of paper Thm. f*gP(1),
(f*rho)(x, theta) = 1/(2pi) int_0^{2pi} int_{R^2} f(y, a) rho(x - y, theta - a) dy da
(eq. (f*gRadialMain)), for f = Gaussian(s) x vonMises(kappa_f, theta0) and
rho = A exp(-|x|^2/2 sigma^2) exp(kappa cos(theta - theta_r)),
A = 1/(2 pi sigma^2 I0(kappa)) (unit Haar mass, eq. (dg)):

* translations: Gaussian widths add, S^2 = s^2 + sigma^2, amplitude 2 pi s^2 sigma^2 / S^2;
* angles: with exp(k cos u) = sum_m I_m(k) e^{i m u}, the normalised circular
  convolution multiplies Fourier coefficients, giving
  I0(kf) I0(k) + 2 sum_{m>=1} I_m(kf) I_m(k) cos(m (theta - theta0 - theta_r)).

A chain multiplies the Bessel ratios I_m(k_j)/I0(k_j), adds the sigma_j^2 and the
theta_j.  The result is periodized over the lattice like the field (eq. (Tf*g)).
"""
from __future__ import annotations

import numpy as np
from scipy.special import ive


def conv_closed_form(bf, chain, nx, ny, m, m_max=200, images=3):
    """Values on Omega_L of f * rho_1 * ... * rho_q (continuous normalisation)."""
    x = -0.5 + np.arange(nx) / nx
    y = -0.5 + np.arange(ny) / ny
    t = 2.0 * np.pi * np.arange(m) / m
    s2 = bf.s ** 2
    big_s2 = s2 + sum(k.sigma ** 2 for k in chain)
    shift = sum(k.theta0 for k in chain)
    mm = np.arange(0, m_max + 1)
    # I_m(kf) e^{-kf} * prod_j I_m(k_j)/I0(k_j); the e^{-kf} is restored below.
    coef = ive(mm, bf.kappa)
    for k in chain:
        coef = coef * ive(mm, k.kappa) / ive(0, k.kappa)
    out = np.zeros((m, ny, nx))
    for b in range(len(bf.weights)):
        cx, cy = bf.centres[b]
        gx = np.zeros(nx)
        gy = np.zeros(ny)
        for l in range(-images, images + 1):
            gx += np.exp(-((x - cx + l) ** 2) / (2 * big_s2))
            gy += np.exp(-((y - cy + l) ** 2) / (2 * big_s2))
        u = t - bf.theta0[b] - shift
        ang = coef[0] + 2.0 * np.sum(coef[1:, None] * np.cos(mm[1:, None] * u[None, :]), axis=0)
        ang = ang * np.exp(bf.kappa)
        amp = bf.weights[b] * s2 / big_s2
        out += amp * ang[:, None, None] * gy[None, :, None] * gx[None, None, :]
    return out


def field_closed_form(bf, nx, ny, m, images=3):
    """The field itself (q = 0 case of conv_closed_form), for self-checks."""
    return conv_closed_form(bf, [], nx, ny, m, images=images)
