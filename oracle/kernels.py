"""Kernel samplers for the oracle (FP64).

A kernel rho: SE(2) -> R is radial in translations when rho(Sx, R) = rho(x, R)
for every rotation S (paper Sec. 5.1, footnote to Thm. f*gP).  The samplers
return the lattice-periodized kernel (eq. (TH)) on Omega_L, layout [theta][y][x].

The test kernels are:
* Gaussian x von Mises:  exp(-|x|^2 / (2 sigma^2)) * exp(kappa cos(theta - theta0))
  (radial in translations; the isotropic case of the paper's deformed Gaussians,
  eq. (fHsnu), with a von Mises angular factor).
* anisotropic Gaussian (NOT radial): the negative control.
* radial profile: piecewise-linear hat basis in r = |x| times free angular samples.

Normalisation "continuous" divides by the Haar mass
(1/2pi) int int rho dx dtheta = 2 pi sigma^2 I0(kappa) (eq. (dg));
"discrete" divides by the grid mean so that rho^[0; L] = 1 exactly.
"""
from __future__ import annotations

import numpy as np
from scipy.special import ive

_IMAGES = 2


def _grid(nx, ny, m):
    x = -0.5 + np.arange(nx) / nx
    y = -0.5 + np.arange(ny) / ny
    t = 2.0 * np.pi * np.arange(m) / m
    return x, y, t


def _periodized_radial_2d(nx, ny, g, images=_IMAGES):
    """G[j, i] = sum_l g(|x_ij + l|) over lattice images l in {-R..R}^2."""
    x, y, _ = _grid(nx, ny, 1)
    acc = np.zeros((ny, nx))
    for l1 in range(-images, images + 1):
        for l2 in range(-images, images + 1):
            dx = x[None, :] + l1
            dy = y[:, None] + l2
            acc += g(np.sqrt(dx * dx + dy * dy))
    return acc


def gauss_vm(nx, ny, m, sigma, kappa, theta0=0.0, normalize="discrete"):
    x, y, t = _grid(nx, ny, m)
    g2 = _periodized_radial_2d(nx, ny, lambda r: np.exp(-(r * r) / (2.0 * sigma * sigma)))
    # exp(kappa cos) scaled by e^-kappa; the scale is removed by normalisation.
    h = np.exp(kappa * (np.cos(t - theta0) - 1.0))
    p = h[:, None, None] * g2[None, :, :]
    if normalize == "discrete":
        return p / p.mean()
    if normalize == "continuous":
        return p / (2.0 * np.pi * sigma * sigma * ive(0, kappa))
    if normalize is None:
        return p * np.exp(kappa)
    raise ValueError(normalize)


def gauss_vm_function(sigma, kappa, theta0=0.0):
    """Continuous-normalised Gaussian x von Mises as a function rho(x, y, theta)."""
    a = 1.0 / (2.0 * np.pi * sigma * sigma * ive(0, kappa))

    def rho(x, y, t):
        return a * np.exp(-(x * x + y * y) / (2.0 * sigma * sigma)) * \
            np.exp(kappa * (np.cos(t - theta0) - 1.0))
    return rho


def se2_log_sq_norm(x, y, t):
    """||log(x, R_t)^v||^2 for the principal matrix logarithm of SE(2), t in [-pi, pi].

    With g = [[R_t, x], [0, 1]], log g = [[t J, v], [0, 0]] where x = V(t) v and
    V(t) = (sin t / t) I + ((1 - cos t) / t) J, a rotation scaled by 2|sin(t/2)|/|t|.
    Hence |v| = |x| (t/2) / sin(t/2) and ||log^v||^2 = ((t/2)/sin(t/2))^2 |x|^2 + t^2.
    """
    h = 0.5 * np.asarray(t, dtype=np.float64)
    safe = np.where(h == 0.0, 1.0, h)
    fac = np.where(h == 0.0, 1.0, safe / np.sin(safe))
    return fac * fac * (x * x + y * y) + (2.0 * h) ** 2


def exp_gauss_function(sigma):
    """Exponential-coordinates Gaussian rho(x, R) = exp(-||log(x, R)^v||^2 / (2 sigma^2))
    (Sec. 6.3, eq. (gbS0)); theta is wrapped to (-pi, pi] for the principal logarithm.
    Radial in translations (it depends on |x| only), not separable."""
    def rho(x, y, t):
        tw = np.where(t > np.pi, t - 2.0 * np.pi, t)
        return np.exp(-se2_log_sq_norm(x, y, tw) / (2.0 * sigma * sigma))
    return rho


def anisotropic_function(sx, sy, kappa, theta0=0.0):
    """Non-radial control kernel exp(-x^2/2sx^2 - y^2/2sy^2) exp(kappa cos(theta-theta0))."""
    def rho(x, y, t):
        return np.exp(-(x * x) / (2 * sx * sx) - (y * y) / (2 * sy * sy)) * \
            np.exp(kappa * (np.cos(t - theta0) - 1.0))
    return rho


def sample_function(rho, nx, ny, m, images=_IMAGES):
    """Periodized samples of an arbitrary kernel function rho(x, y, theta)."""
    x, y, t = _grid(nx, ny, m)
    acc = np.zeros((m, ny, nx))
    for l1 in range(-images, images + 1):
        for l2 in range(-images, images + 1):
            acc += rho((x + l1)[None, None, :], (y + l2)[None, :, None], t[:, None, None])
    return acc


def hat_weights(r, n_knots, r_max):
    """w[q, ...] = max(0, 1 - |r/h - q|), h = r_max/(n_knots-1): piecewise-linear hats."""
    h = r_max / (n_knots - 1)
    q = np.arange(n_knots).reshape((n_knots,) + (1,) * np.ndim(r))
    return np.maximum(0.0, 1.0 - np.abs(np.asarray(r)[None, ...] / h - q))


def radial_profile(nx, ny, m, prof, r_max, images=_IMAGES):
    """P[l, j, i] = sum_images sum_q prof[q, l] * hat_q(|x_ij + image|).

    prof has shape (n_knots, m): knot q at radius q * r_max/(n_knots-1), angular
    sample l at theta_l.  Radial in translations by construction.
    """
    n_knots = prof.shape[0]
    x, y, _ = _grid(nx, ny, 1)
    basis = np.zeros((n_knots, ny, nx))
    for l1 in range(-images, images + 1):
        for l2 in range(-images, images + 1):
            dx = x[None, :] + l1
            dy = y[:, None] + l2
            basis += hat_weights(np.sqrt(dx * dx + dy * dy), n_knots, r_max)
    return np.einsum("ql,qji->lji", prof, basis)


def delta(nx, ny, m):
    """Grid delta at the group identity (x = 0, theta = 0), scaled so rho^[0;L] = 1."""
    p = np.zeros((m, ny, nx))
    p[0, ny // 2, nx // 2] = float(nx * ny * m)
    return p
