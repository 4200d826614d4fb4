"""Seeded synthetic fields on Z^2\\SE(2).

Test fields are sums of Gaussian x von Mises bumps, periodized over the lattice
Z^2 (paper Sec. 2.2, eq. (TH)):

    f(x, theta) = sum_b w_b * sum_{l in Z^2} exp(-|x - c_b + l|^2 / (2 s^2))
                            * exp(kappa_f * cos(theta - theta0_b))

sampled on the grid Omega_L of paper Sec. 3.2, eq. (OmL):
x_i = -1/2 + i/N, y_j = -1/2 + j/N, theta_l = 2*pi*l/M (0-based indices).
Arrays are stored [theta][y][x] with x fastest, which is the memory order of the
paper's F(i, j, l) with i fastest.

Random draws use numpy's PCG64 seeded with [2504_05149, config, stream]; the
draw order is centres, orientations, weights (fields) and sigma, kappa (kernels).
Nothing here computes a transform or a convolution.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

SEED_ROOT = 2504_05149

# Lattice images used when periodizing a bump.  A bump of width s <= 0.1 centred
# in [0,1) has |x - c + l| >= 1 for |l| >= 2 on the grid, i.e. weight < e^-50.
_IMAGES = 3


@dataclasses.dataclass(frozen=True)
class BumpField:
    centres: np.ndarray  # (B, 2) in [0,1)^2, columns (x, y)
    theta0: np.ndarray  # (B,) in [0, 2*pi)
    weights: np.ndarray  # (B,) in [0.5, 1]
    s: float  # translational width
    kappa: float  # von Mises concentration


@dataclasses.dataclass(frozen=True)
class KernelParams:
    sigma: float
    kappa: float
    theta0: float = 0.0


def grid_axes(nx: int, ny: int, m: int):
    """Coordinates of Omega_L (eq. (OmL)), 0-based: x_i = -1/2 + i/nx, theta_l = 2 pi l / m."""
    x = -0.5 + np.arange(nx, dtype=np.float64) / nx
    y = -0.5 + np.arange(ny, dtype=np.float64) / ny
    t = 2.0 * np.pi * np.arange(m, dtype=np.float64) / m
    return x, y, t


def bump_field(config: int, field: int, n_bumps: int, s: float = 0.04,
               kappa: float = 4.0) -> BumpField:
    rng = np.random.default_rng([SEED_ROOT, config, field])
    centres = rng.uniform(0.0, 1.0, size=(n_bumps, 2))
    theta0 = rng.uniform(0.0, 2.0 * np.pi, size=n_bumps)
    weights = rng.uniform(0.5, 1.0, size=n_bumps)
    return BumpField(centres, theta0, weights, float(s), float(kappa))


def chain_kernel_params(config: int, n_kernels: int, sigma_range=(0.01, 0.1),
                        kappa_range=(1.0, 20.0)) -> list[KernelParams]:
    out = []
    for j in range(n_kernels):
        rng = np.random.default_rng([SEED_ROOT, config, 1000 + j])
        sigma = rng.uniform(*sigma_range)
        kappa = rng.uniform(*kappa_range)
        out.append(KernelParams(float(sigma), float(kappa), 0.0))
    return out


def _periodized_gauss_1d(coord: np.ndarray, centre: float, s: float) -> np.ndarray:
    acc = np.zeros_like(coord)
    for l in range(-_IMAGES, _IMAGES + 1):
        d = coord - centre + l
        acc += np.exp(-(d * d) / (2.0 * s * s))
    return acc


def sample_field(bf: BumpField, nx: int, ny: int, m: int,
                 dtype=np.float64) -> np.ndarray:
    """Samples F[theta][y][x] of the periodized bump field on Omega_L."""
    x, y, t = grid_axes(nx, ny, m)
    nb = len(bf.weights)
    gx = np.empty((nb, nx))
    gy = np.empty((nb, ny))
    ht = np.empty((nb, m))
    for b in range(nb):
        gx[b] = _periodized_gauss_1d(x, bf.centres[b, 0], bf.s)
        gy[b] = _periodized_gauss_1d(y, bf.centres[b, 1], bf.s)
        ht[b] = bf.weights[b] * np.exp(bf.kappa * np.cos(t - bf.theta0[b]))
    # Each bump is an outer product of three 1-D profiles; sum them.
    f = np.einsum("bt,by,bx->tyx", ht, gy, gx, optimize=True)
    return np.ascontiguousarray(f.astype(dtype, copy=False))


def sample_fields(config: int, batch: int, n_bumps: int, nx: int, ny: int, m: int,
                  dtype=np.float64, first_field: int = 0, s: float = 0.04,
                  kappa: float = 4.0) -> np.ndarray:
    """[batch][m][ny][nx] samples of fields first_field .. first_field+batch-1."""
    out = np.empty((batch, m, ny, nx), dtype=dtype)
    for b in range(batch):
        bf = bump_field(config, first_field + b, n_bumps, s, kappa)
        out[b] = sample_field(bf, nx, ny, m, dtype)
    return out


def uneven_problem_list(config: int, n_problems: int,
                        sizes_n=(32, 48, 64, 96, 128), sizes_m=(16, 32, 64),
                        chain_max: int = 4, n_bumps: int = 8):
    """Problem descriptions for a heterogeneous batch.

    Each entry: dict(n=N, m=M, chain=[KernelParams...], field=BumpField).
    """
    rng = np.random.default_rng([SEED_ROOT, config, 7777])
    probs = []
    for p in range(n_problems):
        n = int(rng.choice(sizes_n))
        m = int(rng.choice(sizes_m))
        lc = int(rng.integers(1, chain_max + 1))
        chain = []
        for j in range(lc):
            sigma = float(rng.uniform(0.01, 0.1))
            kappa = float(rng.uniform(1.0, 20.0))
            chain.append(KernelParams(sigma, kappa, 0.0))
        bf = bump_field(config, p, n_bumps)
        probs.append(dict(n=n, m=m, chain=chain, field=bf))
    return probs


def rel_l2(a: np.ndarray, b: np.ndarray) -> float:
    """||a - b||_2 / ||b||_2 (real or complex arrays)."""
    dt = np.complex128 if (np.iscomplexobj(a) or np.iscomplexobj(b)) else np.float64
    a = np.asarray(a, dtype=dt)
    b = np.asarray(b, dtype=dt)
    den = math.sqrt(float(np.sum(np.abs(b) ** 2)))
    return math.sqrt(float(np.sum(np.abs(a - b) ** 2))) / (den if den > 0 else 1.0)
