"""Pins for the oracle routines that build reference tables and evaluate the series at a
subset of points: coeff_product, conv_with_coeffs (whole grid and points=), and
synthesize(points=).  Each is checked against something other than itself (direct
quadrature with explicit rotation, the literal grid sums of eqs. (fkLvMain) and (SKfg)
written as loops), and a planted mistake in each must fail its pin.
"""
import numpy as np
import pytest

import oracle.conv as C
import oracle.ffc as FF
import oracle.transforms as T
from inputs import bump_field, rel_l2, sample_field
from oracle import kernels as K
from oracle import quadrature as Q


def _field(nx, ny, m, seed=0):
    return sample_field(bump_field(93, seed, 4, s=0.08, kappa=2.0), nx, ny, m)


RHOS = [(0.09, 1.5, 0.2), (0.13, 3.0, 2.0), (0.07, 6.0, 4.1)]


def _coeff_product_pin(nx=8, ny=12, m=8):
    """Error of conv_with_coeffs(f, coeff_product(ps)) against the direct quadrature of
    the chain, applied one kernel at a time with the explicit rotation (eqs. (f*g),
    (oslash)); nothing on the quadrature side multiplies coefficients."""
    f = _field(nx, ny, m, seed=1)
    rhos = [K.gauss_vm_function(*r) for r in RHOS]
    ps = [K.sample_function(r, nx, ny, m) for r in rhos]
    a = C.conv_with_coeffs(f, C.coeff_product(ps))
    return rel_l2(a, Q.quadrature_chain(f, rhos))


def test_coeff_product_chain_equals_direct_quadrature_chain():
    assert _coeff_product_pin() < 1e-13


def _literal_ffc_all(samples):
    """Every FFC by the literal grid sum of eq. (fkLvMain), at its signed frequency."""
    m, ny, nx = samples.shape
    out = np.zeros((m, ny, nx), complex)
    k1, k2, k3 = FF.signed_freqs(nx), FF.signed_freqs(ny), FF.signed_freqs(m)
    for c in range(m):
        for b in range(ny):
            for a in range(nx):
                out[c, b, a] = FF.ffc_direct(samples, (int(k1[a]), int(k2[b]), int(k3[c])))
    return out


def test_coeff_product_equals_ffc_of_quadrature_composed_kernels():
    # Thm. f*gP on the grid: the FFC of p1 (/) rho2 (direct quadrature, explicit rotation)
    # is the product of the two kernels' FFCs; the FFCs here are literal grid sums.
    nx, ny, m = 6, 8, 4
    r1, r2 = (K.gauss_vm_function(*r) for r in RHOS[:2])
    p1 = K.sample_function(r1, nx, ny, m)
    p2 = K.sample_function(r2, nx, ny, m)
    composed = Q.quadrature_conv(p1, r2)
    lit = _literal_ffc_all(composed)
    tab = C.coeff_product([p1, p2])
    assert np.max(np.abs(tab - lit)) <= 1e-13 * np.max(np.abs(lit))


def test_coeff_product_dropped_factor_is_caught(monkeypatch):
    orig = C.coeff_product

    def dropped_last(kernels):
        return orig(list(kernels)[:-1])
    monkeypatch.setattr(C, "coeff_product", dropped_last)
    assert _coeff_product_pin() > 1e-3


def test_coeff_product_unscaled_factor_is_caught(monkeypatch):
    # a table built from raw DFTs (missing 1/n and W) instead of FFCs
    def raw(kernels):
        t = None
        for p in kernels:
            c = T.dft3(p)
            t = c if t is None else t * c
        return t
    monkeypatch.setattr(C, "coeff_product", raw)
    assert _coeff_product_pin() > 1e-3


# ------------------------------------------------------------ points= evaluation
def _literal_series(coeffs, grid, pts):
    """S(w) = sum_k c[k] phi_k(w) (eq. (SKfg)) by explicit loops over k, at the
    tensor-product points pts = (ax, ay, at) of a G-grid; odd coefficient grids only
    (no Nyquist index).  phi_k = exp(2 pi i (k1 x + k2 y)) exp(i k3 theta) (eq. (phik)),
    x = -1/2 + a/Gx, theta = 2 pi a / Gm (eq. (OmL))."""
    m, ny, nx = coeffs.shape
    gx, gy, gm = grid
    ax, ay, at = pts
    k1, k2, k3 = FF.signed_freqs(nx), FF.signed_freqs(ny), FF.signed_freqs(m)
    out = np.zeros((len(at), len(ay), len(ax)), complex)
    for ic, c in enumerate(at):
        th = 2 * np.pi * c / gm
        for ib, b in enumerate(ay):
            y = -0.5 + b / gy
            for ia, a in enumerate(ax):
                x = -0.5 + a / gx
                ph = np.exp(2j * np.pi * (k1[None, None, :] * x + k2[None, :, None] * y)) * \
                    np.exp(1j * k3[:, None, None] * th)
                out[ic, ib, ia] = np.sum(coeffs * ph)
    return out


PTS_CASES = [
    # coefficient grid (nx, ny, m), evaluation grid, ragged point lists
    ((9, 7, 5), (9, 7, 5), ([0, 2, 5], [1, 4, 6], [0, 3])),
    ((9, 7, 5), (15, 11, 10), ([1, 8, 14], [0, 5, 10, 3], [9, 2, 4])),
]


@pytest.mark.parametrize("shape,grid,pts", PTS_CASES)
def test_synthesize_points_equals_literal_sum(shape, grid, pts, rng):
    nx, ny, m = shape
    c = rng.standard_normal((m, ny, nx)) + 1j * rng.standard_normal((m, ny, nx))
    got = FF.synthesize(c, grid=grid, points=pts)
    ref = _literal_series(c, grid, pts)
    assert np.max(np.abs(got - ref)) <= 1e-12 * np.max(np.abs(ref))


@pytest.mark.parametrize("shape,grid", [((9, 7, 5), (15, 11, 10)), ((8, 12, 6), (8, 12, 6)),
                                        ((8, 12, 6), (16, 20, 9))])
def test_synthesize_points_equals_sliced_full_synthesis(shape, grid, rng):
    # even coefficient grids included: the Nyquist split must act point by point
    nx, ny, m = shape
    c = rng.standard_normal((m, ny, nx)) + 1j * rng.standard_normal((m, ny, nx))
    full = FF.synthesize(c, grid=grid)
    gx, gy, gm = grid
    ax = np.array([gx - 1, 0, gx // 2, 3])
    ay = np.array([1, gy - 2, 5])
    at = np.array([gm - 1, 2])
    got = FF.synthesize(c, grid=grid, points=(ax, ay, at))
    assert np.max(np.abs(got - full[np.ix_(at, ay, ax)])) <= 1e-13 * np.max(np.abs(full))


def test_synthesize_swapped_point_axes_is_caught(monkeypatch, rng):
    shape, grid, pts = PTS_CASES[0]
    nx, ny, m = shape
    c = rng.standard_normal((m, ny, nx)) + 1j * rng.standard_normal((m, ny, nx))
    ref = _literal_series(c, grid, pts)
    orig = FF.synthesize

    def swapped(coeffs, grid=None, points=None):
        ax, ay, at = points
        return orig(coeffs, grid=grid, points=(ay, ax, at))
    monkeypatch.setattr(FF, "synthesize", swapped)
    got = FF.synthesize(c, grid=grid, points=pts)
    assert np.max(np.abs(got - ref)) > 1e-3 * np.max(np.abs(ref))


def test_conv_with_coeffs_points_equals_quadrature_at_points():
    # the subsampled scoring of the large grid: the series at every 2nd x, y and 2nd
    # theta against the direct quadrature (route 2) at the same points
    nx, ny, m = 8, 12, 8
    f = _field(nx, ny, m, seed=2)
    rhos = [K.gauss_vm_function(*r) for r in RHOS[:2]]
    ps = [K.sample_function(r, nx, ny, m) for r in rhos]
    pts = (np.arange(0, nx, 2), np.arange(1, ny, 2), np.arange(0, m, 2))
    sub = C.conv_with_coeffs(f, C.coeff_product(ps), points=pts)
    quad = Q.quadrature_chain(f, rhos)
    ref = quad[np.ix_(pts[2], pts[1], pts[0])]
    assert rel_l2(sub, ref) < 1e-13
    # and the whole grid
    assert rel_l2(C.conv_with_coeffs(f, C.coeff_product(ps)), quad) < 1e-13


# ------------------------------------- the FFT evaluation at the workloads' axis lengths
@pytest.mark.parametrize("length", [64, 128, 256, 512])
@pytest.mark.parametrize("sign", [-1, +1])
def test_fft_route_equals_dense_route_at_workload_lengths(length, sign, rng, monkeypatch):
    """The oracle switches to numpy's FFT for large arrays (the 256^2 x 64 and 512^2 x 128
    references).  At exactly those axis lengths, along every axis position, the FFT
    evaluation must equal the dense matrix evaluation of the same sum (eq. (3DFT))."""
    shapes = [(3, 5, length), (3, length, 4), (length, 2, 5)]
    for ax, shp in zip((2, 1, 0), shapes):
        a = rng.standard_normal(shp) + 1j * rng.standard_normal(shp)
        monkeypatch.setattr(T, "DENSE_LIMIT", 1 << 62)
        dense = T._dft_axis(a, ax, sign)
        monkeypatch.setattr(T, "DENSE_LIMIT", 0)
        fast = T._dft_axis(a, ax, sign)
        assert np.max(np.abs(dense - fast)) <= 1e-12 * np.max(np.abs(dense))


def test_axis_routes_report():
    # the routes the oracle's forward DFT takes for one headline field
    assert T.axis_routes((64, 256, 256)) == {"x": "fft", "y": "fft", "theta": "dense"}
    assert T.axis_routes((128, 512, 512)) == {"x": "fft", "y": "fft", "theta": "fft"}
    assert T.axis_routes((32, 32, 32)) == {"x": "dense", "y": "dense", "theta": "dense"}
