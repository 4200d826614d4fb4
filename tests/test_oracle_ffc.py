"""Pins for oracle.ffc: finite Fourier coefficients (paper Sec. 3.2, eqs. (fkLvMain),
(FkLv)) and the finite Fourier series on the grid."""
import numpy as np
import pytest

from oracle.ffc import ffc, ffc_direct, signed_freqs, synthesize, tau


def _trig_poly(nx, ny, m, coeffs):
    """Evaluate sum c_k phi_k on Omega_L from a dict {(k1,k2,k3): c}."""
    x = -0.5 + np.arange(nx) / nx
    y = -0.5 + np.arange(ny) / ny
    t = 2 * np.pi * np.arange(m) / m
    out = np.zeros((m, ny, nx), complex)
    for (k1, k2, k3), c in coeffs.items():
        out += c * np.exp(2j * np.pi * (k1 * x[None, None, :] + k2 * y[None, :, None])) * \
            np.exp(1j * k3 * t[:, None, None])
    return out


@pytest.mark.parametrize("shape", [(5, 7, 9), (4, 6, 8), (8, 8, 8)])
def test_matrix_form_equals_literal_grid_sum(shape, rng):
    # (FkLv) (sign, scale and tau indexing) against the literal sum (fkLvMain).
    f = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    m, ny, nx = shape
    c = ffc(f)
    for k in [(0, 0, 0), (1, -2, 3), (-1, 1, -1), (2, 0, -3), (-(nx // 2), ny // 2 - 1, 1)]:
        idx = (tau(k[2], m), tau(k[1], ny), tau(k[0], nx))
        assert abs(c[idx] - ffc_direct(f, k)) < 1e-13


@pytest.mark.parametrize("shape", [(7, 9, 11), (8, 10, 12)])
def test_trig_polynomial_exactness(shape, rng):
    # Lemma TrigL (Annex): the FFC of a trigonometric polynomial of degree K on
    # L = 2K+1 points is its Fourier coefficient exactly; for even L the same
    # holds for |k| < L/2.
    m, ny, nx = shape
    coeffs = {}
    for _ in range(12):
        k = (int(rng.integers(-((nx - 1) // 2), (nx - 1) // 2 + 1)),
             int(rng.integers(-((ny - 1) // 2), (ny - 1) // 2 + 1)),
             int(rng.integers(-((m - 1) // 2), (m - 1) // 2 + 1)))
        coeffs[k] = complex(rng.standard_normal(), rng.standard_normal())
    f = _trig_poly(nx, ny, m, coeffs)
    c = ffc(f)
    for k, val in coeffs.items():
        idx = (tau(k[2], m), tau(k[1], ny), tau(k[0], nx))
        assert abs(c[idx] - val) < 1e-13
    total = sum(abs(v) ** 2 for v in coeffs.values())
    assert abs(np.sum(np.abs(c) ** 2) - total) < 1e-12 * total


def test_series_reproduces_samples_on_grid(rng):
    # With N = L, S_K[f] evaluated on Omega_L returns the samples (end of Sec. 4.1).
    f = rng.standard_normal((8, 12, 16))
    s = synthesize(ffc(f))
    assert np.max(np.abs(s - f)) < 1e-13


def test_signed_freqs_sets():
    assert list(signed_freqs(5)) == [0, 1, 2, -2, -1]
    assert list(signed_freqs(6)) == [0, 1, 2, -3, -2, -1]


def test_series_on_finer_grid_interpolates_trig_poly(rng):
    # A band-limited trig polynomial: its FFT-series on a finer grid equals the
    # polynomial evaluated there (zero-padded evaluation, Sec. 4.1 / Annex).
    coeffs = {(1, -2, 1): 1.0 + 0.5j, (0, 1, -2): -0.3, (-2, 0, 0): 0.7j}
    f = _trig_poly(7, 7, 7, coeffs)
    fine = synthesize(ffc(f), grid=(11, 13, 9))
    ref = _trig_poly(11, 13, 9, coeffs)
    assert np.max(np.abs(fine - ref)) < 1e-13
