"""Pins for oracle.transforms: the 3-D DFT of paper Sec. 2.3, eqs. (3DFT), (3iDFT)."""
import numpy as np
import pytest

from oracle import transforms as T
from oracle.transforms import dft1, dft3, dft_matrix, idft3


@pytest.mark.parametrize("shape", [(4, 8, 8), (8, 6, 10), (16, 48, 12), (3, 5, 7)])
def test_dft3_matches_library_fft(shape, rng):
    # Special case reducing to a library routine: numpy's FFT uses the same
    # un-normalised forward convention as (3DFT).
    a = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    ours = dft3(a)
    ref = np.fft.fftn(a)
    assert np.max(np.abs(ours - ref)) <= 1e-12 * np.max(np.abs(ref))
    inv = idft3(a)
    ref_inv = np.fft.ifftn(a)
    assert np.max(np.abs(inv - ref_inv)) <= 1e-12 * np.max(np.abs(ref_inv))


def test_dft_matrix_entries_by_definition():
    # D[k, i] = exp(-2 pi i k i / L) written out for L = 6, entry by entry.
    d = dft_matrix(6)
    for k in range(6):
        for i in range(6):
            assert abs(d[k, i] - np.exp(-2j * np.pi * k * i / 6)) < 1e-14


def test_round_trip_and_parseval(rng):
    a = rng.standard_normal((8, 12, 16))
    fa = dft3(a)
    assert np.max(np.abs(idft3(fa) - a)) < 1e-13
    n = a.size
    assert abs(np.sum(np.abs(a) ** 2) - np.sum(np.abs(fa) ** 2) / n) < 1e-10 * np.sum(a * a)


def test_dft1_of_pure_tone():
    # A single complex exponential of frequency 3 transforms to L at index 3.
    L = 16
    v = np.exp(2j * np.pi * 3 * np.arange(L) / L)
    fv = dft1(v)
    expect = np.zeros(L, complex)
    expect[3] = L
    assert np.max(np.abs(fv - expect)) < 1e-12


@pytest.mark.parametrize("sign", [-1, +1])
def test_large_array_route_equals_dense_route(sign, rng, monkeypatch):
    """Above DENSE_LIMIT the per-axis sum is taken by numpy's FFT: it must equal the dense
    matrix evaluation of the same definition (forced here on a small ragged array)."""
    a = rng.standard_normal((6, 10, 12)) + 1j * rng.standard_normal((6, 10, 12))
    dense = [T._dft_axis(a, ax, sign) for ax in range(3)]
    monkeypatch.setattr(T, "DENSE_LIMIT", 0)
    fast = [T._dft_axis(a, ax, sign) for ax in range(3)]
    for d, f in zip(dense, fast):
        assert np.max(np.abs(d - f)) <= 1e-12 * np.max(np.abs(d))
    assert np.allclose(T.idft3(T.dft3(a)), a, atol=1e-13)
