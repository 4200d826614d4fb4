"""Pins for the evaluation of S_K on a grid finer than the sampling grid (Sec. 4.1
eq. (MatSKfonG), Sec. 6.1 eq. (MatSKfgonG), Prop. LtoN1D).

Two oracle routes: explicit synthesis sum_k H[k] phi_k(w') at the finer points, and
the paper's zero-padded matrix form (N_prod / n^2) iDFT_N(W . Q_f . Q_rho).  They are
checked against each other, against the continuous closed form at the finer points,
against trigonometric polynomials, and against the Nyquist reading for even L.
"""
import numpy as np
import pytest

from inputs import bump_field, rel_l2, sample_field
from inputs.fields import KernelParams
from oracle import closed_form as CF
from oracle import conv as C
from oracle import ffc as FF
from oracle import kernels as K

_CHAIN = [KernelParams(0.04, 5.0, 0.4), KernelParams(0.03, 2.0, 1.1), KernelParams(0.05, 3.0, 0.2)]


def _setup(shape, nk):
    bf = bump_field(93, 0, 6, s=0.05, kappa=3.0)
    f = sample_field(bf, *shape)
    ps = [K.gauss_vm(*shape, k.sigma, k.kappa, k.theta0, normalize="continuous") for k in _CHAIN[:nk]]
    return bf, f, ps


@pytest.mark.parametrize("shape,grid,nk", [
    ((25, 27, 23), (40, 41, 30), 1),   # odd L (the paper's case)
    ((24, 26, 20), (48, 39, 20), 2),   # even L, Nyquist split on x and y
    ((33, 33, 33), (33, 33, 33), 1),   # N = L
    ((32, 32, 16), (33, 40, 17), 3),   # even L, odd N
])
def test_synthesis_equals_papers_zero_padded_matrix_form(shape, grid, nk):
    _, f, ps = _setup(shape, nk)
    a = C.conv_on_grid(f, ps, grid)
    b = C.padded_matrix_form(f, ps, grid)
    assert rel_l2(a, b) < 1e-14


def test_n_equal_l_is_the_on_grid_series():
    _, f, ps = _setup((24, 26, 20), 2)
    assert np.max(np.abs(C.conv_on_grid(f, ps, (24, 26, 20)) - C.conv_chain(f, ps))) < 1e-15


@pytest.mark.parametrize("shape,grid,bar", [
    ((41, 43, 45), (64, 64, 64), 1e-9),
    ((40, 42, 44), (80, 84, 88), 1e-9),
])
def test_finer_grid_matches_continuous_closed_form(shape, grid, bar):
    # the finer-grid values are the trigonometric interpolant of the convolution:
    # spectrally close to the continuous result at points the sampling grid lacks
    bf, f, ps = _setup(shape, 2)
    out = C.conv_on_grid(f, ps, grid)
    assert rel_l2(out, CF.conv_closed_form(bf, _CHAIN[:2], *grid)) < bar


def test_nyquist_cosine_is_reproduced_off_grid():
    # Reading for even L: the index L/2 carries both frequencies +-L/2.  A real
    # cosine at the Nyquist frequency must come back as that cosine, real, at the
    # finer points (the unsplit choice phi_{-L/2} alone would give a complex wave).
    nx, ny, m = 8, 6, 4
    gx, gy, gm = 20, 15, 12
    x = -0.5 + np.arange(nx) / nx
    t = 2 * np.pi * np.arange(m) / m
    f = np.cos(np.pi * nx * x)[None, None, :] * np.cos(2 * t)[:, None, None] * np.ones((1, ny, 1))
    s = FF.synthesize(FF.ffc(f), grid=(gx, gy, gm))
    xg = -0.5 + np.arange(gx) / gx
    tg = 2 * np.pi * np.arange(gm) / gm
    ref = np.cos(np.pi * nx * xg)[None, None, :] * np.cos(2 * tg)[:, None, None] * np.ones((1, gy, 1))
    assert np.max(np.abs(s - ref)) < 1e-13


def test_trig_polynomial_on_finer_grid_even_l(rng):
    # band-limited (|k| < L/2): the series equals the polynomial everywhere
    nx, ny, m = 10, 8, 6
    coeffs = {(2, -3, 1): 1.0 + 0.5j, (-4, 1, -2): -0.3, (0, 3, 2): 0.7j, (1, 0, 0): 0.2}
    grid = (17, 16, 11)

    def poly(gx, gy, gm):
        x = -0.5 + np.arange(gx) / gx
        y = -0.5 + np.arange(gy) / gy
        t = 2 * np.pi * np.arange(gm) / gm
        out = np.zeros((gm, gy, gx), complex)
        for (k1, k2, k3), c in coeffs.items():
            out += c * np.exp(2j * np.pi * (k1 * x[None, None, :] + k2 * y[None, :, None])) * \
                np.exp(1j * k3 * t[:, None, None])
        return out
    s = FF.synthesize(FF.ffc(poly(nx, ny, m)), grid=grid)
    assert np.max(np.abs(s - poly(*grid))) < 1e-13


def test_unsplit_nyquist_is_caught(monkeypatch):
    # planted mistake: phi_{-L/2} alone at the Nyquist index
    orig = FF._phi_axis

    def unsplit(length, points, grid, spatial):
        k = FF.signed_freqs(length)
        a = np.asarray(points, dtype=np.int64)
        e = np.exp(2j * np.pi * np.mod(np.outer(a, k), grid).astype(float) / grid)
        if spatial:
            e = e * np.where(k % 2 == 0, 1.0, -1.0)[None, :]
        return e
    assert orig is not unsplit
    monkeypatch.setattr(FF, "_phi_axis", unsplit)
    nx, ny, m = 8, 6, 4
    x = -0.5 + np.arange(nx) / nx
    f = np.cos(np.pi * nx * x)[None, None, :] * np.ones((m, ny, 1))
    s = FF.synthesize(FF.ffc(f), grid=(20, 6, 4))
    ref = np.cos(np.pi * nx * (-0.5 + np.arange(20) / 20))[None, None, :] * np.ones((4, 6, 1))
    assert np.max(np.abs(s - ref)) > 0.1
