"""Pins for oracle.shifted: convolution with sums of SE(2)-shifted radial kernels
(Sec. 1 outlook, with the product of coefficients of Thm. f*gP applied after moving each
shift onto the field).  Pinned by the direct quadrature of route 2, which takes the
shifted kernel sum as an arbitrary (non-radial) function with the explicit rotation."""
import numpy as np
import pytest

import oracle.shifted as S
from inputs import bump_field, rel_l2, sample_field
from oracle import conv as C
from oracle import kernels as K
from oracle import quadrature as Q


def _field(nx, ny, m, seed=0):
    return sample_field(bump_field(94, seed, 4, s=0.08, kappa=2.0), nx, ny, m)


RHO = (0.08, 2.0, 0.3)


def _exact_case(n=12, m=4):
    # square grid, M = 4: every R_alpha t of a grid vector t is a grid vector, and the
    # angles phi are grid angles, so every shift is an exact index roll
    shifts = [(2 / n, -3 / n, 0.0), (-1 / n, 5 / n, np.pi / 2), (4 / n, 1 / n, np.pi), (0.0, 0.0, 3 * np.pi / 2)]
    weights = [0.7, -0.4, 1.3, 0.25]
    return n, m, shifts, weights


def _pin_error(fn=None):
    n, m, shifts, weights = _exact_case()
    f = _field(n, n, m, seed=1)
    rho = K.gauss_vm_function(*RHO)
    p = K.sample_function(rho, n, n, m)
    fn = fn or S.shifted_sum_conv
    a = fn(f, p, shifts, weights)
    b = Q.quadrature_conv(f, S.shifted_kernel_function(rho, shifts, weights))
    return rel_l2(a, b)


def test_exact_grid_shifts_equal_direct_quadrature():
    assert _pin_error() < 1e-13


@pytest.mark.parametrize("m", [2, 4])
def test_exact_grid_shifts_rectangular_grid(m):
    # M = 2 (alpha in {0, pi}) keeps any grid vector on the grid, also for Nx != Ny
    nx, ny = 10, 8
    if m == 4:
        nx = ny = 8
    shifts = [(3 / nx, -2 / ny, 0.0), (-1 / nx, 1 / ny, np.pi)]
    weights = [1.0, 0.5]
    f = _field(nx, ny, m, seed=2)
    rho = K.gauss_vm_function(0.1, 1.5, 0.0)
    p = K.sample_function(rho, nx, ny, m)
    a = S.shifted_sum_conv(f, p, shifts, weights)
    b = Q.quadrature_conv(f, S.shifted_kernel_function(rho, shifts, weights))
    assert rel_l2(a, b) < 1e-13


def test_off_grid_shifts_converge_to_direct_quadrature():
    # general translations and angles: the series shifts the trigonometric interpolant,
    # the quadrature samples the shifted kernel; both converge as the grid is refined
    shifts = [(0.137, -0.052, 0.61), (-0.211, 0.093, 2.2)]
    weights = [1.0, -0.6]
    rho = K.gauss_vm_function(0.09, 1.5, 0.0)
    errs = []
    for n in (12, 16, 24):
        f = sample_field(bump_field(94, 5, 3, s=0.1, kappa=1.0), n, n, n)
        p = K.sample_function(rho, n, n, n)
        a = S.shifted_sum_conv(f, p, shifts, weights)
        b = Q.quadrature_conv(f, S.shifted_kernel_function(rho, shifts, weights))
        errs.append(rel_l2(a, b))
    assert errs[0] > errs[1] > errs[2] and errs[2] < 1e-5, errs


def test_shifted_sum_is_not_the_plain_series_of_its_samples():
    # the shifted sum is not radial: the plain product of coefficients of its samples
    # (what a radial kernel would allow) misses the SE(2) convolution
    n, m, shifts, weights = _exact_case()
    f = _field(n, n, m, seed=3)
    rho = K.gauss_vm_function(*RHO)
    kern = S.shifted_kernel_function(rho, shifts, weights)
    plain = C.conv_chain(f, [K.sample_function(kern, n, n, m)])
    quad = Q.quadrature_conv(f, kern)
    assert rel_l2(plain, quad) > 1e-2
    assert rel_l2(S.shifted_sum_conv(f, K.sample_function(rho, n, n, m), shifts, weights), quad) < 1e-13


def test_zero_shift_is_the_plain_convolution():
    f = _field(8, 12, 6, seed=4)
    p = K.gauss_vm(8, 12, 6, 0.07, 3.0, 0.5)
    a = S.shifted_sum_conv(f, p, [(0.0, 0.0, 0.0), (0.0, 0.0, 0.0)], [0.25, 0.75])
    assert rel_l2(a, C.conv_chain(f, [p])) < 1e-14


def test_theta_grid_shift_is_an_index_roll():
    f = _field(8, 8, 6, seed=5)
    p = K.gauss_vm(8, 8, 6, 0.07, 3.0, 0.5)
    a = S.shifted_sum_conv(f, p, [(0.0, 0.0, 2 * 2 * np.pi / 6)], [1.0])
    assert rel_l2(a, np.roll(C.conv_chain(f, [p]), 2, axis=0)) < 1e-14


def test_real_field_gives_real_result_on_even_grids():
    f = _field(8, 10, 6, seed=6)
    p = K.gauss_vm(8, 10, 6, 0.07, 3.0, 0.5)
    z = S.shifted_sum_conv(f, p, [(0.173, -0.31, 0.9)], [1.0], return_complex=True)
    assert np.max(np.abs(z.imag)) < 1e-14 * np.max(np.abs(z.real))


def test_planted_rotation_sign_is_caught(monkeypatch):
    # R_{-alpha} t instead of R_alpha t in the translation phase
    monkeypatch.setattr(S, "slice_translation",
                        lambda a, tx, ty: (np.cos(a) * tx + np.sin(a) * ty, -np.sin(a) * tx + np.cos(a) * ty))
    assert _pin_error() > 1e-3


def test_planted_unrotated_slices_are_caught(monkeypatch):
    # every slice translated by t itself (R_alpha forgotten)
    monkeypatch.setattr(S, "slice_translation", lambda a, tx, ty: (np.full_like(a, tx), np.full_like(a, ty)))
    assert _pin_error() > 1e-3


def test_planted_unrotated_translation_is_caught(monkeypatch):
    # translating every slice by t itself (forgetting R_alpha) is the wrong operator
    def unrotated(f, p, shifts, weights, return_complex=False):
        m = f.shape[0]
        out = 0.0
        for (tx, ty, phi), a in zip(shifts, weights):
            # translate by t without rotation: one term per shift, all slices alike
            fk = np.roll(np.roll(f, int(round(ty * f.shape[1])), axis=1), int(round(tx * f.shape[2])), axis=2)
            fk = np.roll(fk, int(round(phi / (2 * np.pi / m))), axis=0)
            out = out + a * C.conv_chain(fk, [p])
        return out
    assert _pin_error(unrotated) > 1e-3
