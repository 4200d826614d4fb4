"""Pins for oracle.adjoint: gradients against brute force and finite differences."""
import numpy as np
import pytest

from oracle import adjoint as A
from oracle import conv as C
from oracle import kernels as K


def test_kernel_gradient_matches_explicit_loop_form(rng):
    f = rng.standard_normal((4, 6, 8))
    g = rng.standard_normal((4, 6, 8))
    assert np.max(np.abs(A.grad_kernel_samples(f, g) - A.grad_kernel_direct(f, g))) < 1e-13


@pytest.mark.parametrize("shape", [(4, 8, 8), (5, 7, 9)])  # even grid, odd grid (L = 2K+1)
def test_kernel_gradient_by_finite_differences(rng, shape):
    f = rng.standard_normal(shape)
    p = rng.standard_normal(shape)
    target = rng.standard_normal(shape)

    def loss(pp):
        r = C.conv_chain(f, [pp]) - target
        return float(np.sum(r * r))
    g = 2.0 * (C.conv_chain(f, [p]) - target)
    grad = A.grad_kernel_samples(f, g)
    h = 1e-3
    for idx in [(0, 0, 0), (1, 3, 5), (3, 6, 2), (2, 4, 4)]:
        e = np.zeros_like(p)
        e[idx] = h
        fd = (loss(p + e) - loss(p - e)) / (2 * h)
        # the loss is quadratic in p, so central differences are exact up to rounding
        assert abs(fd - grad[idx]) < 1e-8 * max(1.0, abs(fd))


@pytest.mark.parametrize("shape", [(4, 8, 8), (5, 7, 9)])
def test_field_gradient_by_finite_differences(rng, shape):
    m, ny, nx = shape
    f = rng.standard_normal(shape)
    p = K.gauss_vm(nx, ny, m, 0.1, 2.0, 0.5)
    target = rng.standard_normal(shape)

    def loss(ff):
        r = C.conv_chain(ff, [p]) - target
        return float(np.sum(r * r))
    grad = A.grad_field(2.0 * (C.conv_chain(f, [p]) - target), [p])
    h = 1e-3
    for idx in [(0, 1, 2), (3, 6, 6), (2, 0, 5)]:
        e = np.zeros_like(f)
        e[idx] = h
        fd = (loss(f + e) - loss(f - e)) / (2 * h)
        assert abs(fd - grad[idx]) < 1e-8 * max(1.0, abs(fd))


def test_profile_gradient_by_finite_differences(rng):
    nx = ny = 8
    m, nk, rmax = 4, 5, 0.45
    prof = rng.uniform(0, 1, (nk, m))
    f = rng.standard_normal((m, ny, nx))
    target = rng.standard_normal((m, ny, nx))

    def loss(pr):
        r = C.conv_chain(f, [K.radial_profile(nx, ny, m, pr, rmax)]) - target
        return float(np.sum(r * r))
    g = 2.0 * (C.conv_chain(f, [K.radial_profile(nx, ny, m, prof, rmax)]) - target)
    grad = A.grad_profile(A.grad_kernel_samples(f, g), nk, rmax)
    h = 1e-3
    for q, l in [(0, 0), (2, 3), (4, 1), (1, 2)]:
        e = np.zeros_like(prof)
        e[q, l] = h
        fd = (loss(prof + e) - loss(prof - e)) / (2 * h)
        assert abs(fd - grad[q, l]) < 1e-8 * max(1.0, abs(fd))


def test_profile_basis_reproduces_sampler(rng):
    prof = rng.uniform(0, 1, (7, 6))
    p = K.radial_profile(12, 10, 6, prof, 0.5)
    basis = A.profile_basis(12, 10, 7, 0.5)
    assert np.max(np.abs(np.einsum("ql,qji->lji", prof, basis) - p)) < 1e-14
