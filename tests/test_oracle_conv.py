"""Pins for oracle.conv (route 1) against things the paper and mathematics fix:
direct quadrature with explicit rotation (route 2), closed forms, invariants,
textbook reductions, and the paper's Algorithms 3, 4, 6 and 7."""
import numpy as np
import pytest

from inputs import bump_field, rel_l2, sample_field
from inputs.fields import KernelParams
from oracle import closed_form as CF
from oracle import conv as C
from oracle import kernels as K
from oracle import quadrature as Q
from oracle.ffc import ffc


def _field(nx, ny, m, nb=4, s=0.08, kappa=2.0, seed=0):
    return sample_field(bump_field(90, seed, nb, s=s, kappa=kappa), nx, ny, m)


@pytest.mark.parametrize("shape", [(8, 8, 8), (8, 12, 16), (12, 8, 8)])
def test_route1_equals_direct_quadrature_radial(shape):
    # For radial kernels the FFT route equals the rectangle rule of the coset
    # convolution with explicit R_{-alpha} and lattice images (Thm. f*gP, eq. (oslash)).
    m, ny, nx = shape
    f = _field(nx, ny, m)
    rho = K.gauss_vm_function(0.11, 2.5, 0.7)
    p = K.sample_function(rho, nx, ny, m)
    a = C.conv_chain(f, [p])
    b = Q.quadrature_conv(f, rho)
    assert rel_l2(a, b) < 1e-13


def test_complex_field_route1_equals_quadrature_of_parts():
    # f: SE(2) -> C (Sec. 3.2): route 1 on the complex field against the direct
    # quadrature applied to its real and imaginary parts (the kernel is real)
    a = _field(8, 12, 8, seed=6)
    b = _field(8, 12, 8, seed=7)
    rho = K.gauss_vm_function(0.1, 2.0, 0.4)
    p = K.sample_function(rho, 8, 12, 8)
    out = C.conv_chain(a + 1j * b, [p], return_complex=True)
    ref = Q.quadrature_conv(a, rho) + 1j * Q.quadrature_conv(b, rho)
    assert rel_l2(out, ref) < 1e-13


def test_route1_equals_direct_quadrature_chain():
    f = _field(8, 8, 8, seed=1)
    rhos = [K.gauss_vm_function(0.09, 1.5, 0.2), K.gauss_vm_function(0.13, 3.0, 2.0)]
    ps = [K.sample_function(r, 8, 8, 8) for r in rhos]
    assert rel_l2(C.conv_chain(f, ps), Q.quadrature_chain(f, rhos)) < 1e-13


def test_radial_profile_kernel_route1_equals_quadrature(rng):
    # A kernel radial in translations with a free angular dependence.
    nk, rmax = 6, 0.45
    prof = rng.uniform(0.0, 1.0, size=(nk, 8))
    p = K.radial_profile(8, 8, 8, prof, rmax)
    h = rmax / (nk - 1)
    t = 2 * np.pi * np.arange(8) / 8

    def rho(x, y, th):
        r = np.sqrt(x * x + y * y)
        l = np.rint(th / (2 * np.pi / 8)).astype(int) % 8
        w = np.maximum(0.0, 1.0 - np.abs(r[..., None] / h - np.arange(nk)))
        return np.sum(w * prof.T[l], axis=-1)
    f = _field(8, 8, 8, seed=2)
    assert np.allclose(t, 2 * np.pi * np.arange(8) / 8)
    assert rel_l2(C.conv_chain(f, [p]), Q.quadrature_conv(f, rho)) < 1e-13


def test_non_radial_kernel_is_detected():
    # Negative control: without radiality the rotation does not drop out and the
    # product of coefficients is not the SE(2) convolution.
    f = _field(8, 8, 8, seed=3)
    rho = K.anisotropic_function(0.05, 0.16, 2.0)
    p = K.sample_function(rho, 8, 8, 8)
    assert rel_l2(C.conv_chain(f, [p]), Q.quadrature_conv(f, rho)) > 1e-2


def test_alg3_matrix_form_equals_route1():
    f = _field(16, 16, 8, seed=4)
    p = K.gauss_vm(16, 16, 8, 0.07, 3.0, 1.0)
    assert rel_l2(C.alg3_matrix_form(f, p), C.conv_chain(f, [p])) < 1e-14


def test_closed_form_c0_and_convergence():
    # Gaussian x von Mises bumps * Gaussian x von Mises kernel: widths add,
    # angular coefficients multiply.  Error is aliasing-limited and must shrink
    # as the grid is refined.
    bf = bump_field(0, 0, 8)
    ker = KernelParams(0.05, 4.0, 0.0)
    errs = []
    for n, m in [(32, 32), (64, 32), (64, 64)]:
        f = sample_field(bf, n, n, m)
        p = K.gauss_vm(n, n, m, ker.sigma, ker.kappa, 0.0, normalize="continuous")
        errs.append(rel_l2(C.conv_chain(f, [p]), CF.conv_closed_form(bf, [ker], n, n, m)))
    assert errs[0] < 1e-7
    assert errs[1] < 1e-12 and errs[2] < 1e-12


def test_closed_form_on_odd_grids():
    # The paper's own grids are odd, L = 2K+1 with |k| <= K (Sec. 3.2).  There the
    # sign (-1)^{k1+k2} belongs to the signed frequency, not the DFT index, and the
    # series is a trigonometric interpolant of the convolution: the error against
    # the continuous closed form must fall quickly as L grows (odd x, y and theta).
    bf = bump_field(93, 0, 6, s=0.05, kappa=3.0)
    chain = [KernelParams(0.04, 5.0, 0.4), KernelParams(0.03, 2.0, 1.1)]
    errs = []
    for nx, ny, m in [(25, 27, 25), (41, 43, 45), (61, 63, 65)]:
        f = sample_field(bf, nx, ny, m)
        ps = [K.gauss_vm(nx, ny, m, k.sigma, k.kappa, k.theta0, normalize="continuous") for k in chain]
        errs.append(rel_l2(C.conv_chain(f, ps), CF.conv_closed_form(bf, chain, nx, ny, m)))
    assert errs[0] < 1e-3 and errs[1] < 1e-9 and errs[2] < 1e-13, errs


def test_closed_form_chain_with_angle_offsets():
    # Asymmetric bumps and kernels with theta offsets: catches transposed axes,
    # a conjugated angular phase or a dropped kernel.
    bf = bump_field(91, 0, 5, s=0.05, kappa=3.0)
    chain = [KernelParams(0.04, 5.0, 0.4), KernelParams(0.03, 2.0, 1.1), KernelParams(0.05, 8.0, 5.0)]
    n, m = 64, 64
    f = sample_field(bf, n, n, m)
    ps = [K.gauss_vm(n, n, m, k.sigma, k.kappa, k.theta0, normalize="continuous") for k in chain]
    assert rel_l2(C.conv_chain(f, ps), CF.conv_closed_form(bf, chain, n, n, m)) < 1e-10


def test_field_closed_form_matches_generator():
    bf = bump_field(0, 3, 8)
    assert rel_l2(sample_field(bf, 16, 16, 8), CF.field_closed_form(bf, 16, 16, 8)) < 1e-13


def test_mass_is_multiplicative():
    # rho^[0;L] = mean(P), so the mean of the output is mean(f) * prod mean(P_j).
    f = _field(16, 16, 8, seed=5)
    ps = [K.gauss_vm(16, 16, 8, 0.06, 2.0, normalize=None),
          K.gauss_vm(16, 16, 8, 0.1, 7.0, 0.3, normalize=None)]
    out = C.conv_chain(f, ps)
    expect = f.mean() * ps[0].mean() * ps[1].mean()
    assert abs(out.mean() - expect) < 1e-13 * abs(expect)


def test_radial_coefficients_have_d4_symmetry():
    n, m = 16, 8
    p = K.gauss_vm(n, n, m, 0.07, 3.0, 0.9)
    c = ffc(p)
    neg = (-np.arange(n)) % n
    assert np.max(np.abs(c - np.swapaxes(c, 1, 2))) < 1e-15          # k1 <-> k2
    assert np.max(np.abs(c - c[:, :, neg])) < 1e-15                   # k1 -> -k1
    assert np.max(np.abs(c - c[:, neg, :])) < 1e-15                   # k2 -> -k2


def _rotate90(f):
    # (L_h f)(x, theta) = f(h^{-1} o (x, theta)) with h = (0, R_{pi/2}):
    # f(R_{-pi/2} x, theta - pi/2) = f((y, -x), theta - pi/2).
    m, n, _ = f.shape
    out = np.empty_like(f)
    i = np.arange(n)
    for l in range(m):
        src = f[(l - m // 4) % m]
        # out[l][j][i] = src[y-index (-x_i) = (n - i) mod n][x-index (y_j) = j]
        out[l] = src[((n - i) % n)[None, :], i[:, None]]
    return out


def test_left_rotation_equivariance():
    f = _field(16, 16, 8, seed=6)
    p = K.gauss_vm(16, 16, 8, 0.08, 2.0, 0.5)
    a = C.conv_chain(_rotate90(f), [p])
    b = _rotate90(C.conv_chain(f, [p]))
    assert rel_l2(a, b) < 1e-13
    # and the rotation is not trivial on this field
    assert rel_l2(_rotate90(f), f) > 1e-2


def test_delta_kernel_is_identity():
    f = _field(8, 12, 8, seed=7)
    assert rel_l2(C.conv_chain(f, [K.delta(8, 12, 8)]), f) < 1e-14


def test_theta_delta_reduces_to_2d_circular_convolution():
    # rho = g(x) * delta(theta): per theta-slice 2-D circular convolution of the
    # samples with the periodized g centred at index N/2 (brute-force shifts).
    n, m = 8, 4
    f = _field(n, n, m, seed=8)
    g = K.gauss_vm(n, n, 1, 0.09, 0.0, normalize=None)[0]
    p = np.zeros((m, n, n))
    p[0] = g * m
    out = C.conv_chain(f, [p])
    ref = np.zeros_like(f)
    for l in range(m):
        for j in range(n):
            for i in range(n):
                ref[l] += f[l, j, i] * np.roll(np.roll(g, j - n // 2, axis=0), i - n // 2, axis=1)
    ref /= n * n
    assert rel_l2(out, ref) < 1e-14


def test_x_delta_reduces_to_1d_circular_convolution_in_theta():
    n, m = 4, 16
    f = _field(n, n, m, seed=9)
    h = np.exp(3.0 * np.cos(2 * np.pi * np.arange(m) / m - 0.4))
    p = np.zeros((m, n, n))
    p[:, n // 2, n // 2] = h * n * n
    out = C.conv_chain(f, [p])
    ref = np.zeros_like(f)
    for c in range(m):
        for l in range(m):
            ref[c] += f[l] * h[(c - l) % m]
    ref /= m
    assert rel_l2(out, ref) < 1e-14


def test_chain_is_order_free():
    f = _field(8, 8, 8, seed=10)
    ps = [K.gauss_vm(8, 8, 8, s, k, t) for s, k, t in [(0.05, 2, 0), (0.1, 5, 1), (0.07, 1, 3)]]
    a = C.conv_chain(f, ps)
    b = C.conv_chain(f, ps[::-1])
    assert rel_l2(a, b) < 1e-14


@pytest.mark.parametrize("q", [1, 2, 3, 4])
def test_alg4_power_matches_chain_of_identical_kernels(q):
    # Algorithm 4 (W only for odd q) against q explicit factors.
    f = _field(8, 8, 8, seed=11)
    p = K.gauss_vm(8, 8, 8, 0.06, 2.0, 0.3)
    assert rel_l2(C.alg4_power(f, p, q), C.conv_chain(f, [p] * q)) < 1e-13


def test_alg7_equals_alg6_and_alg4():
    f = _field(8, 8, 8, seed=12)
    p = K.gauss_vm(8, 8, 8, 0.05, 3.0, 0.6)
    fast = C.alg7_all_powers(f, p, 5)
    naive = C.alg6_naive_recursive(f, p, 5)
    for q, (a, b) in enumerate(zip(fast, naive), start=1):
        assert rel_l2(a, b) < 1e-13
        assert rel_l2(a, C.alg4_power(f, p, q)) < 1e-13


def test_adjoint_flag_is_transpose(rng):
    # <A x, y> = <x, A^T y> for the real-linear convolution operator.
    f = rng.standard_normal((8, 8, 8))
    g = rng.standard_normal((8, 8, 8))
    p = K.gauss_vm(8, 8, 8, 0.06, 2.0, 0.9)
    lhs = np.sum(C.conv_chain(f, [p]) * g)
    rhs = np.sum(f * C.conv_chain(g, [p], adjoint=True))
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)


def test_real_input_gives_real_output():
    f = _field(8, 8, 8, seed=13)
    p = K.gauss_vm(8, 8, 8, 0.06, 2.0, 0.9)
    z = C.conv_chain(f, [p], return_complex=True)
    assert np.max(np.abs(z.imag)) < 1e-15 * np.max(np.abs(z.real))


def test_closed_form_at_the_gradient_benchmark_kernel():
    # sigma* = 0.04, kappa* = 8 (the target kernel of the differentiation workload)
    bf = bump_field(4, 0, 32)
    f = sample_field(bf, 64, 64, 64)
    p = K.gauss_vm(64, 64, 64, 0.04, 8.0, 0.0, normalize="continuous")
    ref = CF.conv_closed_form(bf, [KernelParams(0.04, 8.0)], 64, 64, 64)
    assert rel_l2(C.conv_chain(f, [p]), ref) < 1e-8
