"""Pins for the exponential-coordinates Gaussian on SE(2) (Sec. 6.3, eq. (gbS0); the
multidimensional Gaussian of eq. (fbS) with mean identity and Sigma = sigma^2 I).

The closed form of ||log(x, R)^v||^2 is checked against a library matrix logarithm;
the kernel is radial in translations but not separable, so the FFT route must equal
the direct quadrature with explicit rotations (Thm. f*gP), and its coefficients must
carry the D4 symmetry of radial kernels.
"""
import numpy as np
import scipy.linalg as sl

from inputs import bump_field, rel_l2, sample_field
from oracle import conv as C
from oracle import kernels as K
from oracle import quadrature as Q
from oracle.ffc import ffc


def test_log_norm_matches_matrix_logarithm():
    rng = np.random.default_rng([2504_05149, 81])
    for _ in range(200):
        x, y = rng.uniform(-1.0, 1.0, 2)
        t = rng.uniform(-np.pi + 1e-3, np.pi - 1e-3)
        g = np.array([[np.cos(t), -np.sin(t), x], [np.sin(t), np.cos(t), y], [0.0, 0.0, 1.0]])
        lg = sl.logm(g).real
        v = np.array([lg[0, 2], lg[1, 2], lg[1, 0]])
        assert abs(v @ v - K.se2_log_sq_norm(x, y, t)) < 1e-10
    # identity rotation: the plain Euclidean norm; half turn: |x| scaled by pi/2
    assert K.se2_log_sq_norm(0.3, -0.4, 0.0) == 0.25
    assert abs(K.se2_log_sq_norm(0.3, -0.4, np.pi) - (np.pi / 2) ** 2 * 0.25 - np.pi ** 2) < 1e-14


def test_kernel_is_not_separable():
    # the x-width depends on theta: the sampled kernel is not a product g(x) h(theta)
    p = K.sample_function(K.exp_gauss_function(0.3), 16, 16, 8)
    u, s, vt = np.linalg.svd(p.reshape(8, -1), full_matrices=False)
    assert s[1] / s[0] > 1e-3


def test_route1_equals_direct_quadrature():
    f = sample_field(bump_field(94, 0, 4, s=0.08, kappa=2.0), 8, 12, 8)
    rho = K.exp_gauss_function(0.12)
    p = K.sample_function(rho, 8, 12, 8)
    assert rel_l2(C.conv_chain(f, [p]), Q.quadrature_conv(f, rho)) < 1e-13


def test_route1_equals_direct_quadrature_wider_kernel():
    # a wider kernel reaches larger angles, where (t/2)/sin(t/2) departs from 1; the
    # bar reflects the lattice images (+-2) the two routes truncate differently
    f = sample_field(bump_field(94, 1, 4, s=0.1, kappa=1.0), 8, 8, 12)
    rho = K.exp_gauss_function(0.3)
    p = K.sample_function(rho, 8, 8, 12)
    assert rel_l2(C.conv_chain(f, [p]), Q.quadrature_conv(f, rho)) < 1e-11


def test_coefficients_have_d4_symmetry():
    n, m = 16, 8
    c = ffc(K.sample_function(K.exp_gauss_function(0.2), n, n, m))
    neg = (-np.arange(n)) % n
    assert np.max(np.abs(c - np.swapaxes(c, 1, 2))) < 1e-15
    assert np.max(np.abs(c - c[:, :, neg])) < 1e-15
    assert np.max(np.abs(c - c[:, neg, :])) < 1e-15


def test_power_form_equals_repeated_convolution():
    # V_q(f, rho) = f * rho^(q) (Sec. 6.3, eq. (Vq)) via Alg. 4 and via q convolutions
    f = sample_field(bump_field(94, 2, 4, s=0.08, kappa=2.0), 12, 12, 8)
    p = K.sample_function(K.exp_gauss_function(0.15), 12, 12, 8)
    for q in (2, 3):
        rep = f
        for _ in range(q):
            rep = C.conv_chain(rep, [p])
        assert rel_l2(C.alg4_power(f, p, q), rep) < 1e-13


def test_reflection_symmetry_on_rectangular_and_odd_grids():
    # the quarter tables keep the coefficients at nonnegative k1, k2: a kernel radial in
    # translations sampled on any grid (odd, even, rectangular) is even in x and in y, so
    # its coefficients are fixed by k1 -> -k1 and k2 -> -k2 separately
    for nx, ny, m in [(12, 20, 8), (15, 9, 7), (11, 16, 6)]:
        c = ffc(K.sample_function(K.exp_gauss_function(0.2), nx, ny, m))
        big = np.max(np.abs(c))
        assert np.max(np.abs(c - c[:, :, (-np.arange(nx)) % nx])) < 1e-15 * big * 8
        assert np.max(np.abs(c - c[:, (-np.arange(ny)) % ny, :])) < 1e-15 * big * 8
    # a Gaussian stretched along a 30-degree axis is not radial: its table is not fixed
    cs, sn = np.cos(np.pi / 6), np.sin(np.pi / 6)

    def tilted(x, y, t):
        u, v = cs * x + sn * y, -sn * x + cs * y
        return np.exp(-u * u / (2 * 0.05 ** 2) - v * v / (2 * 0.15 ** 2)) * np.exp(np.cos(t))

    c = ffc(K.sample_function(tilted, 12, 20, 8))
    assert np.max(np.abs(c - c[:, :, (-np.arange(12)) % 12])) > 1e-3 * np.max(np.abs(c))
