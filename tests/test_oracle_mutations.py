"""The pins must fail when a plausible mistake is planted in the oracle.

Each case monkeypatches one oracle routine with a wrong variant (on the CPU) and
checks that at least one independent pin (direct quadrature, closed form, mass)
then reports a large error.
"""
import numpy as np
import pytest

import oracle.conv as C
import oracle.ffc as FF
from inputs import bump_field, rel_l2, sample_field
from inputs.fields import KernelParams
from oracle import closed_form as CF
from oracle import kernels as K
from oracle import quadrature as Q


def _pins():
    """Return the errors of three independent pins of route 1."""
    bf = bump_field(92, 0, 4, s=0.08, kappa=2.0)
    f = sample_field(bf, 8, 12, 8)
    rho = K.gauss_vm_function(0.11, 2.5, 0.7)
    p = K.sample_function(rho, 8, 12, 8)
    e_quad = rel_l2(C.conv_chain(f, [p]), Q.quadrature_conv(f, rho))
    chain = [KernelParams(0.04, 5.0, 0.4), KernelParams(0.05, 2.0, 1.1)]
    bf2 = bump_field(92, 1, 5, s=0.05, kappa=3.0)
    f2 = sample_field(bf2, 64, 64, 32)
    ps = [K.gauss_vm(64, 64, 32, k.sigma, k.kappa, k.theta0, normalize="continuous") for k in chain]
    e_cf = rel_l2(C.conv_chain(f2, ps), CF.conv_closed_form(bf2, chain, 64, 64, 32))
    pm = K.gauss_vm(8, 12, 8, 0.06, 2.0, normalize=None)
    out = C.conv_chain(f, [pm])
    e_mass = abs(out.mean() - f.mean() * pm.mean()) / abs(f.mean() * pm.mean())
    return e_quad, e_cf, e_mass


def test_unmutated_pins_are_tight():
    e = _pins()
    assert e[0] < 1e-13 and e[1] < 1e-9 and e[2] < 1e-13


def _no_sign(nx, ny, m):
    return np.ones((m, ny, nx))


def _ffc_no_scale(samples):
    m, ny, nx = samples.shape[-3:]
    return FF.sign_w(nx, ny, m) * FF.dft3(samples)


_orig_phi = FF._phi_axis


def _phi_conj_theta(length, points, grid, spatial):
    e = _orig_phi(length, points, grid, spatial)
    return e if spatial else np.conj(e)


def _phi_no_parity(length, points, grid, spatial):
    k = FF.signed_freqs(length)
    red = np.mod(np.outer(np.asarray(points), k), grid).astype(float)
    return np.exp(2j * np.pi * red / grid)


@pytest.mark.parametrize("target,name,repl", [
    (FF, "sign_w", _no_sign),
    (C, "ffc", _ffc_no_scale),
    (FF, "_phi_axis", _phi_conj_theta),
    (FF, "_phi_axis", _phi_no_parity),
])
def test_planted_mistake_is_caught(monkeypatch, target, name, repl):
    monkeypatch.setattr(target, name, repl)
    e = _pins()
    assert max(e) > 1e-3, (name, e)


def _odd_grid_pin():
    """Closed-form error of a two-kernel chain on an odd grid (Sec. 3.2, L = 2K+1)."""
    bf = bump_field(93, 0, 6, s=0.05, kappa=3.0)
    chain = [KernelParams(0.04, 5.0, 0.4), KernelParams(0.03, 2.0, 1.1)]
    nx, ny, m = 41, 43, 45
    f = sample_field(bf, nx, ny, m)
    ps = [K.gauss_vm(nx, ny, m, k.sigma, k.kappa, k.theta0, normalize="continuous") for k in chain]
    return rel_l2(C.conv_chain(f, ps), CF.conv_closed_form(bf, chain, nx, ny, m))


def _index_parity_w(nx, ny, m):
    # (-1)^{t1+t2} of the DFT index instead of the signed frequency
    s1 = np.where(np.arange(nx) % 2 == 0, 1.0, -1.0)
    s2 = np.where(np.arange(ny) % 2 == 0, 1.0, -1.0)
    return np.broadcast_to(np.outer(s2, s1)[None], (m, ny, nx)).copy()


def _phi_index_parity(length, points, grid, spatial):
    e = _orig_phi(length, points, grid, False)
    if spatial:
        e = e * np.where(np.arange(length) % 2 == 0, 1.0, -1.0)[None, :]
    return e


def test_unmutated_odd_grid_pin_is_tight():
    assert _odd_grid_pin() < 1e-9


@pytest.mark.parametrize("target,name,repl", [
    (FF, "sign_w", _index_parity_w),
    (FF, "_phi_axis", _phi_index_parity),
])
def test_index_parity_on_odd_grids_is_caught(monkeypatch, target, name, repl):
    # on even grids index parity and signed parity agree; on odd grids they do not
    monkeypatch.setattr(target, name, repl)
    assert _odd_grid_pin() > 1e-3


def _phi_parity_on_theta(length, points, grid, spatial):
    # The (-1)^k parity factor applied to the angular axis instead of x and y.
    return _orig_phi(length, points, grid, not spatial)


def test_parity_on_wrong_axis_is_caught(monkeypatch):
    monkeypatch.setattr(FF, "_phi_axis", _phi_parity_on_theta)
    assert max(_pins()) > 1e-3
