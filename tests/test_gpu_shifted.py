"""GPU parity: convolution with sums of SE(2)-shifted radial kernels (se2conv_shift_table,
se2conv_apply_shifted) against the FP64 oracle (oracle.shifted), and on exact-grid shifts
against the direct quadrature of the shifted kernel sum."""
import numpy as np
import pytest
import torch

import paper_2504_05149_amd as se2
from gpu_common import TOL64, case, parity_err, tol32
from inputs import sample_fields
from oracle import kernels as ok
from oracle import quadrature as oq
from oracle import shifted as osh

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _shifts(rng, m, n_terms, n_rolls):
    rolls = rng.choice(m, size=n_rolls, replace=False)
    out = []
    for k in range(n_terms):
        out.append((float(rng.uniform(-0.4, 0.4)), float(rng.uniform(-0.4, 0.4)), int(rolls[k % n_rolls]),
                    float(rng.uniform(-1.0, 1.0))))
    return out


def _oracle(f, p, shifts, m):
    sh = [(tx, ty, 2 * np.pi * r / m) for tx, ty, r, _ in shifts]
    w = [a for _, _, _, a in shifts]
    return osh.shifted_sum_conv(f, p, sh, w)


CASES = [
    # (nx, ny, m, batch, terms, rolls, dtype)
    (16, 16, 8, 2, 3, 1, "f64"),
    (24, 20, 12, 3, 5, 3, "f64"),
    (15, 9, 7, 2, 4, 2, "f64"),
    (32, 32, 16, 4, 8, 2, "f32"),
    (24, 20, 12, 3, 5, 3, "f32"),
    (48, 36, 10, 1, 6, 4, "f32"),
    (64, 64, 64, 2, 8, 8, "f32"),
    # register kernels around the shift-mix pass: odd batch, a single field, rectangular grids
    (64, 32, 32, 3, 5, 3, "f32"),
    (128, 64, 16, 1, 4, 2, "f32"),
]


@pytest.mark.parametrize("nx,ny,m,batch,terms,nrolls,dt", CASES)
def test_shifted_sum_matches_oracle(nx, ny, m, batch, terms, nrolls, dt):
    case(f"shifted kernel sum {nx}x{ny}x{m} batch {batch}, {terms} shifts in {nrolls} rolls, {dt}")
    rng = np.random.default_rng(nx * 1000 + ny * 10 + m)
    shifts = _shifts(rng, m, terms, nrolls)
    tdt = torch.float32 if dt == "f32" else torch.float64
    f = sample_fields(21, batch, 8, nx, ny, m)
    plan = se2.Plan([(nx, ny, m)], dtype=dt)
    q = plan.shift_table(0, shifts)
    rho = plan.coeffs(0, [se2.GaussVM(0.07, 3.0, 0.4)])
    out = plan.apply_shifted(0, torch.from_numpy(f).to(DEV, tdt), q, [rho])
    torch.cuda.synchronize()
    out = out.cpu().numpy().astype(np.float64)
    p = ok.gauss_vm(nx, ny, m, 0.07, 3.0, 0.4)
    tol = TOL64 if dt == "f64" else tol32(nx * ny * m)
    for b in range(batch):
        err = parity_err(out[b], _oracle(f[b], p, shifts, m))
        print(f"  field {b}: err {err:.2e} (tol {tol:.1e})", flush=True)
        assert err <= tol
    plan.close()


@pytest.mark.parametrize("dt", ["f64", "f32"])
def test_exact_grid_shifts_equal_direct_quadrature(dt):
    case(f"shifted kernel sum on exact grid shifts (12x12x4) vs direct quadrature, {dt}")
    n, m = 12, 4
    shifts = [(2 / n, -3 / n, 0, 0.7), (-1 / n, 5 / n, 1, -0.4), (4 / n, 1 / n, 2, 1.3), (0.0, 0.0, 3, 0.25)]
    f = sample_fields(22, 2, 4, n, n, m)
    rho = ok.gauss_vm_function(0.08, 2.0, 0.3)
    p = ok.sample_function(rho, n, n, m)
    plan = se2.Plan([(n, n, m)], dtype=dt)
    q = plan.shift_table(0, shifts)
    # the radial kernel from its raw samples (no renormalisation), as route 2 sees it
    tk = plan.coeffs(0, [se2.Samples(torch.from_numpy(p).to(DEV), norm=2)])
    tdt = torch.float32 if dt == "f32" else torch.float64
    out = plan.apply_shifted(0, torch.from_numpy(f).to(DEV, tdt), q, [tk]).cpu().numpy().astype(np.float64)
    kern = osh.shifted_kernel_function(rho, [(tx, ty, 2 * np.pi * r / m) for tx, ty, r, _ in shifts],
                                       [a for *_, a in shifts])
    tol = TOL64 if dt == "f64" else tol32(n * n * m)
    for b in range(2):
        err = parity_err(out[b], oq.quadrature_conv(f[b], kern))
        print(f"  field {b}: err {err:.2e}", flush=True)
        assert err <= tol
    plan.close()


def test_shift_table_fp64_matches_oracle_phases():
    case("shift table FP64 (20x16x6, 3 rolls) against the oracle's phases")
    nx, ny, m = 20, 16, 6
    rng = np.random.default_rng(5)
    shifts = _shifts(rng, m, 7, 3)
    plan = se2.Plan([(nx, ny, m)], dtype="f64")
    q = plan.shift_table(0, shifts)
    torch.cuda.synchronize()
    got = q.buf.view(torch.complex128).cpu().numpy()
    rolls = []
    for _, _, r, _ in shifts:
        if r not in rolls:
            rolls.append(r)
    assert got.size == len(rolls) * nx * ny * m
    got = got.reshape(len(rolls), m, ny, nx)
    alpha = 2 * np.pi * np.arange(m) / m
    for j, r in enumerate(rolls):
        ref = np.zeros((m, ny, nx), complex)
        for tx, ty, rr, a in shifts:
            if rr != r:
                continue
            ux, uy = osh.slice_translation(alpha, tx, ty)
            ref += a * osh.axis_phase(ny, uy)[:, :, None] * osh.axis_phase(nx, ux)[:, None, :]
        err = np.max(np.abs(got[j] - ref)) / np.max(np.abs(ref))
        print(f"  roll {r}: max rel err {err:.2e}", flush=True)
        assert err < 1e-13
    plan.close()


def test_shifted_with_full_kernel_table_at_256x256x64():
    case("shifted sum, exponential-coordinates Gaussian, 256x256x64 fp32 batch 4, 2 fields vs oracle")
    nx = ny = 256
    m = 64
    rng = np.random.default_rng(7)
    shifts = _shifts(rng, m, 8, 2)
    f = sample_fields(23, 4, 32, nx, ny, m, dtype=np.float32)
    plan = se2.Plan([(nx, ny, m)], dtype="f32")
    q = plan.shift_table(0, shifts)
    rho = plan.coeffs(0, [se2.ExpGauss(0.05)])
    out = plan.apply_shifted(0, torch.from_numpy(f).to(DEV), q, [rho])
    torch.cuda.synchronize()
    out = out.cpu().numpy().astype(np.float64)
    p = ok.sample_function(ok.exp_gauss_function(0.05), nx, ny, m, images=3)
    p = p / p.mean()
    tol = tol32(nx * ny * m)
    for b in (0, 3):
        err = parity_err(out[b], _oracle(f[b].astype(np.float64), p, shifts, m))
        print(f"  field {b}: err {err:.2e} (tol {tol:.1e})", flush=True)
        assert err <= tol
    plan.close()
