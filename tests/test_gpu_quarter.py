"""GPU parity: FULL tables folded by the reflection symmetries of a radial kernel
(se2conv_table_quarter, the coefficients at nonnegative k1, k2 only) in every path that
takes a FULL table, against the FP64 oracle and against the FULL table they come from.

A kernel radial in translations (Sec. 5.1, footnote to Thm. f*gP) is unchanged by
x1 -> -x1 and x2 -> -x2 on the lattice, so its coefficients are: the quarter table holds
the same information, and a convolution with it must equal the one with the FULL table
up to the rounding of the FULL table's own (not quite symmetric) entries."""
import numpy as np
import pytest
import torch

import paper_2504_05149_amd as se2
from paper_2504_05149_amd import _lib as L
from gpu_common import TOL64, case, parity_err, tol32
from inputs import sample_fields
from oracle import conv as oc
from oracle import kernels as ok

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
SIGMA = 0.07
# full and quarter tables differ only where the FULL table's FP64 values, symmetric to
# rounding, rounded to different neighbours: results agree far below the oracle bar
AGREE32, AGREE64 = 2e-6, 1e-12


def _dev(a, dtype):
    return torch.from_numpy(np.ascontiguousarray(a)).to(device=DEV, dtype=dtype)


def _p(shape):
    p = ok.sample_function(ok.exp_gauss_function(SIGMA), *shape, images=3)
    return p / p.mean()


def _tables(plan, shape_idx=0):
    full = plan.coeffs(shape_idx, [se2.ExpGauss(SIGMA)])
    quarter = plan.quarter(full)
    torch.cuda.synchronize()
    assert full.kind == L.TABLE_FULL and quarter.kind == L.TABLE_QUARTER
    return full, quarter


@pytest.mark.parametrize("shape,dt", [((32, 24, 16), "f32"), ((33, 29, 25), "f64"), ((15, 9, 7), "f32"),
                                      ((256, 256, 64), "f32")])
def test_quarter_is_the_corner_of_the_full_table(shape, dt):
    case(f"quarter table {shape} {dt}: bytes of the FULL table at nonnegative k1, k2")
    nx, ny, m = shape
    plan = se2.Plan([shape], dtype=dt)
    full, quarter = _tables(plan)
    fv = full.complex_view().cpu().numpy()
    qv = quarter.complex_view().cpu().numpy()
    assert qv.shape == (m, ny // 2 + 1, nx // 2 + 1)
    assert np.array_equal(qv, fv[:, :ny // 2 + 1, :nx // 2 + 1])
    # and the fold reproduces the whole table up to rounding
    ax = np.minimum(np.arange(nx), nx - np.arange(nx))
    ay = np.minimum(np.arange(ny), ny - np.arange(ny))
    unfolded = qv[:, ay][:, :, ax]
    tol = 1e-6 if dt == "f32" else 1e-13
    err = np.max(np.abs(unfolded - fv)) / np.max(np.abs(fv))
    print(f"  unfolded vs FULL: max rel {err:.2e}", flush=True)
    assert err <= tol
    nbytes = quarter.buf.numel()
    assert nbytes == m * (ny // 2 + 1) * (nx // 2 + 1) * (8 if dt == "f32" else 16)
    plan.close()


# (shape, batch, dtype, generic plan): the register kernels (one quarter table) at the
# supported FP32 sizes, the generic LDS pencils at odd / mixed / FP64 shapes
APPLY = [((256, 256, 64), 3, "f32", False), ((64, 64, 32), 2, "f32", False), ((64, 64, 32), 2, "f32", True),
         ((24, 20, 12), 3, "f64", False), ((15, 9, 7), 2, "f32", False), ((45, 27, 21), 1, "f64", False)]


@pytest.mark.parametrize("shape,batch,dt,generic", APPLY)
def test_apply_with_quarter_table(shape, batch, dt, generic):
    case(f"apply with a quarter table {shape} batch {batch} {dt} generic={generic}")
    tdt = torch.float32 if dt == "f32" else torch.float64
    plan = se2.Plan([shape], dtype=dt, generic=generic)
    full, quarter = _tables(plan)
    f = sample_fields(31, batch, 16, *shape)
    fd = _dev(f, tdt)
    for adjoint in (False, True):
        oq = plan.apply(0, fd, quarter, adjoint=adjoint)
        of = plan.apply(0, fd, full, adjoint=adjoint)
        torch.cuda.synchronize()
        oq = oq.cpu().numpy().astype(np.float64)
        of = of.cpu().numpy().astype(np.float64)
        agree = parity_err(oq, of)
        print(f"  adjoint={adjoint}: quarter vs full {agree:.2e}", flush=True)
        assert agree <= (AGREE32 if dt == "f32" else AGREE64)
    # the oracle (the kernel is real and even, so the adjoint is the same convolution)
    p = _p(shape)
    tol = tol32(int(np.prod(shape))) if dt == "f32" else TOL64
    for b in sorted({0, batch - 1}):
        err = parity_err(oq[b], oc.conv_chain(f[b], [p]))
        print(f"  field {b}: vs oracle {err:.2e} (tol {tol:.1e})", flush=True)
        assert err <= tol
    plan.close()


@pytest.mark.parametrize("shape,dt", [((64, 64, 32), "f32"), ((128, 256, 32), "f32"), ((24, 20, 12), "f64")])
def test_chain_of_quarter_and_separable(shape, dt):
    case(f"chain [quarter exp-Gaussian, Gauss-vM] {shape} {dt} through se2conv_chain")
    tdt = torch.float32 if dt == "f32" else torch.float64
    plan = se2.Plan([shape], dtype=dt)
    _, quarter = _tables(plan)
    gvm = plan.coeffs(0, [se2.GaussVM(0.05, 4.0, 0.3)])
    f = sample_fields(32, 2, 16, *shape)
    fd = _dev(f, tdt)
    out = torch.empty_like(fd)
    plan.chain([(0, fd, out, [quarter, gvm])])
    torch.cuda.synchronize()
    out = out.cpu().numpy().astype(np.float64)
    ps = [_p(shape), ok.gauss_vm(*shape, 0.05, 4.0, 0.3)]
    tol = tol32(int(np.prod(shape))) if dt == "f32" else TOL64
    for b in range(2):
        err = parity_err(out[b], oc.conv_chain(f[b], ps))
        print(f"  field {b}: {err:.2e}", flush=True)
        assert err <= tol
    plan.close()


@pytest.mark.parametrize("shape", [(64, 64, 32), (32, 512, 16)])
def test_powers_with_quarter_table(shape):
    case(f"all powers q = 3 with a quarter table {shape} fp32 vs the FULL table")
    plan = se2.Plan([shape], dtype="f32")
    full, quarter = _tables(plan)
    f = _dev(sample_fields(33, 2, 16, *shape), torch.float32)
    pq = plan.powers(0, f, quarter, 3).cpu().numpy().astype(np.float64)
    pf = plan.powers(0, f, full, 3).cpu().numpy().astype(np.float64)
    for k in range(3):
        agree = parity_err(pq[k], pf[k])
        print(f"  power {k + 1}: quarter vs full {agree:.2e}", flush=True)
        assert agree <= AGREE32
    plan.close()


def test_padded_with_quarter_table():
    case("evaluation on a finer grid (64x64x32 -> 128x128x64) with a quarter table vs the FULL table")
    plan = se2.Plan([(64, 64, 32), (128, 128, 64)], dtype="f32")
    full, quarter = _tables(plan)
    f = _dev(sample_fields(34, 2, 16, 64, 64, 32), torch.float32)
    oq = plan.apply_padded(0, f, quarter, 1).cpu().numpy().astype(np.float64)
    of = plan.apply_padded(0, f, full, 1).cpu().numpy().astype(np.float64)
    agree = parity_err(oq, of)
    print(f"  quarter vs full {agree:.2e}", flush=True)
    assert agree <= AGREE32
    plan.close()


def test_save_and_backward_with_quarter_table():
    case("apply_save + backward with a quarter table (256x256x64 fp32, batch 2) vs the FULL table")
    shape = (256, 256, 64)
    plan = se2.Plan([shape], dtype="f32")
    full, quarter = _tables(plan)
    f = _dev(sample_fields(35, 2, 16, *shape), torch.float32)
    g = _dev(sample_fields(36, 2, 16, *shape), torch.float32)
    res = {}
    for name, t in (("quarter", quarter), ("full", full)):
        out, spec = plan.apply_save(0, f, t)
        gf, gp = plan.backward(0, g, t, spec)
        torch.cuda.synchronize()
        res[name] = [x.cpu().numpy().astype(np.float64) for x in (out, gf, gp)]
    for i, what in enumerate(("out", "dL/df", "dL/dP")):
        agree = parity_err(res["quarter"][i], res["full"][i])
        print(f"  {what}: quarter vs full {agree:.2e}", flush=True)
        assert agree <= AGREE32
    plan.close()


def test_shifted_sum_with_quarter_table():
    case("shifted kernel sum (48x36x10, 4 shifts) with a quarter radial table vs the FULL table")
    shape = (48, 36, 10)
    plan = se2.Plan([shape], dtype="f32")
    full, quarter = _tables(plan)
    shifts = [(0.1, -0.2, 0, 0.5), (-0.3, 0.05, 3, 1.0), (0.2, 0.2, 3, -0.7), (0.0, 0.1, 7, 0.3)]
    q = plan.shift_table(0, shifts)
    f = _dev(sample_fields(37, 3, 16, *shape), torch.float32)
    oq = plan.apply_shifted(0, f, q, [quarter]).cpu().numpy().astype(np.float64)
    of = plan.apply_shifted(0, f, q, [full]).cpu().numpy().astype(np.float64)
    agree = parity_err(oq, of)
    print(f"  quarter vs full {agree:.2e}", flush=True)
    assert agree <= AGREE32
    plan.close()


@pytest.mark.parametrize("dt", ["f32", "f64"])
def test_non_radial_table_is_refused(dt):
    case(f"a table of non-symmetric samples (20x16x8, {dt}) cannot be folded")
    shape = (20, 16, 8)
    plan = se2.Plan([shape], dtype=dt)
    rng = np.random.default_rng(3)
    samples = torch.from_numpy(rng.uniform(0.5, 1.5, size=(8, 16, 20))).to(DEV)
    full = plan.coeffs(0, [se2.Samples(samples)])
    torch.cuda.synchronize()
    with pytest.raises(L.Se2convError, match="not symmetric"):
        plan.quarter(full)
    # a sample set mirrored in x and y is accepted
    sym = samples.cpu().numpy()
    sym = sym + sym[:, :, (-np.arange(20)) % 20]
    sym = sym + sym[:, (-np.arange(16)) % 16, :]
    full_sym = plan.coeffs(0, [se2.Samples(torch.from_numpy(sym).to(DEV))])
    qt = plan.quarter(full_sym)
    torch.cuda.synchronize()
    assert qt.kind == L.TABLE_QUARTER
    plan.close()
