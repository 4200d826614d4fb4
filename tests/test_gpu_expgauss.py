"""GPU parity for the exponential-coordinates Gaussian kernel (Sec. 6.3, eq. (gbS0)):
its FULL coefficient table generated on the device in FP64, the convolution through
the full-table passes, and the powers V_q = f * rho^(q) of the paper's fast loop.
"""
import numpy as np
import pytest
import torch

import paper_2504_05149_amd as se2
from gpu_common import TOL64, case, parity_err, tol32
from inputs import sample_fields
from oracle import conv as oc
from oracle import kernels as ok
from oracle.ffc import ffc

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def _dev(a, dtype):
    return torch.from_numpy(np.ascontiguousarray(a)).to(device=DEV, dtype=dtype)


def _samples(shape, sigma):
    return ok.sample_function(ok.exp_gauss_function(sigma), *shape, images=3)


@pytest.mark.parametrize("shape,sigma", [((32, 24, 16), 0.1), ((33, 29, 25), 0.2)])
def test_exp_gauss_table_fp64_matches_oracle(shape, sigma):
    case(f"exp-coordinates Gaussian table fp64 {shape} sigma={sigma}")
    plan = se2.Plan([shape], dtype="f64")
    t = plan.coeffs(0, [se2.ExpGauss(sigma)])
    t_raw = plan.coeffs(0, [se2.ExpGauss(sigma, norm=2)])
    torch.cuda.synchronize()
    assert t.kind == 1
    c = ffc(_samples(shape, sigma))
    for gpu, ref in ((t.complex_view().cpu().numpy(), c / c[0, 0, 0]), (t_raw.complex_view().cpu().numpy(), c)):
        err = np.max(np.abs(gpu - ref)) / np.max(np.abs(ref))
        print(f"max rel err {err:.2e}", flush=True)
        assert err < 1e-13


@pytest.mark.parametrize("shape,batch,dt", [((64, 64, 32), 3, "f32"), ((256, 256, 64), 2, "f32"),
                                            ((48, 40, 24), 2, "f64")])
def test_exp_gauss_convolution(shape, batch, dt):
    case(f"exp-coordinates Gaussian convolution {shape} batch={batch} {dt}")
    tdt = torch.float32 if dt == "f32" else torch.float64
    sigma = 0.08
    plan = se2.Plan([shape], dtype=dt)
    table = plan.coeffs(0, [se2.ExpGauss(sigma)])
    f = sample_fields(11, batch, 16, *shape)
    out = plan.apply(0, _dev(f, tdt), table)
    torch.cuda.synchronize()
    out = out.cpu().numpy().astype(np.float64)
    p = _samples(shape, sigma)
    p = p / p.mean()
    tol = tol32(shape[0] * shape[1] * shape[2]) if dt == "f32" else TOL64
    worst = 0.0
    for b in range(batch):
        worst = max(worst, parity_err(out[b], oc.conv_chain(f[b], [p])))
        print(f"field {b}: rel-L2 {worst:.2e}", flush=True)
    assert worst <= tol


def test_exp_gauss_powers_fast_loop():
    shape, q = (64, 64, 32), 4
    case(f"V_q = f * rho^(q), q = 1..{q}, exp-coordinates Gaussian {shape} fp32")
    sigma = 0.06
    plan = se2.Plan([shape], dtype="f32")
    table = plan.coeffs(0, [se2.ExpGauss(sigma)])
    f = sample_fields(12, 3, 16, *shape)
    pw = plan.powers(0, _dev(f, torch.float32), table, q)
    torch.cuda.synchronize()
    p = _samples(shape, sigma)
    p = p / p.mean()
    tol = tol32(shape[0] * shape[1] * shape[2])
    for b in range(3):
        ref = f[b]
        for k in range(q):
            ref = oc.conv_chain(ref, [p])
            err = parity_err(pw[k][b].cpu().numpy().astype(np.float64), ref)
            assert err <= tol, (b, k + 1, err)
    print("all powers within tolerance", flush=True)
