"""GPU parity of the zero-padded evaluation (Sec. 4.1 eq. (MatSKfonG), Sec. 6.1 eq.
(MatSKfgonG)): S_K on a grid finer than the sampling grid, against the FP64 oracle's
synthesis at the finer points.  Bars as elsewhere: FP32 rel-L2 <= 2e-6 log2(N^2 M) of
the evaluation grid, FP64 <= 1e-12.
"""
import numpy as np
import pytest
import torch

import paper_2504_05149_amd as se2
from gpu_common import TOL64, case, parity_err, tol32
from inputs import chain_kernel_params, sample_fields
from oracle import conv as oc
from oracle import kernels as ok

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def _dev(a, dtype):
    return torch.from_numpy(np.ascontiguousarray(a)).to(device=DEV, dtype=dtype)


PADDED_CASES = [
    # (sampling grid L, evaluation grid N, batch, chain length, dtype)
    ((25, 27, 23), (40, 41, 30), 3, 2, "f32"),    # odd L (the paper's grids)
    ((24, 26, 20), (48, 39, 20), 2, 1, "f64"),    # even L: Nyquist index split
    ((64, 64, 32), (128, 128, 64), 2, 3, "f32"),  # 2x upsampling of a register-kernel shape
    ((33, 31, 17), (33, 31, 17), 1, 1, "f64"),    # N = L
    ((32, 24, 16), (45, 35, 49), 1, 2, "f32"),    # odd finer grid with radix-5/7 stages
]


@pytest.mark.parametrize("L,N,batch,lc,dt", PADDED_CASES)
def test_padded_evaluation_matches_oracle(L, N, batch, lc, dt):
    case(f"padded evaluation {L} -> {N} batch={batch} chain={lc} {dt}")
    tdt = torch.float32 if dt == "f32" else torch.float64
    plan = se2.Plan([L, N], dtype=dt)
    ks = chain_kernel_params(9, lc)
    table = plan.coeffs(0, [se2.GaussVM(k.sigma, k.kappa, 0.4 * j) for j, k in enumerate(ks)])
    f = sample_fields(9, batch, 8, *L)
    out = plan.apply_padded(0, _dev(f, tdt), table, 1)
    torch.cuda.synchronize()
    out = out.cpu().numpy().astype(np.float64)
    assert out.shape == (batch, N[2], N[1], N[0])
    ps = [ok.gauss_vm(*L, k.sigma, k.kappa, 0.4 * j) for j, k in enumerate(ks)]
    tol = tol32(N[0] * N[1] * N[2]) if dt == "f32" else TOL64
    worst = max(parity_err(out[b], oc.conv_on_grid(f[b], ps, N)) for b in range(batch))
    print(f"rel-L2 {worst:.2e} (tol {tol:.1e})", flush=True)
    assert worst <= tol


def test_padded_full_table_adjoint_and_identity_grid():
    L, N = (33, 33, 17), (64, 64, 32)
    case(f"padded evaluation, radial-profile table, adjoint, {L} -> {N} fp32; N = L equals apply")
    rng = np.random.default_rng([2504_05149, 80])
    prof = rng.uniform(0, 1, size=(10, L[2]))
    plan = se2.Plan([L, N], dtype="f32")
    table = plan.coeffs(0, [se2.RadialProfile(_dev(prof, torch.float64), 0.4)])
    f = sample_fields(10, 3, 8, *L)
    fd = _dev(f, torch.float32)
    out = plan.apply_padded(0, fd, table, 1, adjoint=True)
    same = plan.apply_padded(0, fd, table, 0)
    ref_apply = plan.apply(0, fd, table)
    torch.cuda.synchronize()
    p = ok.radial_profile(*L, prof, 0.4)
    tol = tol32(N[0] * N[1] * N[2])
    for b in range(3):
        err = parity_err(out[b].cpu().numpy().astype(np.float64), oc.conv_on_grid(f[b], [p], N, adjoint=True))
        print(f"field {b}: adjoint rel-L2 {err:.2e}", flush=True)
        assert err <= tol
    d = parity_err(same.cpu().numpy().astype(np.float64), ref_apply.cpu().numpy().astype(np.float64))
    print(f"N = L against se2conv_apply: rel-L2 {d:.2e}", flush=True)
    assert d <= tol32(L[0] * L[1] * L[2])


@pytest.mark.parametrize("L,N,kind,adjoint", [((128, 128, 32), (256, 256, 64), "full", True),
                                              ((64, 32, 16), (128, 64, 32), "sep", False),
                                              ((32, 32, 16), (32, 32, 16), "full", False)])
def test_padded_register_kernels(L, N, kind, adjoint):
    # even FP32 batches on register-kernel grids: x-theta and y spectra on the sampling grid,
    # then one y pass on the evaluation grid that pads, multiplies and inverts
    case(f"padded evaluation on register kernels {L} -> {N} {kind} adjoint={adjoint}")
    plan = se2.Plan([L, N], dtype="f32")
    if kind == "sep":
        ps = [ok.gauss_vm(*L, 0.05, 4.0, 0.3), ok.gauss_vm(*L, 0.03, 8.0, 1.2)]
        table = plan.coeffs(0, [se2.GaussVM(0.05, 4.0, 0.3), se2.GaussVM(0.03, 8.0, 1.2)])
    else:
        prof = np.random.default_rng([2504_05149, 85]).uniform(0, 1, size=(12, L[2]))
        ps = [ok.radial_profile(*L, prof, 0.4)]
        table = plan.coeffs(0, [se2.RadialProfile(_dev(prof, torch.float64), 0.4)])
    f = sample_fields(18, 4, 16, *L)
    fd = _dev(f, torch.float32)
    out = plan.apply_padded(0, fd, table, 1, adjoint=adjoint).cpu().numpy().astype(np.float64)
    tol = tol32(N[0] * N[1] * N[2])
    for b in range(4):
        err = parity_err(out[b], oc.conv_on_grid(f[b], ps, N, adjoint=adjoint))
        print(f"  field {b}: rel-L2 {err:.2e}", flush=True)
        assert err <= tol
    if L == N:
        same = plan.apply(0, fd, table, adjoint=adjoint).cpu().numpy().astype(np.float64)
        assert parity_err(out, same) <= tol
