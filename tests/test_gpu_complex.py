"""GPU parity for complex-valued fields f: SE(2) -> C (Sec. 3.2): se2conv_apply_complex
against the FP64 oracle, which is complex throughout (route 1 with return_complex)."""
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


def _cfield(cfg, batch, shape):
    a = sample_fields(cfg, 2 * batch, 8, *shape)
    return a[:batch] + 1j * a[batch:]


@pytest.mark.parametrize("shape,batch,lc,dt,adjoint", [
    ((32, 24, 16), 3, 2, "f32", False),
    ((64, 64, 32), 2, 3, "f32", True),
    ((33, 31, 17), 2, 1, "f64", False),
    ((45, 40, 21), 1, 2, "f32", False),
])
def test_complex_fields_separable_chain(shape, batch, lc, dt, adjoint):
    case(f"complex fields {shape} batch={batch} chain={lc} {dt} adjoint={adjoint}")
    cdt = torch.complex64 if dt == "f32" else torch.complex128
    plan = se2.Plan([shape], dtype=dt)
    ks = chain_kernel_params(13, lc)
    chain = [(k.sigma, k.kappa, 0.5 * j) for j, k in enumerate(ks)]
    table = plan.coeffs(0, [se2.GaussVM(*c) for c in chain])
    f = _cfield(13, batch, shape)
    out = plan.apply_complex(0, torch.from_numpy(f).to(DEV, cdt), table, adjoint=adjoint)
    torch.cuda.synchronize()
    out = out.cpu().numpy().astype(np.complex128)
    ps = [ok.gauss_vm(*shape, *c) for c in chain]
    tol = tol32(shape[0] * shape[1] * shape[2]) if dt == "f32" else TOL64
    worst = max(parity_err(out[b], oc.conv_chain(f[b], ps, return_complex=True, adjoint=adjoint))
                for b in range(batch))
    print(f"rel-L2 {worst:.2e} (tol {tol:.1e})", flush=True)
    assert worst <= tol


def test_complex_fields_full_table_in_place_and_real_consistency():
    shape, batch = (48, 40, 24), 3
    case(f"complex fields, radial-profile table, in place, {shape} fp32; Re/Im against the real path")
    rng = np.random.default_rng([2504_05149, 82])
    prof = rng.uniform(0, 1, size=(10, shape[2]))
    plan = se2.Plan([shape], dtype="f32")
    table = plan.coeffs(0, [se2.RadialProfile(torch.from_numpy(prof).to(DEV), 0.4)])
    f = _cfield(14, batch, shape)
    fd = torch.from_numpy(f).to(DEV, torch.complex64)
    re = plan.apply(0, fd.real.contiguous(), table)
    im = plan.apply(0, fd.imag.contiguous(), table)
    plan.apply_complex(0, fd, table, out=fd)
    torch.cuda.synchronize()
    out = fd.cpu().numpy().astype(np.complex128)
    p = ok.radial_profile(*shape, prof, 0.4)
    tol = tol32(shape[0] * shape[1] * shape[2])
    for b in range(batch):
        err = parity_err(out[b], oc.conv_chain(f[b], [p], return_complex=True))
        assert err <= tol, (b, err)
    both = (re + 1j * im).cpu().numpy().astype(np.complex128)
    d = parity_err(out, both)
    print(f"complex path against two real applies: rel-L2 {d:.2e}", flush=True)
    assert d <= tol
