"""The remaining workload configurations at their full sizes.

C2: 256 independent problems of mixed sizes in one graph submission.
C3: 512 x 512 x 128, FP32 and FP64 GPU paths, scored on the 64 x 64 x 32 subsample.
C4: 256 x 256 x 64 FP32 batch 8, loss gradients w.r.t. the field and a 64 x 64 radial profile.
"""
import numpy as np
import pytest
import torch

import paper_2504_05149_amd as se2
from gpu_common import TOL64, case, oracle_table_gauss, parity_err, tol32
from inputs import chain_kernel_params, sample_field, sample_fields, uneven_problem_list
from oracle import adjoint as OA
from oracle import conv as oc
from oracle import kernels as ok
from oracle.ffc import ffc
from paper_2504_05149_amd.autograd import radial_profile_conv

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _dev(a, dtype):
    return torch.from_numpy(np.ascontiguousarray(a)).to(device=DEV, dtype=dtype)


def test_c2_uneven_batch_graph():
    case("C2: 256 problems, N in {32,48,64,96,128}, M in {16,32,64}, chains of 1..4, one graph")
    probs = uneven_problem_list(2, 256)
    shapes = sorted({(p["n"], p["n"], p["m"]) for p in probs})
    sidx = {s: i for i, s in enumerate(shapes)}
    plan = se2.Plan(shapes, dtype="f32")
    items, host = [], []
    for p in probs:
        s = (p["n"], p["n"], p["m"])
        f = sample_field(p["field"], *s)
        table = plan.coeffs(sidx[s], [se2.GaussVM(k.sigma, k.kappa, k.theta0) for k in p["chain"]])
        fd = _dev(f[None], torch.float32)
        items.append((sidx[s], fd, torch.empty_like(fd), [table]))
        host.append((f, p))
    stream = torch.cuda.Stream()
    torch.cuda.synchronize()
    plan.chain(items, stream=stream)
    torch.cuda.synchronize()
    eager = [it[2].clone() for it in items]
    for rep in range(3):
        for it in items:
            it[2].zero_()
        torch.cuda.synchronize()
        plan.chain(items, graph=True, stream=stream)
        torch.cuda.synchronize()
        for e, it in zip(eager, items):
            assert torch.equal(e, it[2]), f"replay {rep}"
    for i, ((f, p), e) in enumerate(zip(host, eager)):
        out = e.cpu().numpy()[0].astype(np.float64)
        assert abs(out.mean() - f.mean()) <= 1e-5 * abs(f.mean())
        if i % 8 == 0:  # every 8th problem against the oracle
            n, m = p["n"], p["m"]
            ref_t = oracle_table_gauss(n, n, m, [(k.sigma, k.kappa, k.theta0) for k in p["chain"]])
            err = parity_err(out, oc.conv_with_coeffs(f, ref_t))
            assert err <= tol32(n * n * m), (i, n, m, err)


@pytest.fixture(scope="module")
def c3_data():
    nx = ny = 512
    m = 128
    ks = chain_kernel_params(3, 4)
    chain = [(k.sigma, k.kappa, 0.0) for k in ks]
    f = sample_fields(3, 4, 128, nx, ny, m)
    print("  C3 fields sampled", flush=True)
    pts = (np.arange(0, nx, 8), np.arange(0, ny, 8), np.arange(0, m, 4))
    table = oracle_table_gauss(nx, ny, m, chain)
    print("  C3 oracle table done", flush=True)
    ref = oc.conv_with_coeffs(f[0], table, points=pts)
    print("  C3 oracle subsample done", flush=True)
    return f, chain, pts, ref


@pytest.mark.parametrize("dt", ["f32", "f64"])
def test_c3_512x512x128_subsampled(dt, c3_data):
    case(f"C3: 512x512x128 {dt} batch 4, 128 bumps, chain of 4; oracle on the 64x64x32 subsample of field 0")
    f, chain, pts, ref = c3_data
    nx = ny = 512
    m = 128
    f = f.astype(np.float32 if dt == "f32" else np.float64)
    plan = se2.Plan([(nx, ny, m)], dtype=dt)
    table = plan.coeffs(0, [se2.GaussVM(s, k, th) for s, k, th in chain])
    fd = torch.from_numpy(f).to(DEV)
    out = plan.apply(0, fd, table)
    torch.cuda.synchronize()
    del fd
    out0 = out[0].cpu().numpy().astype(np.float64)
    sub = out0[np.ix_(pts[2], pts[1], pts[0])]
    err = parity_err(sub, ref)
    tol = tol32(nx * ny * m) if dt == "f32" else TOL64
    print(f"  subsampled rel-L2 {err:.2e} (tol {tol:.1e})", flush=True)
    assert err <= tol
    o = out.cpu().numpy()
    for b in range(4):
        assert abs(o[b].mean() - f[b].mean()) <= (1e-5 if dt == "f32" else 1e-13) * abs(f[b].mean())


def _c4_problem():
    nx = ny = 256
    m, batch, nk, rmax = 64, 8, 64, 0.5
    f = sample_fields(4, batch, 32, nx, ny, m)
    # target: the convolution with sigma* = 0.04, kappa* = 8 (oracle) plus 1% Gaussian noise
    clean_t = oracle_table_gauss(nx, ny, m, [(0.04, 8.0, 0.0)])
    clean = np.stack([oc.conv_with_coeffs(f[b], clean_t) for b in range(batch)])
    rng = np.random.default_rng([2504_05149, 4, 9999])
    target = clean + 0.01 * np.sqrt(np.mean(clean ** 2)) * rng.standard_normal(clean.shape)
    # initial profile: Gaussian (sigma 0.06) in r times von Mises (kappa 4) at the theta grid
    r = np.arange(nk) * rmax / (nk - 1)
    th = 2 * np.pi * np.arange(m) / m
    prof = np.exp(-r[:, None] ** 2 / (2 * 0.06 ** 2)) * np.exp(4.0 * (np.cos(th)[None, :] - 1.0))
    prof /= ok.radial_profile(nx, ny, m, prof, rmax).mean()
    return f, target, prof, nk, rmax


def test_c4_gradients_256x256x64_batch8():
    case("C4: 256x256x64 fp32 batch 8, grads w.r.t. f and the 64x64 radial profile vs oracle")
    f, target, prof, nk, rmax = _c4_problem()
    m, ny, nx = f.shape[1:]
    plan = se2.Plan([(nx, ny, m)], dtype="f32")
    fd = _dev(f, torch.float32).requires_grad_(True)
    pd = _dev(prof, torch.float64).requires_grad_(True)
    out = radial_profile_conv(fd, pd, plan, 0, rmax, checkpoint=True)
    loss = ((out.double() - _dev(target, torch.float64)) ** 2).sum()
    loss.backward()
    # oracle: loss, grad_f of fields 0 and 5, grad_prof over the whole batch
    table = ffc(ok.radial_profile(nx, ny, m, prof, rmax))
    outs = np.stack([oc.conv_with_coeffs(f[b], table) for b in range(f.shape[0])])
    g = 2.0 * (outs - target)
    ref_loss = float(np.sum((outs - target) ** 2))
    gP = np.stack([OA.grad_kernel_samples(f[b], g[b]) for b in range(f.shape[0])])
    ref_gprof = OA.grad_profile(gP, nk, rmax)
    e_loss = abs(loss.item() - ref_loss) / ref_loss
    e_gp = parity_err(pd.grad.cpu().numpy(), ref_gprof)
    print(f"  loss {e_loss:.2e} grad_prof {e_gp:.2e}", flush=True)
    assert e_loss <= 1e-4 and e_gp <= 1e-4
    gf = fd.grad.cpu().numpy()
    for b in (0, 5):
        e_gf = parity_err(gf[b], oc.conv_with_coeffs(g[b], np.conj(table)))
        print(f"  grad_f field {b}: {e_gf:.2e}", flush=True)
        assert e_gf <= 1e-4


def test_c4_finite_differences_fp64_at_full_size():
    """Central differences of the C4 loss at its full size, on the FP64 GPU path: the loss is
    quadratic in the field and in the profile (the output is linear in each), so the central
    difference equals the derivative up to rounding, whatever h; a large h keeps the
    rounding of the two loss sums (33.5 M terms each) small against 2h."""
    case("C4 shape 256x256x64 batch 8, FP64: central differences on 6 field and 6 profile coordinates")
    f, target, prof, nk, rmax = _c4_problem()
    m, ny, nx = f.shape[1:]
    plan = se2.Plan([(nx, ny, m)], dtype="f64")
    fd0 = _dev(f, torch.float64)
    pd0 = _dev(prof, torch.float64)
    tgt = _dev(target, torch.float64)

    def loss_of(fa, pa):
        with torch.no_grad():
            out = radial_profile_conv(fa, pa, plan, 0, rmax, True)
            return float(((out - tgt) ** 2).sum().item())

    fd = fd0.clone().requires_grad_(True)
    pd = pd0.clone().requires_grad_(True)
    out = radial_profile_conv(fd, pd, plan, 0, rmax, True)
    ((out - tgt) ** 2).sum().backward()
    rng = np.random.default_rng([2504_05149, 4, 7])
    h = 0.1
    for _ in range(6):
        idx = tuple(int(rng.integers(0, s)) for s in f.shape)
        fp, fm = fd0.clone(), fd0.clone()
        fp[idx] += h
        fm[idx] -= h
        num = (loss_of(fp, pd0) - loss_of(fm, pd0)) / (2 * h)
        ana = fd.grad[idx].item()
        print(f"  d/df{idx}: {num:.9e} vs {ana:.9e}", flush=True)
        assert abs(num - ana) <= 1e-5 * max(1.0, abs(ana)), (idx, num, ana)
    for _ in range(6):
        idx = (int(rng.integers(0, nk // 4)), int(rng.integers(0, m)))  # knots inside the kernel's reach
        pp, pm = pd0.clone(), pd0.clone()
        pp[idx] += h
        pm[idx] -= h
        num = (loss_of(fd0, pp) - loss_of(fd0, pm)) / (2 * h)
        ana = pd.grad[idx].item()
        print(f"  d/dprof{idx}: {num:.9e} vs {ana:.9e}", flush=True)
        assert abs(num - ana) <= 1e-5 * max(1.0, abs(ana)), (idx, num, ana)
    plan.close()
