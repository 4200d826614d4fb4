"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle.

Bars: FP32 path rel-L2 <= 2e-6 log2(N^2 M); FP64 path <= 1e-12.  Every case prints
its name before touching the GPU.
"""
import numpy as np
import pytest
import torch

import paper_2504_05149_amd as se2
from gpu_common import TOL64, case, oracle_conv, oracle_table_gauss, parity_err, tol32
from inputs import bump_field, chain_kernel_params, sample_field, sample_fields
from oracle import conv as oc
from oracle import kernels as ok
from oracle import quadrature as oq
from oracle.ffc import ffc

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def _dev(a, dtype):
    return torch.from_numpy(np.ascontiguousarray(a)).to(device=DEV, dtype=dtype)


def _fields(cfg, batch, nb, nx, ny, m):
    return sample_fields(cfg, batch, nb, nx, ny, m)


def _run(plan, sidx, f, table, dtype):
    out = plan.apply(sidx, _dev(f, dtype), table)
    torch.cuda.synchronize()
    return out.cpu().numpy().astype(np.float64)


# ----------------------------------------------------------------- config C0
def test_c0_fp64_against_both_oracle_routes():
    case("C0 32x32x32 fp64, 8 bumps, sigma=0.05 kappa=4, vs route 1 and direct quadrature")
    n = m = 32
    f = sample_field(bump_field(0, 0, 8), n, n, m)
    plan = se2.Plan([(n, n, m)], dtype="f64")
    table = plan.coeffs(0, [se2.GaussVM(0.05, 4.0, 0.0, norm=1)])  # continuous unit Haar mass
    out = _run(plan, 0, f[None], table, torch.float64)[0]
    p = ok.gauss_vm(n, n, m, 0.05, 4.0, 0.0, normalize="continuous")
    ref1 = oc.conv_chain(f, [p])
    e1 = parity_err(out, ref1)
    ref2 = oq.quadrature_conv(f, ok.gauss_vm_function(0.05, 4.0, 0.0))
    e2 = parity_err(out, ref2)
    print(f"C0 rel-L2: vs DFT route {e1:.2e}, vs quadrature {e2:.2e}", flush=True)
    assert e1 <= TOL64 and e2 <= TOL64


# ------------------------------------------------------ coefficient tables (a2)
@pytest.mark.parametrize("norm,oname", [(0, "discrete"), (1, "continuous"), (2, None)])
def test_separable_table_fp64_matches_oracle_ffc(norm, oname):
    case(f"GaussVM table fp64 48x32x24 norm={oname}")
    nx, ny, m = 48, 32, 24
    plan = se2.Plan([(nx, ny, m)], dtype="f64")
    chain = [(0.07, 3.0, 0.8), (0.04, 11.0, 2.5)]
    t = plan.coeffs(0, [se2.GaussVM(s, k, th, norm=norm) for s, k, th in chain])
    torch.cuda.synchronize()
    v = t.complex_view().cpu().numpy()
    tx, ty, tt = v[:nx], v[nx:nx + ny], v[nx + ny:]
    gpu = tt[:, None, None] * ty[None, :, None] * tx[None, None, :]
    ref = oracle_table_gauss(nx, ny, m, chain, norm=oname)
    err = np.max(np.abs(gpu - ref)) / np.max(np.abs(ref))
    print(f"table max rel err {err:.2e}", flush=True)
    assert err < 1e-13


def test_full_table_from_samples_and_profile_fp64(rng):
    case("FULL table fp64 32x24x16 from samples x radial profile x GaussVM")
    nx, ny, m = 32, 24, 16
    plan = se2.Plan([(nx, ny, m)], dtype="f64")
    p1 = ok.gauss_vm(nx, ny, m, 0.08, 2.0, 0.4, normalize=None)
    prof = rng.uniform(0, 1, size=(9, m))
    p2 = ok.radial_profile(nx, ny, m, prof, 0.45)
    t = plan.coeffs(0, [se2.Samples(_dev(p1, torch.float64)),
                        se2.RadialProfile(_dev(prof, torch.float64), 0.45, norm=2),
                        se2.GaussVM(0.05, 5.0, 1.0)])
    torch.cuda.synchronize()
    assert t.kind == 1
    gpu = t.complex_view().cpu().numpy()
    p3 = ok.gauss_vm(nx, ny, m, 0.05, 5.0, 1.0)
    c1 = ffc(p1) / ffc(p1)[0, 0, 0]  # discrete normalisation of the samples
    ref = c1 * ffc(p2) * ffc(p3)
    err = np.max(np.abs(gpu - ref)) / np.max(np.abs(ref))
    print(f"full table max rel err {err:.2e}", flush=True)
    assert err < 1e-13


# ------------------------------------------------- separable path, FP32 / FP64
SEP_CASES = [
    # (nx, ny, m, batch, chain length, dtype)
    (32, 32, 16, 2, 2, "f32"),
    (48, 96, 16, 3, 1, "f32"),
    (64, 64, 32, 1, 3, "f32"),
    (96, 48, 64, 2, 4, "f32"),
    (16, 8, 6, 5, 2, "f32"),
    (64, 64, 32, 2, 3, "f64"),
    (96, 96, 48, 1, 2, "f64"),
    (512, 16, 64, 2, 2, "f32"),   # x-theta slab too large for LDS: three-pass schedule
    (256, 32, 64, 1, 2, "f64"),   # FP64 slab too large: three-pass schedule
]


@pytest.mark.parametrize("nx,ny,m,batch,lc,dt", SEP_CASES)
def test_separable_path_parity(nx, ny, m, batch, lc, dt):
    case(f"separable {nx}x{ny}x{m} batch={batch} chain={lc} {dt}")
    ks = chain_kernel_params(1, lc)
    chain = [(k.sigma, k.kappa, 0.3 * j) for j, k in enumerate(ks)]
    f = _fields(1, batch, 16, nx, ny, m)
    plan = se2.Plan([(nx, ny, m)], dtype=dt)
    table = plan.coeffs(0, [se2.GaussVM(s, k, th) for s, k, th in chain])
    tdt = torch.float32 if dt == "f32" else torch.float64
    out = _run(plan, 0, f, table, tdt)
    ref_t = oracle_table_gauss(nx, ny, m, chain)
    tol = tol32(nx * ny * m) if dt == "f32" else TOL64
    for b in range(batch):
        err = parity_err(out[b], oracle_conv(f[b], ref_t))
        print(f"  field {b}: rel-L2 {err:.2e} (tol {tol:.1e})", flush=True)
        assert err <= tol


def test_c1_128x128x64_batch16_chain8():
    case("C1 128x128x64 fp32 batch 16, 32 bumps, chain of 8")
    nx = ny = 128
    m = 64
    ks = chain_kernel_params(1, 8)
    chain = [(k.sigma, k.kappa, 0.0) for k in ks]
    f = _fields(1, 16, 32, nx, ny, m)
    plan = se2.Plan([(nx, ny, m)], dtype="f32")
    table = plan.coeffs(0, [se2.GaussVM(s, k, th) for s, k, th in chain])
    out = _run(plan, 0, f, table, torch.float32)
    ref_t = oracle_table_gauss(nx, ny, m, chain)
    tol = tol32(nx * ny * m)
    for b in range(16):
        err = parity_err(out[b], oracle_conv(f[b], ref_t))
        print(f"  field {b}: err {err:.2e}", flush=True)
        assert err <= tol
        # mass is multiplicative (discrete normalisation => mean preserved)
        assert abs(out[b].mean() - f[b].mean()) <= 1e-5 * abs(f[b].mean())


def test_headline_256x256x64_batch16_chain8_all_fields():
    case("headline 256x256x64 fp32 batch 16, chain of 8: every field vs oracle, mass on all")
    nx = ny = 256
    m = 64
    ks = chain_kernel_params(2, 8)
    chain = [(k.sigma, k.kappa, 0.0) for k in ks]
    f = _fields(2, 16, 32, nx, ny, m)
    plan = se2.Plan([(nx, ny, m)], dtype="f32")
    table = plan.coeffs(0, [se2.GaussVM(s, k, th) for s, k, th in chain])
    out = _run(plan, 0, f, table, torch.float32)
    ref_t = oracle_table_gauss(nx, ny, m, chain)
    tol = tol32(nx * ny * m)
    for b in range(16):
        err = parity_err(out[b], oracle_conv(f[b], ref_t))
        print(f"  field {b}: err {err:.2e} (tol {tol:.1e})", flush=True)
        assert err <= tol
        assert abs(out[b].mean() - f[b].mean()) <= 1e-5 * abs(f[b].mean())


@pytest.mark.parametrize("nx,ny,m", [(64, 64, 16), (128, 64, 32), (256, 128, 64), (64, 256, 64), (128, 96, 16),
                                     # slab too large for LDS: x rows + y pencils + theta pencils
                                     (512, 64, 64), (128, 64, 256), (64, 64, 512),
                                     # 512-point y pencils after the slab
                                     (64, 512, 64),
                                     # 32-point lines
                                     (32, 32, 16), (32, 64, 64), (64, 32, 32),
                                     # 3 * 2^k lines (mixed-radix register DFTs, 8-column pencils)
                                     (48, 48, 16), (96, 96, 64), (48, 96, 32), (96, 48, 64), (48, 64, 64)])
def test_register_kernels_match_generic_and_oracle(nx, ny, m):
    batch = 3 if nx * ny * m < (1 << 20) else 2
    case(f"register vs generic kernels {nx}x{ny}x{m} fp32 batch {batch}, chain of 3, adjoint too")
    ks = chain_kernel_params(9, 3)
    chain = [(k.sigma, k.kappa, 0.4 * j) for j, k in enumerate(ks)]
    f = _fields(9, batch, 16, nx, ny, m)
    ref_t = oracle_table_gauss(nx, ny, m, chain)
    print("  oracle table done", flush=True)
    outs = {}
    for generic in (False, True):
        plan = se2.Plan([(nx, ny, m)], dtype="f32", generic=generic)
        table = plan.coeffs(0, [se2.GaussVM(s, k, th) for s, k, th in chain])
        fd = _dev(f, torch.float32)
        outs[generic] = (plan.apply(0, fd, table).cpu().numpy().astype(np.float64),
                         plan.apply(0, fd, table, adjoint=True).cpu().numpy().astype(np.float64))
        print(f"  GPU generic={generic} done", flush=True)
    tol = tol32(nx * ny * m)
    for b in range(batch):
        ref = oracle_conv(f[b], ref_t)
        ref_adj = oc.conv_with_coeffs(f[b], np.conj(ref_t))
        for generic in (False, True):
            e1 = parity_err(outs[generic][0][b], ref)
            e2 = parity_err(outs[generic][1][b], ref_adj)
            print(f"  field {b} generic={generic}: {e1:.2e} adj {e2:.2e}", flush=True)
            assert e1 <= tol and e2 <= tol


# ---------------------------------------------------------------- full path
@pytest.mark.parametrize("dt,batch", [("f32", 1), ("f32", 2), ("f32", 3), ("f64", 3), ("f64", 2)])
def test_full_path_parity(dt, batch, rng):
    case(f"full-table path 32x48x16 {dt} batch={batch}")
    nx, ny, m = 32, 48, 16
    prof = rng.uniform(0, 1, size=(12, m))
    p_prof = ok.radial_profile(nx, ny, m, prof, 0.4)
    plan = se2.Plan([(nx, ny, m)], dtype=dt)
    table = plan.coeffs(0, [se2.RadialProfile(_dev(prof, torch.float64), 0.4, norm=2),
                            se2.GaussVM(0.05, 3.0, 0.7)])
    f = _fields(3, batch, 8, nx, ny, m)
    tdt = torch.float32 if dt == "f32" else torch.float64
    out = _run(plan, 0, f, table, tdt)
    ref_t = ffc(p_prof) * ffc(ok.gauss_vm(nx, ny, m, 0.05, 3.0, 0.7))
    tol = tol32(nx * ny * m) if dt == "f32" else TOL64
    for b in range(batch):
        err = parity_err(out[b], oracle_conv(f[b], ref_t))
        print(f"  field {b}: rel-L2 {err:.2e}", flush=True)
        assert err <= tol


@pytest.mark.parametrize("nx,ny,m,batch", [(64, 64, 16, 3), (128, 64, 32, 2), (256, 128, 64, 3), (64, 512, 64, 1),
                                           (256, 256, 64, 2), (32, 32, 64, 3), (32, 64, 16, 2)])
def test_full_path_register_kernels(nx, ny, m, batch, rng):
    case(f"full-table register kernels {nx}x{ny}x{m} fp32 batch={batch}: profile x Gauss-vM chain, adjoint, "
         "generic kernels and oracle")
    prof = rng.uniform(0, 1, size=(16, m))
    p_prof = ok.radial_profile(nx, ny, m, prof, 0.45)
    f = _fields(5, batch, 8, nx, ny, m)
    outs = {}
    for generic in (False, True):
        plan = se2.Plan([(nx, ny, m)], dtype="f32", generic=generic)
        table = plan.coeffs(0, [se2.RadialProfile(_dev(prof, torch.float64), 0.45, norm=2),
                                se2.GaussVM(0.05, 3.0, 0.7)])
        fd = _dev(f, torch.float32)
        outs[generic] = (plan.apply(0, fd, table).cpu().numpy().astype(np.float64),
                         plan.apply(0, fd, table, adjoint=True).cpu().numpy().astype(np.float64))
        print(f"  GPU generic={generic} done", flush=True)
    ref_t = ffc(p_prof) * ffc(ok.gauss_vm(nx, ny, m, 0.05, 3.0, 0.7))
    print("  oracle table done", flush=True)
    tol = tol32(nx * ny * m)
    for b in range(batch):
        ref = oracle_conv(f[b], ref_t)
        ref_adj = oc.conv_with_coeffs(f[b], np.conj(ref_t))
        for generic in (False, True):
            e1 = parity_err(outs[generic][0][b], ref)
            e2 = parity_err(outs[generic][1][b], ref_adj)
            print(f"  field {b} generic={generic}: {e1:.2e} adj {e2:.2e}", flush=True)
            assert e1 <= tol and e2 <= tol


def test_full_path_large_three_pass_fp64():
    case("full-table path 256x16x64 fp64 (split x / theta passes)")
    nx, ny, m = 256, 16, 64
    p = ok.gauss_vm(nx, ny, m, 0.06, 4.0, 0.2, normalize=None)
    plan = se2.Plan([(nx, ny, m)], dtype="f64")
    table = plan.coeffs(0, [se2.Samples(_dev(p, torch.float64), norm=2)])
    f = _fields(4, 3, 8, nx, ny, m)
    out = _run(plan, 0, f, table, torch.float64)
    ref_t = ffc(p)
    for b in range(3):
        err = parity_err(out[b], oracle_conv(f[b], ref_t))
        print(f"  field {b}: rel-L2 {err:.2e}", flush=True)
        assert err <= TOL64


# ------------------------------------------------------- adjoint, in place
@pytest.mark.parametrize("kind", ["sep", "full"])
def test_adjoint_matches_oracle(kind):
    case(f"adjoint {kind} 32x32x16 fp64")
    nx = ny = 32
    m = 16
    plan = se2.Plan([(nx, ny, m)], dtype="f64")
    if kind == "sep":
        table = plan.coeffs(0, [se2.GaussVM(0.06, 3.0, 1.2)])
        p = ok.gauss_vm(nx, ny, m, 0.06, 3.0, 1.2)
    else:
        p = ok.gauss_vm(nx, ny, m, 0.06, 3.0, 1.2)
        table = plan.coeffs(0, [se2.Samples(_dev(p, torch.float64))])
    g = _fields(5, 2, 8, nx, ny, m)
    out = plan.apply(0, _dev(g, torch.float64), table, adjoint=True).cpu().numpy()
    for b in range(2):
        ref = oc.conv_chain(g[b], [p], adjoint=True)
        assert parity_err(out[b], ref) <= TOL64


def test_in_place_operation():
    case("in place out == f, 64x64x32 fp32")
    nx = ny = 64
    m = 32
    plan = se2.Plan([(nx, ny, m)], dtype="f32")
    table = plan.coeffs(0, [se2.GaussVM(0.05, 4.0)])
    f = _fields(6, 2, 8, nx, ny, m)
    fd = _dev(f, torch.float32)
    plan.apply(0, fd, table, out=fd)
    out = fd.cpu().numpy().astype(np.float64)
    ref_t = oracle_table_gauss(nx, ny, m, [(0.05, 4.0, 0.0)])
    for b in range(2):
        assert parity_err(out[b], oracle_conv(f[b], ref_t)) <= tol32(nx * ny * m)


# --------------------------------------------- chain API, graphs, many problems
def test_chain_runtime_product_and_graph_replay():
    case("se2conv_chain: heterogeneous problems, runtime table products, graph replays")
    shapes = [(32, 32, 16), (48, 48, 32), (64, 32, 16)]
    plan = se2.Plan(shapes, dtype="f32")
    probs, refs = [], []
    for i, (nx, ny, m) in enumerate(shapes):
        k1, k2 = (0.04 + 0.01 * i, 3.0, 0.0), (0.07, 8.0 - i, 0.5)
        t1 = plan.coeffs(i, [se2.GaussVM(*k1)])
        t2 = plan.coeffs(i, [se2.GaussVM(*k2)])
        f = _fields(7 + i, 2, 8, nx, ny, m)
        fd = _dev(f, torch.float32)
        out = torch.empty_like(fd)
        probs.append((i, fd, out, [t1, t2]))
        ref_t = oracle_table_gauss(nx, ny, m, [k1, k2])
        refs.append([oracle_conv(f[b], ref_t) for b in range(2)])
    stream = torch.cuda.Stream()  # graph capture needs a created stream
    torch.cuda.synchronize()
    plan.chain(probs, stream=stream)
    torch.cuda.synchronize()
    eager = [p[2].clone() for p in probs]
    for (i, _, out, _), ref in zip(probs, refs):
        nx, ny, m = shapes[i]
        o = out.cpu().numpy().astype(np.float64)
        for b in range(2):
            assert parity_err(o[b], ref[b]) <= tol32(nx * ny * m)
    for rep in range(4):
        for _, _, out, _ in probs:
            out.zero_()
        torch.cuda.synchronize()
        plan.chain(probs, graph=True, stream=stream)
        torch.cuda.synchronize()
        _ = torch.ones(1024, device=DEV).sum().item()  # unrelated eager work between replays
        for e, (_, _, out, _) in zip(eager, probs):
            assert torch.equal(e, out), f"graph replay {rep} differs from eager"


def test_timing_hook_reports_each_pass():
    case("pass timing hook 64x64x32 fp32")
    plan = se2.Plan([(64, 64, 32)], dtype="f32")
    table = plan.coeffs(0, [se2.GaussVM(0.05, 4.0)])
    f = _dev(_fields(8, 2, 8, 64, 64, 32), torch.float32)
    for _ in range(3):
        plan.apply(0, f, table, timing=True)
    times = plan.pass_times()
    assert [k for k, _ in times] == ["xt_slab", "y_pencil"] * 3
    assert all(t > 0 for _, t in times)


def test_graph_on_null_stream_is_rejected():
    case("graph capture on the null stream rejected")
    plan = se2.Plan([(32, 32, 16)], dtype="f32")
    t = plan.coeffs(0, [se2.GaussVM(0.05, 4.0)])
    f = torch.zeros(1, 16, 32, 32, device=DEV)
    with pytest.raises(se2.Se2convError) as e:
        plan.chain([(0, f, f, [t])], graph=True, stream=torch.cuda.default_stream())
    assert e.value.status == 1
    plan.apply(0, f, t)  # the plan and device are still usable
    torch.cuda.synchronize()


def test_foreign_table_is_rejected():
    case("foreign table rejected")
    p1 = se2.Plan([(32, 32, 16)], dtype="f32")
    p2 = se2.Plan([(32, 32, 16)], dtype="f32")
    t1 = p1.coeffs(0, [se2.GaussVM(0.05, 4.0)])
    f = torch.zeros(1, 16, 32, 32, device=DEV)
    with pytest.raises(se2.Se2convError) as e:
        p2.apply(0, f, t1)
    assert e.value.status == 1


# ------------------------------------------------------- Algorithm 7 (powers)
@pytest.mark.parametrize("nx,ny,m,batch,q,dt,kind", [
    (32, 24, 16, 3, 4, "f64", "sep"),
    (32, 32, 16, 2, 3, "f32", "full"),
    (64, 64, 32, 1, 5, "f32", "sep"),
    (48, 32, 24, 2, 2, "f64", "full"),
    # even FP32 batches on register-kernel shapes: one y pass for every power
    (64, 64, 32, 2, 5, "f32", "sep"),
    (128, 64, 64, 4, 3, "f32", "full"),
    (32, 512, 16, 2, 2, "f32", "full"),
])
def test_all_powers_match_oracle_alg7(nx, ny, m, batch, q, dt, kind, rng):
    case(f"Algorithm 7 powers {nx}x{ny}x{m} {dt} batch={batch} q={q} {kind} table")
    plan = se2.Plan([(nx, ny, m)], dtype=dt)
    tdt = torch.float32 if dt == "f32" else torch.float64
    if kind == "sep":
        p = ok.gauss_vm(nx, ny, m, 0.06, 3.0, 0.5)
        table = plan.coeffs(0, [se2.GaussVM(0.06, 3.0, 0.5)])
    else:
        prof = rng.uniform(0, 1, size=(10, m))
        p = ok.radial_profile(nx, ny, m, prof, 0.4)
        p = p / p.mean()
        table = plan.coeffs(0, [se2.RadialProfile(_dev(prof, torch.float64), 0.4, norm=0)])
    f = _fields(11, batch, 8, nx, ny, m)
    out = plan.powers(0, _dev(f, tdt), table, q).cpu().numpy().astype(np.float64)
    adj = plan.powers(0, _dev(f, tdt), table, q, adjoint=True).cpu().numpy().astype(np.float64)
    tol = tol32(nx * ny * m) if dt == "f32" else TOL64
    for b in range(batch):
        refs = oc.alg7_all_powers(f[b], p, q)
        for k in range(q):
            err = parity_err(out[k, b], refs[k])
            print(f"  field {b} power {k + 1}: {err:.2e}", flush=True)
            assert err <= tol
        # the adjoint power p is the correlation with rho p times (conjugated coefficients)
        ref_adj = f[b]
        for k in range(q):
            ref_adj = oc.conv_chain(ref_adj, [p], adjoint=True)
            assert parity_err(adj[k, b], ref_adj) <= tol, (b, k)


# ------------------------------------------------------------ field sampling
@pytest.mark.parametrize("dt,shape,nb", [("f64", (32, 48, 16), 8), ("f32", (256, 256, 64), 32), ("f64", (96, 64, 24), 5)])
def test_gpu_sampler_matches_generator(dt, shape, nb):
    from inputs import bump_field
    case(f"GPU bump sampler {shape} {dt} {nb} bumps")
    nx, ny, m = shape
    bf = bump_field(12, 3, nb)
    plan = se2.Plan([shape], dtype=dt)
    out = plan.sample_bumps(0, bf.centres, bf.theta0, bf.weights, bf.s, bf.kappa).cpu().numpy()
    ref = sample_field(bf, nx, ny, m)
    err = np.max(np.abs(out - ref)) / np.max(np.abs(ref))
    assert err <= (1e-14 if dt == "f64" else 1e-6), err


def test_autotuned_schedules_stay_correct(tmp_path, monkeypatch):
    case("autotune: 48x48x32 (generic), 64x64x16 (register kernels), 512x16x64 (three-pass); results vs oracle")
    monkeypatch.setenv("SE2CONV_TUNE_CACHE", str(tmp_path / "tune.jsonl"))
    shapes = [(48, 48, 32), (64, 64, 16), (512, 16, 64)]
    plan = se2.Plan(shapes, dtype="f32")
    for i in range(len(shapes)):
        plan.autotune(i, batch=2)
    lines = (tmp_path / "tune.jsonl").read_text().strip().splitlines()
    assert len(lines) == 3
    for i, (nx, ny, m) in enumerate(shapes):
        chain = [(0.05, 3.0, 0.2), (0.03, 9.0, 0.0)]
        table = plan.coeffs(i, [se2.GaussVM(*k) for k in chain])
        f = _fields(13, 2, 8, nx, ny, m)
        out = plan.apply(i, _dev(f, torch.float32), table).cpu().numpy().astype(np.float64)
        ref_t = oracle_table_gauss(nx, ny, m, chain)
        for b in range(2):
            assert parity_err(out[b], oracle_conv(f[b], ref_t)) <= tol32(nx * ny * m)


@pytest.mark.parametrize("nx,ny,m", [(128, 64, 64), (512, 64, 32), (64, 128, 128), (256, 256, 32), (64, 512, 64)])
def test_fp64_register_kernels_match_generic_and_oracle(nx, ny, m):
    batch = 2 if nx * ny * m >= (1 << 20) else 3
    case(f"FP64 register vs generic kernels {nx}x{ny}x{m} batch {batch}, chain of 2, adjoint too")
    ks = chain_kernel_params(10, 2)
    chain = [(k.sigma, k.kappa, 0.6 * j) for j, k in enumerate(ks)]
    f = _fields(10, batch, 16, nx, ny, m)
    ref_t = oracle_table_gauss(nx, ny, m, chain)
    outs = {}
    for generic in (False, True):
        plan = se2.Plan([(nx, ny, m)], dtype="f64", generic=generic)
        table = plan.coeffs(0, [se2.GaussVM(s, k, th) for s, k, th in chain])
        fd = _dev(f, torch.float64)
        outs[generic] = (plan.apply(0, fd, table).cpu().numpy(), plan.apply(0, fd, table, adjoint=True).cpu().numpy())
        print(f"  GPU generic={generic} done", flush=True)
    for b in range(batch):
        ref = oracle_conv(f[b], ref_t)
        ref_adj = oc.conv_with_coeffs(f[b], np.conj(ref_t))
        for generic in (False, True):
            e1 = parity_err(outs[generic][0][b], ref)
            e2 = parity_err(outs[generic][1][b], ref_adj)
            print(f"  field {b} generic={generic}: {e1:.2e} adj {e2:.2e}", flush=True)
            assert e1 <= TOL64 and e2 <= TOL64
