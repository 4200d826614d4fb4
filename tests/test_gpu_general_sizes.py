"""GPU parity on general grid sizes: the paper's odd grids L = 2K+1 (Sec. 3.2) and
lengths with prime factors above 3 (radix-5/7 codelets, Rader's algorithm for prime
lengths above 7, direct-summation stages for other prime factors).

Same bars as the other parity tests: FP32 rel-L2 <= 2e-6 log2(N^2 M), FP64 <= 1e-12,
against the FP64 oracle (signed frequencies, |k| <= K on odd axes).
"""
import numpy as np
import pytest
import torch

import paper_2504_05149_amd as se2
from gpu_common import TOL64, case, oracle_table_gauss, parity_err, tol32
from inputs import chain_kernel_params, sample_fields
from oracle import adjoint as OA
from oracle import conv as oc
from oracle import kernels as ok
from oracle.ffc import ffc

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def _dev(a, dtype):
    return torch.from_numpy(np.ascontiguousarray(a)).to(device=DEV, dtype=dtype)


def _tdt(dt):
    return torch.float32 if dt == "f32" else torch.float64


def _tol(dt, n):
    return tol32(n) if dt == "f32" else TOL64


GENERAL_CASES = [
    # (nx, ny, m, batch, chain length, dtype)
    (31, 31, 31, 3, 2, "f32"),     # odd prime grid (direct stages)
    (33, 41, 43, 2, 1, "f32"),     # 3 * 11, primes 41 and 43
    (45, 35, 49, 2, 3, "f32"),     # radix-5 and radix-7 codelets
    (101, 53, 17, 1, 2, "f64"),    # primes
    (40, 50, 35, 3, 2, "f32"),     # even x and y, non-2^a 3^b: separable pair passes on the odd kernels
    (40, 50, 35, 2, 2, "f64"),
    (121, 27, 20, 1, 1, "f32"),    # 11^2
    (101, 24, 101, 1, 2, "f32"),   # x-theta slab above the 512-thread tile: split x / theta passes
    (61, 61, 61, 2, 4, "f64"),
]


@pytest.mark.parametrize("nx,ny,m,batch,lc,dt", GENERAL_CASES)
def test_general_size_separable_chain(nx, ny, m, batch, lc, dt):
    case(f"general size {nx}x{ny}x{m} batch={batch} chain={lc} {dt}")
    ks = chain_kernel_params(5, lc)
    chain = [(k.sigma, k.kappa, 0.3 * j) for j, k in enumerate(ks)]
    f = sample_fields(5, batch, 8, nx, ny, m)
    plan = se2.Plan([(nx, ny, m)], dtype=dt)
    table = plan.coeffs(0, [se2.GaussVM(s, k, th) for s, k, th in chain])
    out = plan.apply(0, _dev(f, _tdt(dt)), table)
    torch.cuda.synchronize()
    out = out.cpu().numpy().astype(np.float64)
    ref_t = oracle_table_gauss(nx, ny, m, chain)
    worst = 0.0
    for b in range(batch):
        worst = max(worst, parity_err(out[b], oc.conv_with_coeffs(f[b], ref_t)))
    print(f"rel-L2 {worst:.2e} (tol {_tol(dt, nx * ny * m):.1e})", flush=True)
    assert worst <= _tol(dt, nx * ny * m)


@pytest.mark.parametrize("nx,ny,m,batch,dt", [(31, 31, 31, 3, "f32"), (45, 35, 49, 1, "f64"), (33, 24, 301, 2, "f32")])
def test_general_size_separable_adjoint(nx, ny, m, batch, dt):
    """The separable schedule on field pairs (odd Nx or Ny) with the conjugated factors: the
    x-theta slab where it fits, x rows and theta pencils where it does not (M = 301)."""
    case(f"general size {nx}x{ny}x{m} batch={batch} {dt}: separable chain of 2, adjoint")
    ks = chain_kernel_params(6, 2)
    chain = [(k.sigma, k.kappa, 0.5 + 0.4 * j) for j, k in enumerate(ks)]
    f = sample_fields(6, batch, 8, nx, ny, m)
    plan = se2.Plan([(nx, ny, m)], dtype=dt)
    table = plan.coeffs(0, [se2.GaussVM(s, k, th) for s, k, th in chain])
    out = plan.apply(0, _dev(f, _tdt(dt)), table, adjoint=True)
    torch.cuda.synchronize()
    out = out.cpu().numpy().astype(np.float64)
    ref_t = np.conj(oracle_table_gauss(nx, ny, m, chain))
    for b in range(batch):
        err = parity_err(out[b], oc.conv_with_coeffs(f[b], ref_t))
        print(f"  field {b}: {err:.2e} (tol {_tol(dt, nx * ny * m):.1e})", flush=True)
        assert err <= _tol(dt, nx * ny * m)
    plan.close()


@pytest.mark.parametrize("nx,ny,m,dt", [(33, 29, 25, "f64"), (45, 35, 21, "f32")])
def test_general_size_tables_match_oracle_ffc(nx, ny, m, dt):
    case(f"tables on odd grid {nx}x{ny}x{m} {dt}: separable and full (samples x profile)")
    plan = se2.Plan([(nx, ny, m)], dtype=dt)
    chain = [(0.07, 3.0, 0.8), (0.04, 11.0, 2.5)]
    t = plan.coeffs(0, [se2.GaussVM(s, k, th) for s, k, th in chain])
    torch.cuda.synchronize()
    v = t.complex_view().cpu().numpy()
    gpu = v[nx + ny:][:, None, None] * v[nx:nx + ny][None, :, None] * v[:nx][None, None, :]
    ref = oracle_table_gauss(nx, ny, m, chain)
    err = np.max(np.abs(gpu - ref)) / np.max(np.abs(ref))
    bar = 1e-13 if dt == "f64" else 1e-6
    print(f"separable table max rel err {err:.2e}", flush=True)
    assert err < bar
    rng = np.random.default_rng([2504_05149, 77])
    prof = rng.uniform(0, 1, size=(9, m))
    t2 = plan.coeffs(0, [se2.RadialProfile(_dev(prof, torch.float64), 0.45, norm=2), se2.GaussVM(0.05, 5.0, 1.0)])
    torch.cuda.synchronize()
    gpu2 = t2.complex_view().cpu().numpy()
    ref2 = ffc(ok.radial_profile(nx, ny, m, prof, 0.45)) * ffc(ok.gauss_vm(nx, ny, m, 0.05, 5.0, 1.0))
    err2 = np.max(np.abs(gpu2 - ref2)) / np.max(np.abs(ref2))
    print(f"full table max rel err {err2:.2e}", flush=True)
    assert err2 < bar


@pytest.mark.parametrize("nx,ny,m,batch,dt", [(33, 35, 25, 3, "f32"), (31, 29, 19, 2, "f64")])
def test_general_size_full_table_apply(nx, ny, m, batch, dt):
    case(f"radial-profile full table on odd grid {nx}x{ny}x{m} batch={batch} {dt}")
    rng = np.random.default_rng([2504_05149, 78])
    prof = rng.uniform(0, 1, size=(12, m))
    plan = se2.Plan([(nx, ny, m)], dtype=dt)
    table = plan.coeffs(0, [se2.RadialProfile(_dev(prof, torch.float64), 0.4)])
    f = sample_fields(6, batch, 8, nx, ny, m)
    out = plan.apply(0, _dev(f, _tdt(dt)), table)
    adj = plan.apply(0, _dev(f, _tdt(dt)), table, adjoint=True)
    torch.cuda.synchronize()
    p = ok.radial_profile(nx, ny, m, prof, 0.4)  # no normalisation (the descriptor's default)
    worst = 0.0
    for b in range(batch):
        worst = max(worst, parity_err(out[b].cpu().numpy().astype(np.float64), oc.conv_chain(f[b], [p])))
        worst = max(worst, parity_err(adj[b].cpu().numpy().astype(np.float64), oc.conv_chain(f[b], [p], adjoint=True)))
    print(f"rel-L2 {worst:.2e}", flush=True)
    assert worst <= _tol(dt, nx * ny * m)


@pytest.mark.parametrize("streams", ["1", "4"])
def test_general_sizes_in_one_chain_submission(streams, monkeypatch):
    # the shape classes in sequence on the caller's stream (default), or forked over four
    # auxiliary streams (SE2CONV_CHAIN_STREAMS, read at each call)
    monkeypatch.setenv("SE2CONV_CHAIN_STREAMS", streams)
    case(f"heterogeneous submission on {streams} stream(s): odd, non-2^a3^b and 2^a3^b shapes, eager and graph")
    shapes = [(31, 31, 31), (32, 32, 16), (40, 50, 35), (45, 35, 49)]
    plan = se2.Plan(shapes, dtype="f32")
    items, host = [], []
    for i, s in enumerate(shapes):
        nx, ny, m = s
        chain = [(k.sigma, k.kappa, 0.2 * j) for j, k in enumerate(chain_kernel_params(7 + i, 1 + i % 3))]
        f = sample_fields(7, 2, 8, nx, ny, m)
        t = plan.coeffs(i, [se2.GaussVM(a, b, c) for a, b, c in chain])
        fd = _dev(f, torch.float32)
        items.append((i, fd, torch.empty_like(fd), [t]))
        host.append((f, chain))
    stream = torch.cuda.Stream()
    torch.cuda.synchronize()
    plan.chain(items, stream=stream)
    torch.cuda.synchronize()
    eager = [it[2].clone() for it in items]
    for rep in range(2):
        for it in items:
            it[2].zero_()
        torch.cuda.synchronize()
        plan.chain(items, graph=True, stream=stream)
        torch.cuda.synchronize()
        for e, it in zip(eager, items):
            assert torch.equal(e, it[2]), f"replay {rep}"
    for (nx, ny, m), (f, chain), e in zip(shapes, host, eager):
        ref_t = oracle_table_gauss(nx, ny, m, chain)
        out = e.cpu().numpy().astype(np.float64)
        err = max(parity_err(out[b], oc.conv_with_coeffs(f[b], ref_t)) for b in range(f.shape[0]))
        print(f"{nx}x{ny}x{m}: rel-L2 {err:.2e}", flush=True)
        assert err <= tol32(nx * ny * m)


@pytest.mark.parametrize("dt", ["f32", "f64"])
def test_general_size_powers_and_gradients(dt):
    nx, ny, m = 33, 27, 25
    case(f"powers (Alg. 7) and field tables on odd grid {nx}x{ny}x{m} {dt}")
    plan = se2.Plan([(nx, ny, m)], dtype=dt)
    chain = [(0.06, 4.0, 0.5)]
    table = plan.coeffs(0, [se2.GaussVM(*chain[0])])
    f = sample_fields(8, 3, 8, nx, ny, m)
    pw = plan.powers(0, _dev(f, _tdt(dt)), table, 3)
    ft = plan.field_coeffs(0, _dev(f, _tdt(dt)))
    torch.cuda.synchronize()
    p = ok.gauss_vm(nx, ny, m, *chain[0])
    tol = _tol(dt, nx * ny * m)
    for q in range(3):
        for b in range(3):
            ref = oc.conv_chain(f[b], [p] * (q + 1))
            err = parity_err(pw[q][b].cpu().numpy().astype(np.float64), ref)
            assert err <= tol, (q, b, err)
    for b in range(3):
        gpu = ft[b].complex_view().cpu().numpy()
        ref = ffc(f[b])
        err = np.linalg.norm(gpu - ref) / np.linalg.norm(ref)
        print(f"field table {b}: rel-L2 {err:.2e}", flush=True)
        assert err <= tol
    g = np.random.default_rng([2504_05149, 79]).standard_normal((3, m, ny, nx))
    kg = plan.kernel_grad(0, _dev(g, _tdt(dt)), ft).cpu().numpy().astype(np.float64)
    ref = sum(OA.grad_kernel_samples(f[b], g[b]) for b in range(3))
    err = parity_err(kg, ref)
    print(f"kernel gradient: rel-L2 {err:.2e}", flush=True)
    assert err <= tol


RADER_CASES = [
    # (nx, ny, m, dtype): prime axes above 7 run by Rader's algorithm on the stages of L - 1
    (11, 13, 17, "f64"),   # smallest: inner lengths 10 = 2*5, 12 = 4*3, 16
    (47, 23, 97, "f32"),   # inner 46 = 2*23 and 22 = 2*11 (direct stages), 96 = 16*2*3
    (509, 16, 8, "f32"),   # largest prime length, along x: inner 508 = 4*127
    (16, 509, 8, "f64"),   # along y
    (40, 34, 37, "f32"),   # even x and y: pair passes with a prime theta axis
    (8, 16, 509, "f32"),   # largest prime length along theta (x rows, then theta pencils)
]


@pytest.mark.parametrize("nx,ny,m,dt", RADER_CASES)
def test_prime_lengths_field_coeffs_and_apply(nx, ny, m, dt):
    case(f"prime lengths (Rader) {nx}x{ny}x{m} {dt}: field coefficients and a chain")
    plan = se2.Plan([(nx, ny, m)], dtype=dt)
    f = sample_fields(11, 2, 8, nx, ny, m)
    fd = _dev(f, _tdt(dt))
    ft = plan.field_coeffs(0, fd)
    chain = [(0.05, 6.0, 0.4), (0.03, 2.0, 1.9)]
    table = plan.coeffs(0, [se2.GaussVM(*c) for c in chain])
    out = plan.apply(0, fd, table)
    adj = plan.apply(0, fd, table, adjoint=True)
    torch.cuda.synchronize()
    tol = _tol(dt, nx * ny * m)
    ref_t = oracle_table_gauss(nx, ny, m, chain)
    for b in range(2):
        gpu = ft[b].complex_view().cpu().numpy()
        ref = ffc(f[b])
        err = np.linalg.norm(gpu - ref) / np.linalg.norm(ref)
        e1 = parity_err(out[b].cpu().numpy().astype(np.float64), oc.conv_with_coeffs(f[b], ref_t))
        e2 = parity_err(adj[b].cpu().numpy().astype(np.float64), oc.conv_with_coeffs(f[b], np.conj(ref_t)))
        print(f"field {b}: coefficients {err:.2e}, apply {e1:.2e}, adjoint {e2:.2e} (tol {tol:.1e})", flush=True)
        assert max(err, e1, e2) <= tol
