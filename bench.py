"""Benchmark of the convolutional finite Fourier series on one MI355X.

Default workload: 256 x 256 x 64 grid (x, y on the unit torus, theta on the
circle), FP32, batch of 16 fields (32 Gaussian x von Mises bumps each), convolved
with a chain of 8 Gaussian x von Mises kernels (sigma ~ U[0.01, 0.1], kappa ~
U[1, 20]) whose coefficients are folded into one table in FP64 by se2conv_coeffs.
A step is one se2conv_apply over the whole batch (every pass of the hot path).

Prints ONE JSON line: conv/s over the timed steps (wall clock), the median step
time over graph replays timed with HIP events, the per-kernel roofline of the
dominant pass (measured live with HIP events on the launch stream) beside the
whole path's, the relative L2 error against the FP64 oracle, the oracle's own CPU
throughput, and a "secondary" object with the plain single-kernel convolution at
the same shape, the uneven batch of 256 problems (one graph), the differentiated
form (forward + gradients), a sum of SE(2)-shifted kernels, the FP64 path at
512x512x128 and the prime length 101, and the chain-expanded rate.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "SE(2) convolutions/sec + HBM GB/s at 256×256×64 fp32, rel L2 err vs FP64 oracle"

WORKLOADS = {
    # name: (nx, ny, m, batch, bumps, chain length, dtype, seed config)
    "headline": (256, 256, 64, 16, 32, 8, "f32", 2),
    "headline_plain": (256, 256, 64, 16, 32, 1, "f32", 2),
    "c1": (128, 128, 64, 16, 32, 8, "f32", 1),
    "c3": (512, 512, 128, 4, 128, 4, "f32", 3),
    "c3_f64": (512, 512, 128, 4, 128, 4, "f64", 3),
    "c0": (32, 32, 32, 1, 8, 1, "f64", 0),
    # the paper's odd grids L = 2K+1: a prime length (direct-summation stages)
    "odd101": (101, 101, 101, 4, 32, 2, "f32", 5),
    "odd101_f64": (101, 101, 101, 4, 32, 2, "f64", 5),
    # exponential-coordinates Gaussian (non-separable radial kernel, FULL table)
    "expgauss": (256, 256, 64, 8, 32, 1, "f32", 2),
}
# workloads whose kernel is not a chain of Gauss-vM kernels: (kind, sigma)
EXP_GAUSS_SIGMA = {"expgauss": 0.05}
SPECIAL = ("c2", "c4", "padded", "powers", "shifted")


def lib_source_hash() -> str:
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2504_05149_amd", "csrc")
    for name in sorted(os.listdir(csrc)):
        with open(os.path.join(csrc, name), "rb") as fh:
            h.update(name.encode())
            h.update(fh.read())
    return h.hexdigest()[:16]


def describe(name):
    nx, ny, m, batch, nb, lc, dt, cfg = WORKLOADS[name]
    kern = (f"exponential-coordinates Gaussian kernel sigma={EXP_GAUSS_SIGMA[name]} (FULL FP64-generated table)"
            if name in EXP_GAUSS_SIGMA else f"chain of {lc} Gauss-vM kernels (folded FP64 table)")
    return {"workload": f"{nx}x{ny}x{m} {dt}, batch {batch} fields of {nb} Gauss-vM bumps, {kern}",
            "grid": [nx, ny, m], "batch": batch, "bumps": nb, "chain": lc, "seed_config": cfg}


def replay_median(fn, reps=100, warm=10):
    """Median and mean milliseconds of one replay of a HIP graph captured from fn(stream),
    timed with HIP events on the replay stream; fn runs once eagerly first (so that every
    lazily created resource exists before capture).  Returns (median, mean, replays)."""
    import torch

    s = torch.cuda.Stream()
    torch.cuda.synchronize()
    fn(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        fn(s)
    torch.cuda.synchronize()
    with torch.cuda.stream(s):
        for _ in range(warm):
            g.replay()
        evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
        for e0, e1 in evs:
            e0.record(s)
            g.replay()
            e1.record(s)
    torch.cuda.synchronize()
    t = np.array([e0.elapsed_time(e1) for e0, e1 in evs])
    return float(np.median(t)), float(np.mean(t)), reps


def run_gpu(name, steps, warmup, tune=True):
    import torch

    import paper_2504_05149_amd as se2
    from inputs import chain_kernel_params, sample_fields

    nx, ny, m, batch, nb, lc, dt, cfg = WORKLOADS[name]
    tdt = torch.float32 if dt == "f32" else torch.float64
    plan = se2.Plan([(nx, ny, m)], dtype=dt)
    # schedule knobs chosen by the library's autotuner (outside the timed region)
    t_tune = time.perf_counter()
    if tune:
        plan.autotune(0, batch=batch)
    t_tune = time.perf_counter() - t_tune
    ks = chain_kernel_params(cfg, lc)
    if name in EXP_GAUSS_SIGMA:
        ks = None
        table = plan.coeffs(0, [se2.ExpGauss(EXP_GAUSS_SIGMA[name])])
    else:
        table = plan.coeffs(0, [se2.GaussVM(k.sigma, k.kappa, k.theta0) for k in ks])
    f_host = sample_fields(cfg, batch, nb, nx, ny, m, dtype=np.float32 if dt == "f32" else np.float64)
    f = torch.from_numpy(f_host).to("cuda")
    out = torch.empty_like(f)
    stream = torch.cuda.current_stream()
    torch.cuda.synchronize()
    for _ in range(warmup):
        plan.apply(0, f, table, out=out, stream=stream)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        plan.apply(0, f, table, out=out, stream=stream)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0

    # the same step captured in a HIP graph: median of event-timed replays
    ref = out.clone()
    med_ms, mean_ms, reps = replay_median(lambda st: plan.apply(0, f, table, out=out, stream=st))
    replay_identical = bool(torch.equal(ref, out))

    # per-pass durations with HIP events recorded by the library on this stream
    for _ in range(steps):
        plan.apply(0, f, table, out=out, stream=stream, timing=True)
    times = plan.pass_times()
    per_kind = {}
    for kind, ms in times:
        per_kind.setdefault(kind, []).append(ms)
    avg = {k: float(np.mean(v)) for k, v in per_kind.items()}
    launches = {k: len(v) / steps for k, v in per_kind.items()}
    out_host = out.cpu().numpy()
    plan.close()
    return dict(elapsed=elapsed, avg_ms=avg, launches=launches, f_host=f_host, out_host=out_host, ks=ks,
                shape=(nx, ny, m), batch=batch, dtype=dt, tune_s=t_tune if tune else None, name=name,
                replay_median_ms=med_ms, replay_mean_ms=mean_ms, replays=reps, replay_identical=replay_identical)


def run_c2(steps, warmup, cpu_budget=None):
    """256 independent problems (mixed N, M, chain lengths) replayed as one HIP graph."""
    import torch

    import paper_2504_05149_amd as se2
    from inputs import sample_field, uneven_problem_list

    probs = uneven_problem_list(2, 256)
    shapes = sorted({(p["n"], p["n"], p["m"]) for p in probs})
    sidx = {s: i for i, s in enumerate(shapes)}
    plan = se2.Plan(shapes, dtype="f32")
    # one schedule per size class, chosen by timing (se2conv_autotune)
    counts = {s: sum(1 for p in probs if (p["n"], p["n"], p["m"]) == s) for s in shapes}
    t_tune = time.perf_counter()
    for sh in shapes:
        plan.autotune(sidx[sh], batch=counts[sh])
    t_tune = time.perf_counter() - t_tune
    items, npts = [], 0
    for p in probs:
        sh = (p["n"], p["n"], p["m"])
        table = plan.coeffs(sidx[sh], [se2.GaussVM(k.sigma, k.kappa, k.theta0) for k in p["chain"]])
        f = torch.from_numpy(sample_field(p["field"], *sh, dtype=np.float32)[None]).to("cuda")
        items.append((sidx[sh], f, torch.empty_like(f), [table]))
        npts += f.numel()
    stream = torch.cuda.Stream()
    sub = plan.chain_submission(items, graph=True)  # marshalled once, replayed as a graph
    torch.cuda.synchronize()
    for _ in range(max(1, warmup)):
        sub.run(stream)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        sub.run(stream)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    ms = el * 1e3 / steps
    # device time of one submission: the eager submission captured in a graph, replays
    # timed with HIP events
    med_ms, mean_ms, reps = replay_median(lambda st: plan.chain(items, stream=st))
    line_cpu = {}
    if cpu_budget:
        # the FP64 oracle (route 1) problem by problem in list order, within the budget, and
        # each of those problems' GPU output against it
        from threadpoolctl import threadpool_info

        from inputs import rel_l2
        from oracle import conv as oc
        from oracle import kernels as ok

        torch.cuda.synchronize()
        done, errs = 0, []
        t0 = time.perf_counter()
        for p, (si, f, o, _) in zip(probs, items):
            n_, m_ = p["n"], p["m"]
            table = oc.coeff_product([ok.gauss_vm(n_, n_, m_, k.sigma, k.kappa, k.theta0) for k in p["chain"]])
            ref = oc.conv_with_coeffs(f[0].cpu().numpy().astype(np.float64), table)
            errs.append(rel_l2(o[0].cpu().numpy().astype(np.float64), ref))
            done += 1
            if time.perf_counter() - t0 > cpu_budget:
                break
        el = time.perf_counter() - t0
        threads = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
        line_cpu = {"cpu_baseline": {"value": done / el, "unit": "conv/s", "cores": int(threads), "kind": "oracle",
                                     "sample": f"the first {done} of 256 problems in list order, FP64 route 1 "
                                               f"(chain table built per problem, included); {el:.1f} s; {host_cpu()}"},
                    "rel_l2_vs_oracle": float(max(errs)), "rel_l2_tol": 2e-6 * float(np.log2(128 * 128 * 64))}
    return {"metric": "SE(2) convolutions/sec, 256 uneven problems in one graph", "value": round(256 / (ms * 1e-3), 1),
            "unit": "conv/s", "n_gpus": 1, "steps": steps, "warmup": warmup, "ms_per_step": round(ms, 4),
            "higher_is_better": True, "dtype": "f32", "data": "synthetic",
            "config": {"workload": "256 problems, N in {32,48,64,96,128}, M in {16,32,64}, chains of 1..4 "
                                   "Gauss-vM kernels, 8 bumps per field", "shape_classes": len(shapes),
                       "points": npts},
            "path_alg_GBps": round(8 * npts / (ms * 1e-3) / 1e9, 1), "autotune_s": round(t_tune, 2),
            "replay_median_ms": round(med_ms, 4), "replay_mean_ms": round(mean_ms, 4), "replays": reps,
            "conv_per_s_replay_median": round(256 / (med_ms * 1e-3), 1),
            "replay_alg_GBps": round(8 * npts / (med_ms * 1e-3) / 1e9, 1), **line_cpu}


def run_padded(steps, warmup, cpu_budget=None):
    """S_K evaluated on a grid twice as fine (zero-padded inverse): 128x128x32 -> 256x256x64 FP32."""
    import torch

    import paper_2504_05149_amd as se2
    from inputs import chain_kernel_params, sample_fields

    L, N, batch, lc = (128, 128, 32), (256, 256, 64), 8, 4
    plan = se2.Plan([L, N], dtype="f32")
    ks = chain_kernel_params(9, lc)
    table = plan.coeffs(0, [se2.GaussVM(k.sigma, k.kappa, k.theta0) for k in ks])
    f_host = sample_fields(9, batch, 32, *L, dtype=np.float32)
    f = torch.from_numpy(f_host).to("cuda")
    out = torch.empty((batch, N[2], N[1], N[0]), dtype=torch.float32, device="cuda")
    for _ in range(warmup):
        plan.apply_padded(0, f, table, 1, out=out)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        plan.apply_padded(0, f, table, 1, out=out)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    for _ in range(steps):
        plan.apply_padded(0, f, table, 1, out=out, timing=True)
    per_kind = {}
    for kind, t in plan.pass_times():
        per_kind.setdefault(kind, []).append(t)
    out_host = out.cpu().numpy()
    plan.close()
    nl, nn = L[0] * L[1] * L[2], N[0] * N[1] * N[2]
    alg = 4 * (nl + nn) * batch  # read the samples, write the finer-grid values
    gbps = alg / (ms * 1e-3) / 1e9
    line = {"metric": "SE(2) convolutions/sec evaluated on a 2x finer grid (zero-padded inverse)",
            "value": round(batch / (ms * 1e-3), 1), "unit": "conv/s", "n_gpus": 1, "steps": steps,
            "warmup": warmup, "ms_per_step": round(ms, 4), "higher_is_better": True, "dtype": "f32",
            "data": "synthetic",
            "config": {"workload": f"{L[0]}x{L[1]}x{L[2]} -> {N[0]}x{N[1]}x{N[2]} fp32, batch {batch} fields of "
                                   f"32 Gauss-vM bumps, chain of {lc} Gauss-vM kernels"},
            "pass_ms_total_per_step": {k: round(float(np.sum(v)) / steps, 4) for k, v in per_kind.items()},
            "roofline": {"bound": "hbm", "kernel": "whole path", "achieved": round(gbps, 1), "peak": HBM_PEAK_GBS,
                         "unit": "GB/s", "frac": round(gbps / HBM_PEAK_GBS, 4), "traffic": None,
                         "alg_bytes_per_step": alg}}
    if cpu_budget is not None:
        cb, errs = cpu_baseline_padded(f_host, out_host, ks, L, N, cpu_budget)
        line["cpu_baseline"] = cb
        line["rel_l2_vs_oracle"] = float(max(errs))
        line["rel_l2_tol"] = float(2e-6 * np.log2(nn))
    return line


def cpu_baseline_padded(f_host, out_host, ks, L, N, budget_s):
    """The FP64 oracle's finer-grid evaluation (synthesis at the finer points) on a bounded sample."""
    from threadpoolctl import threadpool_info

    from inputs import rel_l2
    from oracle import conv as oc
    from oracle import kernels as ok

    ps = [ok.gauss_vm(*L, k.sigma, k.kappa, k.theta0) for k in ks]
    done, errs = 0, []
    t0 = time.perf_counter()
    while done < f_host.shape[0]:
        ref = oc.conv_on_grid(f_host[done].astype(np.float64), ps, N)
        errs.append(rel_l2(out_host[done].astype(np.float64), ref))
        done += 1
        if time.perf_counter() - t0 > budget_s:
            break
    el = time.perf_counter() - t0
    threads = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
    return {"value": done / el, "unit": "conv/s", "cores": int(threads), "kind": "oracle",
            "sample": f"{done} of {f_host.shape[0]} fields, FP64 route 1 with synthesis on the finer grid; "
                      f"{el:.1f} s; {host_cpu()}"}, errs


def run_powers(steps, warmup, cpu_budget=None):
    """All powers V_p = f * rho^(p), p = 1..4 (Alg. 7: one forward transform, running product,
    q inverses) with the exponential-coordinates Gaussian, 256x256x64 FP32, batch 8."""
    import torch

    import paper_2504_05149_amd as se2
    from inputs import sample_fields

    shape, batch, q, sigma = (256, 256, 64), 8, 4, 0.04
    plan = se2.Plan([shape], dtype="f32")
    table = plan.coeffs(0, [se2.ExpGauss(sigma)])
    f_host = sample_fields(2, batch, 32, *shape, dtype=np.float32)
    f = torch.from_numpy(f_host).to("cuda")
    out = None
    for _ in range(warmup):
        out = plan.powers(0, f, table, q)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        out = plan.powers(0, f, table, q)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    out_host = out[:, 0].cpu().numpy()
    plan.close()
    n = shape[0] * shape[1] * shape[2]
    alg = 4 * n * batch * (1 + q)  # read the fields once, write q outputs
    gbps = alg / (ms * 1e-3) / 1e9
    line = {"metric": "SE(2) convolutions/sec, all powers f * rho^(p), p = 1..4 (Alg. 7)",
            "value": round(batch * q / (ms * 1e-3), 1), "unit": "conv/s", "n_gpus": 1, "steps": steps,
            "warmup": warmup, "ms_per_step": round(ms, 4), "higher_is_better": True, "dtype": "f32",
            "data": "synthetic",
            "config": {"workload": f"{shape[0]}x{shape[1]}x{shape[2]} fp32, batch {batch} fields of 32 Gauss-vM "
                                   f"bumps, exponential-coordinates Gaussian sigma={sigma}, q={q} (one output per power)"},
            "roofline": {"bound": "hbm", "kernel": "whole path", "achieved": round(gbps, 1), "peak": HBM_PEAK_GBS,
                         "unit": "GB/s", "frac": round(gbps / HBM_PEAK_GBS, 4), "traffic": None,
                         "alg_bytes_per_step": alg}}
    if cpu_budget is not None:
        from threadpoolctl import threadpool_info

        from inputs import rel_l2
        from oracle import conv as oc
        from oracle import kernels as ok

        p = ok.sample_function(ok.exp_gauss_function(sigma), *shape, images=3)
        t0 = time.perf_counter()
        ref = oc.alg7_all_powers(f_host[0].astype(np.float64), p / p.mean(), q)
        el = time.perf_counter() - t0
        errs = [rel_l2(out_host[k].astype(np.float64), ref[k]) for k in range(q)]
        threads = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
        line["cpu_baseline"] = {"value": q / el, "unit": "conv/s", "cores": int(threads), "kind": "oracle",
                                "sample": f"field 0, all {q} powers by the oracle's Alg. 7 (FP64); {el:.1f} s; "
                                          f"{host_cpu()}"}
        line["rel_l2_vs_oracle"] = float(max(errs))
        line["rel_l2_tol"] = float(2e-6 * np.log2(n))
    return line


def shifted_params(m, n_terms=8, rolls=(0, 5)):
    """Seeded shifts (tx, ty, roll, weight) of the shifted-kernel workload."""
    rng = np.random.default_rng([2504_05149, 6, 2000])
    return [(float(rng.uniform(-0.3, 0.3)), float(rng.uniform(-0.3, 0.3)), int(rolls[k % len(rolls)]),
             float(rng.uniform(-1.0, 1.0))) for k in range(n_terms)]


def run_shifted(steps, warmup, cpu_budget=None):
    """Sums of SE(2)-shifted radial kernels: 8 shifts of a Gauss-vM kernel (sigma 0.04, kappa 6)
    in two theta rolls, 256x256x64 FP32, batch 8 (se2conv_apply_shifted, five passes)."""
    import torch

    import paper_2504_05149_amd as se2
    from inputs import sample_fields

    shape, batch = (256, 256, 64), 8
    shifts = shifted_params(shape[2])
    plan = se2.Plan([shape], dtype="f32")
    q = plan.shift_table(0, shifts)
    rho = plan.coeffs(0, [se2.GaussVM(0.04, 6.0, 0.0)])
    f_host = sample_fields(6, batch, 32, *shape, dtype=np.float32)
    f = torch.from_numpy(f_host).to("cuda")
    out = torch.empty_like(f)
    for _ in range(warmup):
        plan.apply_shifted(0, f, q, [rho], out=out)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        plan.apply_shifted(0, f, q, [rho], out=out)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    med_ms, _, reps = replay_median(lambda st: plan.apply_shifted(0, f, q, [rho], out=out, stream=st))
    for _ in range(steps):
        plan.apply_shifted(0, f, q, [rho], out=out, timing=True)
    per_kind = {}
    for kind, t in plan.pass_times():
        per_kind.setdefault(kind, []).append(t)
    out_host = out.cpu().numpy()
    plan.close()
    n = shape[0] * shape[1] * shape[2]
    alg = 8 * n * batch
    gbps = alg / (med_ms * 1e-3) / 1e9
    line = {"metric": "SE(2) convolutions/sec with a sum of 8 SE(2)-shifted Gauss-vM kernels",
            "value": round(batch / (ms * 1e-3), 1), "unit": "conv/s", "n_gpus": 1, "steps": steps,
            "warmup": warmup, "ms_per_step": round(ms, 4), "replay_median_ms": round(med_ms, 4), "replays": reps,
            "higher_is_better": True, "dtype": "f32", "data": "synthetic",
            "config": {"workload": f"{shape[0]}x{shape[1]}x{shape[2]} fp32, batch {batch} fields of 32 Gauss-vM bumps, "
                                   "kernel = sum of 8 SE(2)-shifts (translations U[-0.3,0.3]^2, theta rolls 0 and 5 "
                                   "grid angles, weights U[-1,1]) of a Gauss-vM kernel sigma=0.04 kappa=6"},
            "pass_ms_total_per_step": {k: round(float(np.sum(v)) / steps, 4) for k, v in per_kind.items()},
            "roofline": {"bound": "hbm", "kernel": "whole path", "achieved": round(gbps, 1), "peak": HBM_PEAK_GBS,
                         "unit": "GB/s", "frac": round(gbps / HBM_PEAK_GBS, 4), "traffic": None,
                         "alg_bytes_per_step": alg}}
    if cpu_budget is not None:
        from threadpoolctl import threadpool_info

        from inputs import rel_l2
        from oracle import kernels as ok
        from oracle import shifted as osh

        p = ok.gauss_vm(*shape, 0.04, 6.0, 0.0)
        sh = [(tx, ty, 2 * np.pi * r / shape[2]) for tx, ty, r, _ in shifts]
        w = [a for *_, a in shifts]
        done, errs = 0, []
        t0 = time.perf_counter()
        while done < batch:
            ref = osh.shifted_sum_conv(f_host[done].astype(np.float64), p, sh, w)
            errs.append(rel_l2(out_host[done].astype(np.float64), ref))
            done += 1
            if time.perf_counter() - t0 > cpu_budget:
                break
        el = time.perf_counter() - t0
        threads = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
        line["cpu_baseline"] = {"value": done / el, "unit": "conv/s", "cores": int(threads), "kind": "oracle",
                                "sample": f"{done} of {batch} fields, FP64 oracle (spatial FFCs per slice, shift "
                                          f"phases, theta FFC, product, dense synthesis); {el:.1f} s; {host_cpu()}"}
        line["rel_l2_vs_oracle"] = float(max(errs))
        line["rel_l2_tol"] = float(2e-6 * np.log2(n))
    return line


def run_c4(steps, warmup, cpu_budget=None):
    """Loss + gradients w.r.t. the field and a 64 x 64 radial profile, 256x256x64 FP32 batch 8."""
    import torch

    import paper_2504_05149_amd as se2
    from inputs import sample_fields
    from paper_2504_05149_amd.autograd import radial_profile_conv

    nx = ny = 256
    m, batch, nk, rmax = 64, 8, 64, 0.5
    plan = se2.Plan([(nx, ny, m)], dtype="f32")
    f = torch.from_numpy(sample_fields(4, batch, 32, nx, ny, m, dtype=np.float32)).to("cuda")
    # target: sigma* = 0.04, kappa* = 8 convolution (on the GPU) plus 1% noise
    tt = plan.coeffs(0, [se2.GaussVM(0.04, 8.0, 0.0)])
    clean = plan.apply(0, f, tt)
    gen = torch.Generator(device="cuda").manual_seed(2504_05149)
    target = clean + 0.01 * clean.pow(2).mean().sqrt() * torch.randn(clean.shape, device="cuda", generator=gen)
    r = torch.arange(nk, dtype=torch.float64) * rmax / (nk - 1)
    th = 2 * np.pi * torch.arange(m, dtype=torch.float64) / m
    prof = (torch.exp(-r[:, None] ** 2 / (2 * 0.06 ** 2)) * torch.exp(4.0 * (torch.cos(th)[None, :] - 1.0))).cuda()
    res, med = {}, {}
    for ck in (True, False):
        def step():
            fd = f.detach().requires_grad_(True)
            pd = prof.detach().requires_grad_(True)
            out = radial_profile_conv(fd, pd, plan, 0, rmax, checkpoint=ck)
            # ||out - target||^2 (sum over batch and grid), one fused kernel each way
            loss = torch.nn.functional.mse_loss(out, target, reduction="sum")
            loss.backward()
            return loss
        for _ in range(warmup):
            step()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            step()
        torch.cuda.synchronize()
        res["checkpoint" if ck else "recompute"] = (time.perf_counter() - t0) * 1e3 / steps
        # HIP events around each step on the current stream (autograd runs there)
        evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
        for e0, e1 in evs:
            e0.record()
            step()
            e1.record()
        torch.cuda.synchronize()
        med["checkpoint" if ck else "recompute"] = float(np.median([e0.elapsed_time(e1) for e0, e1 in evs]))
    line_cpu = {}
    if cpu_budget:
        # the FP64 oracle's differentiated step field by field within the budget: forward,
        # dL/dout, dL/df (the adjoint convolution), dL/dP and its contraction with the hat
        # basis; each sampled field's GPU dL/df against it
        from threadpoolctl import threadpool_info

        from inputs import rel_l2
        from oracle import adjoint as oa
        from oracle import conv as oc
        from oracle import kernels as ok
        from oracle.ffc import ffc

        fd = f.detach().requires_grad_(True)
        pd = prof.detach().requires_grad_(True)
        out = radial_profile_conv(fd, pd, plan, 0, rmax, checkpoint=True)
        torch.nn.functional.mse_loss(out, target, reduction="sum").backward()
        gf = fd.grad.cpu().numpy().astype(np.float64)
        fh = f.cpu().numpy().astype(np.float64)
        th = target.cpu().numpy().astype(np.float64)
        done, errs = 0, []
        t0 = time.perf_counter()
        table = ffc(ok.radial_profile(nx, ny, m, prof.cpu().numpy(), rmax))
        for b in range(batch):
            o = oc.conv_with_coeffs(fh[b], table)
            g = 2.0 * (o - th[b])
            errs.append(rel_l2(gf[b], oc.conv_with_coeffs(g, np.conj(table))))
            oa.grad_profile(oa.grad_kernel_samples(fh[b], g), nk, rmax)
            done += 1
            if time.perf_counter() - t0 > cpu_budget:
                break
        el = time.perf_counter() - t0
        threads = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
        line_cpu = {"cpu_baseline": {"value": done / el, "unit": "conv/s", "cores": int(threads), "kind": "oracle",
                                     "sample": f"{done} of {batch} fields, FP64 oracle: profile table, forward, "
                                               f"dL/df, dL/dP and the profile contraction per field; {el:.1f} s; "
                                               f"{host_cpu()}"},
                    "rel_l2_grad_f_vs_oracle": float(max(errs))}
    # forward alone, for reference
    table = plan.coeffs(0, [se2.RadialProfile(prof.contiguous(), rmax, norm=2)])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        plan.apply(0, f, table)
    torch.cuda.synchronize()
    fwd_ms = (time.perf_counter() - t0) * 1e3 / steps
    best = min(res.values())
    return {"metric": "differentiated SE(2) convolutions/sec (forward + gradients w.r.t. f and profile)",
            "value": round(batch / (best * 1e-3), 1), "unit": "conv/s", "n_gpus": 1, "steps": steps,
            "warmup": warmup, "ms_per_step": round(best, 4), "higher_is_better": True, "dtype": "f32",
            "data": "synthetic",
            "config": {"workload": "256x256x64 f32 batch 8, radial profile 64 knots x 64 angles, "
                                   "target sigma*=0.04 kappa*=8 + 1% noise"},
            "ms_fwd_bwd": {k: round(v, 4) for k, v in res.items()},
            "ms_fwd_bwd_event_median": {k: round(v, 4) for k, v in med.items()},
            "ms_forward_full_table": round(fwd_ms, 4), **line_cpu}


def copy_calibration(name, steps, warmup):
    """A plain copy of the batch (one read + one write of every sample), timed with events."""
    import torch

    nx, ny, m, batch, nb, lc, dt, cfg = WORKLOADS[name]
    tdt = torch.float32 if dt == "f32" else torch.float64
    f = torch.rand(batch, m, ny, nx, device="cuda", dtype=tdt)
    out = torch.empty_like(f)
    for _ in range(warmup):
        out.copy_(f)
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    start.record()
    for _ in range(steps):
        out.copy_(f)
    stop.record()
    torch.cuda.synchronize()
    ms = start.elapsed_time(stop) / steps
    nbytes = 2 * f.numel() * f.element_size()
    return {"copy_calibration": name, "bytes_per_copy": nbytes, "ms_per_copy": round(ms, 5),
            "GBps": round(nbytes / (ms * 1e-3) / 1e9, 1)}


def traffic_for(kernel: str, workload: str, src_hash: str):
    """HBM bytes per launch from a committed rocprofv3 PMC summary, if it matches this source."""
    path = os.path.join(ROOT, "profiles", f"traffic_{kernel}_{workload}.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        rec = json.load(fh)
    if rec.get("source_hash") != src_hash:
        return None
    return rec.get("bytes_per_launch")


def host_cpu() -> str:
    """The host CPU model (Linux /proc/cpuinfo), for the CPU baseline's record."""
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.lower().startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown CPU"


def cpu_baseline(res, budget_s: float):
    """The FP64 oracle (route 1, table precomputed) on the host cores, bounded sample."""
    from threadpoolctl import threadpool_info

    from inputs import rel_l2
    from oracle import conv as oc
    from oracle import kernels as ok

    nx, ny, m = res["shape"]
    if res["ks"] is None:
        p = ok.sample_function(ok.exp_gauss_function(EXP_GAUSS_SIGMA[res["name"]]), nx, ny, m, images=3)
        ps = [p / p.mean()]
    else:
        ps = [ok.gauss_vm(nx, ny, m, k.sigma, k.kappa, k.theta0) for k in res["ks"]]
    table = oc.coeff_product(ps)
    f = res["f_host"].astype(np.float64)
    done = 0
    errs = []
    t0 = time.perf_counter()
    while done < res["batch"]:
        ref = oc.conv_with_coeffs(f[done], table)
        errs.append(rel_l2(res["out_host"][done].astype(np.float64), ref))
        done += 1
        if time.perf_counter() - t0 > budget_s:
            break
    el = time.perf_counter() - t0
    info = threadpool_info()
    threads = max([i.get("num_threads", 1) for i in info] + [1])
    from oracle.transforms import axis_routes
    routes = axis_routes((m, ny, nx))
    how = ", ".join(f"{ax} by {'dense DFT matrix' if r == 'dense' else 'numpy FFT'}" for ax, r in routes.items())
    return {"value": done / el, "unit": "conv/s", "cores": int(threads), "kind": "oracle",
            "sample": f"{done} of {res['batch']} fields, FP64 route 1 (forward 3-D DFT: {how}; product with the "
                      f"chain table, precomputed and excluded as on the GPU; synthesis by explicit dense "
                      f"phi_k matrices per axis); {el:.1f} s; "
                      f"BLAS: {', '.join(sorted(set(i.get('internal_api', '?') for i in info))) or 'none'}; "
                      f"{host_cpu()}"}, errs


def c0_oracle_timings(res):
    """C0 extras for the CPU side: route 1 on one thread, and route 2 (direct quadrature in C)."""
    from threadpoolctl import threadpool_limits

    from inputs import rel_l2
    from oracle import conv as oc
    from oracle import kernels as ok
    from oracle import quadrature as oq

    nx, ny, m = res["shape"]
    k = res["ks"][0]
    f = res["f_host"][0].astype(np.float64)
    gpu = res["out_host"][0].astype(np.float64)
    table = oc.coeff_product([ok.gauss_vm(nx, ny, m, k.sigma, k.kappa, k.theta0)])
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        r1 = oc.conv_with_coeffs(f, table)
        t1 = time.perf_counter() - t0
    # route 2 with the continuous-mass kernel function, rescaled to the discrete unit mass
    # that the GPU table uses (the ratio is the mean of the continuous-mass samples)
    pc = ok.gauss_vm(nx, ny, m, k.sigma, k.kappa, k.theta0, normalize="continuous")
    t0 = time.perf_counter()
    r2 = oq.quadrature_conv(f, ok.gauss_vm_function(k.sigma, k.kappa, k.theta0)) / pc.mean()
    t2 = time.perf_counter() - t0
    return {"route1_single_thread": {"seconds": round(t1, 4), "rel_l2_vs_gpu": rel_l2(gpu, r1)},
            "route2_direct_quadrature": {"seconds": round(t2, 3),
                                         "threads": int(os.environ.get("OMP_NUM_THREADS", os.cpu_count())),
                                         "note": "O(n^2) rectangle rule in C with the image-summed kernel "
                                                 "table (table build included)",
                                         "rel_l2_vs_gpu": rel_l2(gpu, r2)}}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="headline", choices=sorted(WORKLOADS) + list(SPECIAL))
    ap.add_argument("--cpu-budget", type=float, default=15.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-tune", action="store_true", help="keep the default schedule (no autotuning)")
    ap.add_argument("--no-secondary", action="store_true",
                    help="headline only: skip the plain, uneven-batch and differentiated lines")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="time a plain device copy of the workload's input instead (calibrates HBM "
                         "byte counters and gives the achievable streaming bandwidth)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU; --gpus above 1 is not supported "
                                   "(the fields of a batch are independent: a batch would be split across "
                                   "GPUs with no communication)"}))
        sys.exit(2)

    if args.copy_calibration:
        print(json.dumps(copy_calibration(args.workload, args.steps, args.warmup)), flush=True)
        return
    if args.workload == "c2":
        print(json.dumps(run_c2(args.steps, args.warmup, None if args.no_cpu else args.cpu_budget)), flush=True)
        return
    if args.workload == "c4":
        print(json.dumps(run_c4(args.steps, args.warmup, None if args.no_cpu else args.cpu_budget)), flush=True)
        return
    if args.workload == "powers":
        print(json.dumps(run_powers(args.steps, args.warmup, None if args.no_cpu else args.cpu_budget)), flush=True)
        return
    if args.workload == "shifted":
        print(json.dumps(run_shifted(args.steps, args.warmup, None if args.no_cpu else args.cpu_budget)), flush=True)
        return
    if args.workload == "padded":
        print(json.dumps(run_padded(args.steps, args.warmup, None if args.no_cpu else args.cpu_budget)), flush=True)
        return
    res = run_gpu(args.workload, args.steps, args.warmup, tune=not args.no_tune)
    nx, ny, m = res["shape"]
    n = nx * ny * m
    batch = res["batch"]
    ms_per_step = res["elapsed"] * 1e3 / args.steps
    value = batch * args.steps / res["elapsed"]
    rb = 4 if res["dtype"] == "f32" else 8
    alg_bytes_step = 2 * rb * n * batch              # read f, write out (algorithmic)
    # dominant pass = largest total time per step; every launch of a pass streams the whole
    # batch once in and once out (a kind launched twice per step, e.g. the forward and the
    # inverse x-theta pass of the full-table path, does that twice)
    dom = max(res["avg_ms"], key=lambda k: res["avg_ms"][k] * res["launches"][k])
    dom_ms = res["avg_ms"][dom]
    alg_bytes_launch = alg_bytes_step
    achieved = alg_bytes_launch / (dom_ms * 1e-3) / 1e9
    src = lib_source_hash()
    traffic = traffic_for(dom, args.workload, src)
    line = {
        "metric": METRIC,
        "value": round(value, 2),
        "unit": "conv/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": res["dtype"],
        "data": "synthetic",
        "config": describe(args.workload),
        "path_alg_GBps": round(alg_bytes_step / (ms_per_step * 1e-3) / 1e9, 1),
        "pass_ms": {k: round(v, 4) for k, v in res["avg_ms"].items()},
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": traffic, "alg_bytes_per_launch": alg_bytes_launch,
                     "launches_per_step": res["launches"][dom]},
        "source_hash": src,
        "autotune_s": None if res["tune_s"] is None else round(res["tune_s"], 2),
    }
    # the same step as a HIP graph, median of event-timed replays (the dominant kernel's
    # fraction above is the per-kernel roofline; the whole path's is beside it)
    rm = res["replay_median_ms"]
    line["replay_median_ms"] = round(rm, 4)
    line["replays"] = res["replays"]
    line["replay_identical_to_eager"] = res["replay_identical"]
    line["conv_per_s_replay_median"] = round(batch / (rm * 1e-3), 1)
    line["whole_path"] = {"alg_bytes_per_step": alg_bytes_step,
                          "achieved": round(alg_bytes_step / (rm * 1e-3) / 1e9, 1), "peak": HBM_PEAK_GBS,
                          "unit": "GB/s", "frac": round(alg_bytes_step / (rm * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                          "note": "read every field once and write every output once, over the replay median"}
    lc = describe(args.workload)["chain"]
    line["chain_expanded_per_s"] = round(value * lc, 1)
    if args.workload == "headline" and not args.no_secondary:
        line["secondary"] = secondary(args.steps, args.warmup, tune=not args.no_tune)
    if not args.no_cpu:
        cb, errs = cpu_baseline(res, args.cpu_budget)
        line["cpu_baseline"] = cb
        line["rel_l2_vs_oracle"] = float(max(errs))
        line["rel_l2_tol"] = float(2e-6 * np.log2(n))
        if args.workload == "c0":
            line["cpu_oracle_c0"] = c0_oracle_timings(res)
    print(json.dumps(line), flush=True)


def secondary(steps, warmup, tune=True):
    """The plain single-kernel convolution at the headline shape, the uneven batch (C2), the
    differentiated form (C4), a sum of SE(2)-shifted kernels, the FP64 path at 512x512x128
    (C3) and the prime length 101, measured in the same invocation."""
    out = {}
    r = run_gpu("headline_plain", steps, warmup, tune=tune)
    nx, ny, m = r["shape"]
    rm = r["replay_median_ms"]
    out["plain_chain1"] = {"workload": describe("headline_plain")["workload"],
                           "conv_per_s": round(r["batch"] * steps / r["elapsed"], 1),
                           "ms_per_step": round(r["elapsed"] * 1e3 / steps, 4),
                           "replay_median_ms": round(rm, 4),
                           "conv_per_s_replay_median": round(r["batch"] / (rm * 1e-3), 1),
                           "pass_ms": {k: round(v, 4) for k, v in r["avg_ms"].items()}}
    c2 = run_c2(steps, warmup)
    out["uneven_batch_c2"] = {k: c2[k] for k in ("value", "unit", "ms_per_step", "replay_median_ms", "replays",
                                                 "conv_per_s_replay_median", "path_alg_GBps", "replay_alg_GBps")}
    out["uneven_batch_c2"]["workload"] = c2["config"]["workload"]
    c4 = run_c4(max(10, steps // 2), max(2, warmup // 2))
    out["differentiated_c4"] = {k: c4[k] for k in ("value", "unit", "ms_per_step", "ms_fwd_bwd",
                                                   "ms_fwd_bwd_event_median", "ms_forward_full_table")}
    out["differentiated_c4"]["workload"] = c4["config"]["workload"]
    sh = run_shifted(steps, warmup)
    out["shifted_kernel_sum"] = {k: sh[k] for k in ("value", "unit", "ms_per_step", "replay_median_ms",
                                                    "pass_ms_total_per_step")}
    out["shifted_kernel_sum"]["workload"] = sh["config"]["workload"]
    # the FP64 path (three register passes) and a prime grid length (Rader's algorithm)
    for key, name in (("fp64_c3", "c3_f64"), ("prime_length_101", "odd101")):
        r = run_gpu(name, steps, warmup, tune=tune)
        rm = r["replay_median_ms"]
        out[key] = {"workload": describe(name)["workload"], "dtype": WORKLOADS[name][6],
                    "conv_per_s": round(r["batch"] * steps / r["elapsed"], 1),
                    "ms_per_step": round(r["elapsed"] * 1e3 / steps, 4),
                    "replay_median_ms": round(rm, 4),
                    "conv_per_s_replay_median": round(r["batch"] / (rm * 1e-3), 1),
                    "pass_ms": {k: round(v, 4) for k, v in r["avg_ms"].items()}}
    return out


if __name__ == "__main__":
    main()
