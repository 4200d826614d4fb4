"""Uneven batches with both class kinds of the multi-class kernels (2^k and 3 * 2^k points).

With both kinds present, se2conv_chain runs the second kind on one of the plan's auxiliary
streams, forked from and joined back into the caller's stream; with SE2CONV_TIMING, and in
se2conv_chain_noalloc, both kinds run in turn on the caller's stream.  The kernels are the
same either way, so the outputs must be bitwise identical; every problem is also scored
against the FP64 oracle, and graph replays of the forked submission must equal the eager
result, with unrelated work on the stream between them.
"""
import numpy as np
import pytest
import torch

import paper_2504_05149_amd as se2
from gpu_common import case, oracle_table_gauss, parity_err, tol32
from inputs import chain_kernel_params, sample_fields

from oracle import conv as oc

pytestmark = pytest.mark.gpu
DEV = "cuda:0"

# (nx, ny, m, batch): classes of 2^k points (first kind) and of 3 * 2^k (second kind)
PROBLEMS = [(64, 64, 32, 2), (128, 128, 16, 1), (96, 96, 16, 3), (48, 48, 64, 2), (32, 32, 64, 2), (96, 96, 64, 1)]


def _setup():
    shapes = sorted({(nx, ny, m) for nx, ny, m, _ in PROBLEMS})
    plan = se2.Plan(shapes, dtype="f32")
    probs, refs = [], []
    for i, (nx, ny, m, batch) in enumerate(PROBLEMS):
        sidx = shapes.index((nx, ny, m))
        ks = chain_kernel_params(30 + i, 2)
        chain = [(k.sigma, k.kappa, 0.3 * j) for j, k in enumerate(ks)]
        f = sample_fields(30 + i, batch, 8, nx, ny, m)
        fd = torch.from_numpy(f).to(DEV, torch.float32)
        tables = [plan.coeffs(sidx, [se2.GaussVM(*c)]) for c in chain]
        probs.append((sidx, fd, torch.empty_like(fd), tables))
        refs.append((f, oracle_table_gauss(nx, ny, m, chain)))
    return plan, probs, refs


def test_forked_kinds_match_one_stream_and_oracle():
    case("uneven batch with both class kinds: forked (two streams) vs in turn (timing, no-alloc) vs oracle")
    plan, probs, refs = _setup()
    stream = torch.cuda.Stream()
    outs = {}
    for how in ("forked", "timing", "noalloc"):
        for _, _, out, _ in probs:
            out.fill_(float("nan"))
        torch.cuda.synchronize()
        if how == "forked":
            plan.chain(probs, stream=stream)
        elif how == "timing":
            plan.chain(probs, stream=stream, timing=True)
        else:
            plan.chain_noalloc(probs, stream=stream)
        torch.cuda.synchronize()
        outs[how] = [out.clone() for _, _, out, _ in probs]
    plan.pass_times()  # drain the timing records
    for k, (nx, ny, m, batch) in enumerate(PROBLEMS):
        assert torch.equal(outs["forked"][k], outs["timing"][k]), (nx, ny, m)
        assert torch.equal(outs["forked"][k], outs["noalloc"][k]), (nx, ny, m)
        o = outs["forked"][k].cpu().numpy().astype(np.float64)
        f, ref_t = refs[k]
        for b in range(batch):
            err = parity_err(o[b], oc.conv_with_coeffs(f[b], ref_t))
            print(f"  {nx}x{ny}x{m} field {b}: {err:.2e}", flush=True)
            assert err <= tol32(nx * ny * m)
    plan.close()


def test_forked_kinds_graph_replays():
    case("uneven batch with both class kinds: graph replays of the forked submission vs eager")
    plan, probs, _ = _setup()
    stream = torch.cuda.Stream()
    plan.chain(probs, stream=stream)
    torch.cuda.synchronize()
    eager = [out.clone() for _, _, out, _ in probs]
    for rep in range(4):
        for _, _, out, _ in probs:
            out.zero_()
        torch.cuda.synchronize()
        plan.chain(probs, graph=True, stream=stream)
        torch.cuda.synchronize()
        _ = torch.ones(4096, device=DEV).sum().item()  # unrelated eager work between replays
        for e, (_, _, out, _) in zip(eager, probs):
            assert torch.equal(e, out), f"graph replay {rep} differs from eager"
    plan.close()
