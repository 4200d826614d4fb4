"""Python binding of the se2conv C ABI (argument marshalling only).

PyTorch provides device memory and streams; every step of the convolution runs
in the HIP kernels of libse2conv.so.  Names follow the C ABI.
"""
from __future__ import annotations

import ctypes
import dataclasses
import weakref

import torch

from . import _lib as L


@dataclasses.dataclass
class GaussVM:
    """exp(-|x|^2 / 2 sigma^2) * exp(kappa cos(theta - theta0)), radial in translations."""
    sigma: float
    kappa: float
    theta0: float = 0.0
    norm: int = L.KNORM_DISCRETE


@dataclasses.dataclass
class Samples:
    """Kernel samples P[theta][y][x] on the grid (device float64 tensor)."""
    data: torch.Tensor
    norm: int = L.KNORM_DISCRETE


@dataclasses.dataclass
class RadialProfile:
    """Piecewise-linear radial profile prof[n_knots][M] (device float64), knots up to r_max."""
    prof: torch.Tensor
    r_max: float
    norm: int = L.KNORM_NONE


@dataclasses.dataclass
class ExpGauss:
    """Exponential-coordinates Gaussian exp(-||log(x, R)^v||^2 / (2 sigma^2)) (FULL table)."""
    sigma: float
    norm: int = L.KNORM_DISCRETE


def _stream_handle(stream) -> int:
    if stream is None:
        stream = torch.cuda.current_stream()
    return int(stream.cuda_stream)


def _desc(k) -> L.KernelDesc:
    d = L.KernelDesc()
    if isinstance(k, GaussVM):
        d.kind, d.flags = L.K_GAUSS_VM, k.norm
        d.sigma, d.kappa, d.theta0 = k.sigma, k.kappa, k.theta0
    elif isinstance(k, Samples):
        _require(k.data, torch.float64)
        d.kind, d.flags, d.data = L.K_SAMPLES, k.norm, k.data.data_ptr()
    elif isinstance(k, RadialProfile):
        _require(k.prof, torch.float64)
        d.kind, d.flags, d.data = L.K_RADIAL_PROFILE, k.norm, k.prof.data_ptr()
        d.n_knots, d.r_max = int(k.prof.shape[0]), float(k.r_max)
    elif isinstance(k, ExpGauss):
        d.kind, d.flags, d.sigma = L.K_EXP_GAUSS, k.norm, k.sigma
    else:
        raise TypeError(f"unknown kernel descriptor {k!r}")
    return d


def _require(t: torch.Tensor, dtype) -> None:
    if not t.is_cuda or t.dtype != dtype or not t.is_contiguous():
        raise ValueError(f"expected a contiguous {dtype} device tensor")


def _release_table(plan: "Plan", ptr: int) -> None:
    # the buffer is about to be freed: the plan forgets the address, so a later
    # allocation at the same address is not taken for this table
    if plan.handle:
        plan._lib.se2conv_table_release(plan.handle, ptr)


class Table:
    """A coefficient table produced by Plan.coeffs (device buffer + its plan).

    When the Table is garbage-collected its record in the plan is released
    (se2conv_table_release) before the buffer goes back to the allocator."""

    def __init__(self, plan: "Plan", shape_idx: int, buf: torch.Tensor, kind: int):
        self.plan = plan
        self.shape_idx = shape_idx
        self.buf = buf
        self.kind = kind
        weakref.finalize(self, _release_table, plan, buf.data_ptr())

    @property
    def ptr(self) -> int:
        return self.buf.data_ptr()

    def complex_view(self) -> torch.Tensor:
        """The table as a complex tensor (SEPARABLE: [Nx+Ny+M]; FULL: [M][Ny][Nx];
        QUARTER: [M][Ny/2+1][Nx/2+1])."""
        nx, ny, m = self.plan.shapes[self.shape_idx]
        cdt = torch.complex64 if self.plan.dtype == L.F32 else torch.complex128
        v = self.buf.view(cdt)
        if self.kind == L.TABLE_SEPARABLE:
            return v
        if self.kind == L.TABLE_QUARTER:
            return v.view(m, ny // 2 + 1, nx // 2 + 1)
        return v.view(m, ny, nx)


class Plan:
    def __init__(self, shapes, dtype: str = "f32", host_only: bool = False, generic: bool = False):
        self._lib = L.load()
        self.shapes = [tuple(int(v) for v in s) for s in shapes]
        self.dtype = {"f32": L.F32, "f64": L.F64}[dtype]
        self.tdtype = torch.float32 if self.dtype == L.F32 else torch.float64
        arr = (L.Shape * len(self.shapes))(*[L.Shape(*s) for s in self.shapes])
        h = ctypes.c_void_p()
        flags = (L.PLAN_HOST_ONLY if host_only else 0) | (L.PLAN_GENERIC if generic else 0)
        L.check(self._lib.se2conv_plan(arr, len(self.shapes), self.dtype, flags, ctypes.byref(h)))
        self.handle = h
        self._tables = []

    def close(self) -> None:
        if self.handle:
            L.check(self._lib.se2conv_plan_destroy(self.handle))
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def counts(self) -> tuple[int, int]:
        """(tables recorded by the plan, cached chain submissions)."""
        nt, ns = ctypes.c_int64(0), ctypes.c_int64(0)
        L.check(self._lib.se2conv_plan_counts(self.handle, ctypes.byref(nt), ctypes.byref(ns)))
        return int(nt.value), int(ns.value)

    def table_bytes(self, shape_idx: int, kernels) -> int:
        descs = (L.KernelDesc * len(kernels))(*[_desc(k) for k in kernels])
        nbytes = ctypes.c_size_t(0)
        L.check(self._lib.se2conv_coeffs(self.handle, shape_idx, descs, len(kernels), None,
                                         ctypes.byref(nbytes), None))
        return int(nbytes.value)

    def coeffs(self, shape_idx: int, kernels, stream=None) -> Table:
        descs = (L.KernelDesc * len(kernels))(*[_desc(k) for k in kernels])
        nbytes = ctypes.c_size_t(0)
        L.check(self._lib.se2conv_coeffs(self.handle, shape_idx, descs, len(kernels), None,
                                         ctypes.byref(nbytes), None))
        buf = torch.empty(nbytes.value, dtype=torch.uint8, device="cuda")
        L.check(self._lib.se2conv_coeffs(self.handle, shape_idx, descs, len(kernels), buf.data_ptr(),
                                         ctypes.byref(nbytes), _stream_handle(stream)))
        kind = ctypes.c_int32()
        L.check(self._lib.se2conv_table_info(self.handle, buf.data_ptr(), ctypes.byref(kind), None, None))
        t = Table(self, shape_idx, buf, kind.value)
        return t

    def coeffs_sum(self, shape_idx: int, terms, stream=None) -> Table:
        """FULL table of a weighted sum of kernels: terms = [(weight, kernel), ...]
        (se2conv_coeffs_sum)."""
        descs = (L.KernelDesc * len(terms))(*[_desc(k) for _, k in terms])
        w = (ctypes.c_double * len(terms))(*[float(a) for a, _ in terms])
        nbytes = ctypes.c_size_t(0)
        L.check(self._lib.se2conv_coeffs_sum(self.handle, shape_idx, descs, w, len(terms), None,
                                             ctypes.byref(nbytes), None))
        buf = torch.empty(nbytes.value, dtype=torch.uint8, device="cuda")
        L.check(self._lib.se2conv_coeffs_sum(self.handle, shape_idx, descs, w, len(terms), buf.data_ptr(),
                                             ctypes.byref(nbytes), _stream_handle(stream)))
        return Table(self, shape_idx, buf, L.TABLE_FULL)

    def quarter(self, table: Table, stream=None) -> Table:
        """The FULL table folded by the reflection symmetries of a radial kernel
        (se2conv_table_quarter): M (Ny/2+1) (Nx/2+1) coefficients, usable wherever the FULL
        table is.  Raises if the table is not symmetric (a kernel not radial in translations)."""
        nbytes = ctypes.c_size_t(0)
        L.check(self._lib.se2conv_table_quarter(self.handle, table.ptr, None, ctypes.byref(nbytes), None))
        buf = torch.empty(nbytes.value, dtype=torch.uint8, device="cuda")
        L.check(self._lib.se2conv_table_quarter(self.handle, table.ptr, buf.data_ptr(), ctypes.byref(nbytes),
                                                _stream_handle(stream)))
        return Table(self, table.shape_idx, buf, L.TABLE_QUARTER)

    def apply(self, shape_idx: int, f: torch.Tensor, table: Table, out: torch.Tensor | None = None,
              adjoint: bool = False, stream=None, timing: bool = False) -> torch.Tensor:
        _require(f, self.tdtype)
        nx, ny, m = self.shapes[shape_idx]
        if f.shape[-3:] != (m, ny, nx):
            raise ValueError(f"field shape {tuple(f.shape)} does not end in {(m, ny, nx)}")
        batch = f.numel() // (nx * ny * m)
        if out is None:
            out = torch.empty_like(f)
        _require(out, self.tdtype)
        L.check(self._lib.se2conv_apply(self.handle, shape_idx, f.data_ptr(), table.ptr, out.data_ptr(),
                                        batch, (L.ADJOINT if adjoint else 0) | (L.TIMING if timing else 0),
                                        _stream_handle(stream)))
        return out

    def shift_table(self, shape_idx: int, shifts, stream=None) -> Table:
        """Translation-phase tables of a sum of SE(2)-shifted kernels (se2conv_shift_table):
        shifts = [(tx, ty, roll, weight), ...], the rotation of each shift 2 pi roll / M."""
        arr = (L.Shift * len(shifts))(*[L.Shift(float(tx), float(ty), float(w), int(r)) for tx, ty, r, w in shifts])
        nbytes = ctypes.c_size_t(0)
        L.check(self._lib.se2conv_shift_table(self.handle, shape_idx, arr, len(shifts), None, ctypes.byref(nbytes),
                                              None))
        buf = torch.empty(nbytes.value, dtype=torch.uint8, device="cuda")
        L.check(self._lib.se2conv_shift_table(self.handle, shape_idx, arr, len(shifts), buf.data_ptr(),
                                              ctypes.byref(nbytes), _stream_handle(stream)))
        return Table(self, shape_idx, buf, L.TABLE_SHIFT)

    def apply_shifted(self, shape_idx: int, f: torch.Tensor, shift_table: Table, kernel_tables,
                      out: torch.Tensor | None = None, stream=None, timing: bool = False) -> torch.Tensor:
        """Re S_K[f, sum_k a_k rho(s_k^{-1} .)] (se2conv_apply_shifted); kernel_tables: rho's chain."""
        _require(f, self.tdtype)
        nx, ny, m = self.shapes[shape_idx]
        if f.shape[-3:] != (m, ny, nx):
            raise ValueError(f"field shape {tuple(f.shape)} does not end in {(m, ny, nx)}")
        batch = f.numel() // (nx * ny * m)
        if out is None:
            out = torch.empty_like(f)
        _require(out, self.tdtype)
        tp = (ctypes.c_void_p * len(kernel_tables))(*[t.ptr for t in kernel_tables])
        L.check(self._lib.se2conv_apply_shifted(self.handle, shape_idx, f.data_ptr(), shift_table.ptr, tp,
                                                len(kernel_tables), out.data_ptr(), batch,
                                                L.TIMING if timing else 0, _stream_handle(stream)))
        return out

    def apply_complex(self, shape_idx: int, f: torch.Tensor, table: Table, out: torch.Tensor | None = None,
                      adjoint: bool = False, stream=None, timing: bool = False) -> torch.Tensor:
        """S_K[f, chain] for complex-valued fields f (complex64 / complex128 by plan dtype)."""
        cdt = torch.complex64 if self.dtype == L.F32 else torch.complex128
        _require(f, cdt)
        nx, ny, m = self.shapes[shape_idx]
        if f.shape[-3:] != (m, ny, nx):
            raise ValueError(f"field shape {tuple(f.shape)} does not end in {(m, ny, nx)}")
        batch = f.numel() // (nx * ny * m)
        if out is None:
            out = torch.empty_like(f)
        _require(out, cdt)
        L.check(self._lib.se2conv_apply_complex(self.handle, shape_idx, f.data_ptr(), table.ptr, out.data_ptr(),
                                                batch, (L.ADJOINT if adjoint else 0) | (L.TIMING if timing else 0),
                                                _stream_handle(stream)))
        return out

    def apply_padded(self, shape_idx: int, f: torch.Tensor, table: Table, out_shape_idx: int,
                     out: torch.Tensor | None = None, adjoint: bool = False, stream=None,
                     timing: bool = False) -> torch.Tensor:
        """Re S_K[f, chain] on the finer grid of shape out_shape_idx (zero-padded evaluation)."""
        _require(f, self.tdtype)
        nx, ny, m = self.shapes[shape_idx]
        gx, gy, gm = self.shapes[out_shape_idx]
        if f.shape[-3:] != (m, ny, nx):
            raise ValueError(f"field shape {tuple(f.shape)} does not end in {(m, ny, nx)}")
        batch = f.numel() // (nx * ny * m)
        if out is None:
            out = torch.empty(tuple(f.shape[:-3]) + (gm, gy, gx), dtype=f.dtype, device=f.device)
        _require(out, self.tdtype)
        L.check(self._lib.se2conv_apply_padded(self.handle, shape_idx, f.data_ptr(), table.ptr, out_shape_idx,
                                               out.data_ptr(), batch,
                                               (L.ADJOINT if adjoint else 0) | (L.TIMING if timing else 0),
                                               _stream_handle(stream)))
        return out

    def field_coeffs(self, shape_idx: int, f: torch.Tensor, stream=None) -> list:
        """FFC tables of each field of f (FULL tables in the plan dtype), one Table per field."""
        _require(f, self.tdtype)
        nx, ny, m = self.shapes[shape_idx]
        batch = f.numel() // (nx * ny * m)
        nbytes = nx * ny * m * (8 if self.dtype == L.F32 else 16)
        stride = (nbytes + 15) // 16 * 16  # the ABI wants 16-byte aligned tables
        buf = torch.empty(batch * stride, dtype=torch.uint8, device=f.device)
        L.check(self._lib.se2conv_field_coeffs(self.handle, shape_idx, f.data_ptr(), batch, buf.data_ptr(), stride,
                                               _stream_handle(stream)))
        tabs = [Table(self, shape_idx, buf[b * stride:b * stride + nbytes], L.TABLE_FULL) for b in range(batch)]
        for t in tabs:
            t.stride = stride
        return tabs

    def kernel_grad(self, shape_idx: int, g: torch.Tensor, ftables: list, stream=None) -> torch.Tensor:
        """sum_b dL/dP_b for dL/dout_b = g_b, given the fields' FFC tables (one [M, Ny, Nx] tensor)."""
        _require(g, self.tdtype)
        nx, ny, m = self.shapes[shape_idx]
        batch = g.numel() // (nx * ny * m)
        if len(ftables) != batch:
            raise ValueError("need one field table per field")
        base = ftables[0].ptr
        stride = getattr(ftables[0], "stride", None) or ftables[0].buf.numel()
        if any(t.ptr != base + b * stride for b, t in enumerate(ftables)):
            raise ValueError("field tables must come from one se2conv_field_coeffs call")
        out = torch.empty(m, ny, nx, dtype=self.tdtype, device=g.device)
        L.check(self._lib.se2conv_kernel_grad(self.handle, shape_idx, g.data_ptr(), base, stride, batch,
                                              out.data_ptr(), _stream_handle(stream)))
        return out

    def fused_supported(self, shape_idx: int) -> bool:
        """True when field_spectra / apply_save / backward run for this plan and shape."""
        return bool(self._lib.se2conv_fused_supported(self.handle, shape_idx))

    def _spectra_buffer(self, shape_idx: int, batch: int, device) -> torch.Tensor:
        nx, ny, m = self.shapes[shape_idx]
        return torch.empty(2 * ((batch + 1) // 2), m, ny, nx, dtype=torch.float32, device=device)

    def field_spectra(self, shape_idx: int, f: torch.Tensor, stream=None) -> torch.Tensor:
        """3-D DFTs of field pairs packed as re/im: [2 ceil(B/2), M, Ny, Nx] FP32 planes."""
        _require(f, self.tdtype)
        nx, ny, m = self.shapes[shape_idx]
        batch = f.numel() // (nx * ny * m)
        spec = self._spectra_buffer(shape_idx, batch, f.device)
        L.check(self._lib.se2conv_field_spectra(self.handle, shape_idx, f.data_ptr(), batch, spec.data_ptr(),
                                                _stream_handle(stream)))
        return spec

    def apply_save(self, shape_idx: int, f: torch.Tensor, table: Table, out: torch.Tensor | None = None,
                   stream=None):
        """Forward apply that also returns the field spectra (the backward's checkpoint)."""
        _require(f, self.tdtype)
        nx, ny, m = self.shapes[shape_idx]
        batch = f.numel() // (nx * ny * m)
        if out is None:
            out = torch.empty_like(f)
        spec = self._spectra_buffer(shape_idx, batch, f.device)
        L.check(self._lib.se2conv_apply_save(self.handle, shape_idx, f.data_ptr(), table.ptr, out.data_ptr(), batch,
                                             spec.data_ptr(), _stream_handle(stream)))
        return out, spec

    def backward(self, shape_idx: int, g: torch.Tensor, table: Table, spectra: torch.Tensor,
                 grad_f: torch.Tensor | None = None, stream=None):
        """(dL/df, sum_b dL/dP) through out = S_K[f, table] from g = dL/dout and f's spectra."""
        _require(g, self.tdtype)
        nx, ny, m = self.shapes[shape_idx]
        batch = g.numel() // (nx * ny * m)
        if grad_f is None:
            grad_f = torch.empty_like(g)
        grad_p = torch.empty(m, ny, nx, dtype=self.tdtype, device=g.device)
        L.check(self._lib.se2conv_backward(self.handle, shape_idx, g.data_ptr(), table.ptr, spectra.data_ptr(),
                                           batch, grad_f.data_ptr(), grad_p.data_ptr(), _stream_handle(stream)))
        return grad_f, grad_p

    def profile_grad(self, shape_idx: int, grad_samples: torch.Tensor, n_knots: int, r_max: float,
                     stream=None) -> torch.Tensor:
        """sum over the batch of the hat-basis transpose of dL/dP: a float64 [n_knots, M] tensor."""
        _require(grad_samples, self.tdtype)
        nx, ny, m = self.shapes[shape_idx]
        batch = grad_samples.numel() // (nx * ny * m)
        out = torch.empty(n_knots, m, dtype=torch.float64, device=grad_samples.device)
        L.check(self._lib.se2conv_profile_grad(self.handle, shape_idx, grad_samples.data_ptr(), batch, n_knots,
                                               float(r_max), out.data_ptr(), _stream_handle(stream)))
        return out

    def powers(self, shape_idx: int, f: torch.Tensor, table: Table, q: int, adjoint: bool = False,
               stream=None) -> torch.Tensor:
        """All S_K[f, rho^(p)], p = 1..q (the paper's fast loop): a [q, *f.shape] tensor."""
        _require(f, self.tdtype)
        nx, ny, m = self.shapes[shape_idx]
        batch = f.numel() // (nx * ny * m)
        out = torch.empty((q,) + tuple(f.shape), dtype=f.dtype, device=f.device)
        L.check(self._lib.se2conv_powers(self.handle, shape_idx, f.data_ptr(), table.ptr, q, out.data_ptr(), batch,
                                         L.ADJOINT if adjoint else 0, _stream_handle(stream)))
        return out

    def sample_bumps(self, shape_idx: int, centres, theta0, weights, s: float, kappa: float,
                     out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
        """Samples of a periodized Gaussian x von Mises bump field on the grid (one field)."""
        nx, ny, m = self.shapes[shape_idx]
        import numpy as np
        params = np.stack([np.asarray(centres)[:, 0], np.asarray(centres)[:, 1], np.asarray(theta0),
                           np.asarray(weights)], axis=1).astype(np.float64)
        dparams = torch.from_numpy(np.ascontiguousarray(params)).to("cuda")
        if out is None:
            out = torch.empty(m, ny, nx, dtype=self.tdtype, device="cuda")
        _require(out, self.tdtype)
        L.check(self._lib.se2conv_sample_bumps(self.handle, shape_idx, dparams.data_ptr(), params.shape[0],
                                               float(s), float(kappa), out.data_ptr(), _stream_handle(stream)))
        # keep the parameter buffer alive until the kernel has read it
        (torch.cuda.current_stream() if stream is None else stream).synchronize()
        return out

    def autotune(self, shape_idx: int, batch: int = 4, stream=None) -> None:
        """Time candidate launch schedules for one shape and keep the fastest in the plan."""
        L.check(self._lib.se2conv_autotune(self.handle, shape_idx, batch, _stream_handle(stream)))

    def pass_times(self, cap: int = 4096):
        """[(pass kind name, milliseconds)] of passes enqueued with timing=True since the last read."""
        ms = (ctypes.c_float * cap)()
        kinds = (ctypes.c_int32 * cap)()
        n = ctypes.c_int32(0)
        L.check(self._lib.se2conv_pass_times(self.handle, ms, kinds, cap, ctypes.byref(n)))
        return [(L.PASS_KINDS.get(kinds[i], str(kinds[i])), float(ms[i])) for i in range(min(n.value, cap))]

    def chain_noalloc(self, problems, adjoint: bool = False, stream=None) -> None:
        """se2conv_chain_noalloc: problems as for chain(), separable tables only; the item
        lists go into the library's fixed device array (no device allocation)."""
        arr, keep = self._problem_array(problems)
        L.check(self._lib.se2conv_chain_noalloc(self.handle, arr, len(problems), L.ADJOINT if adjoint else 0,
                                                _stream_handle(stream)))

    def _problem_array(self, problems):
        keep = []
        arr = (L.Problem * len(problems))()
        for i, (sidx, f, out, tabs) in enumerate(problems):
            nx, ny, m = self.shapes[sidx]
            tp = (ctypes.c_void_p * len(tabs))(*[t.ptr for t in tabs])
            keep.append(tp)
            arr[i].shape_idx = sidx
            arr[i].batch = f.numel() // (nx * ny * m)
            arr[i].f = f.data_ptr()
            arr[i].out = out.data_ptr()
            arr[i].tables = ctypes.cast(tp, ctypes.POINTER(ctypes.c_void_p))
            arr[i].n_tables = len(tabs)
        return arr, keep

    def chain(self, problems, adjoint: bool = False, graph: bool = False, stream=None,
              timing: bool = False) -> None:
        """problems: list of (shape_idx, f, out, [tables])."""
        arr, keep = self._problem_array(problems)
        flags = (L.ADJOINT if adjoint else 0) | (L.GRAPH if graph else 0) | (L.TIMING if timing else 0)
        L.check(self._lib.se2conv_chain(self.handle, arr, len(problems), flags, _stream_handle(stream)))

    def chain_submission(self, problems, adjoint: bool = False, graph: bool = True) -> "ChainSubmission":
        """A problem list marshalled once, for repeated se2conv_chain calls (a serving loop)."""
        return ChainSubmission(self, problems, adjoint, graph)


class ChainSubmission:
    """A se2conv_chain problem list marshalled once (the argument arrays are built here and
    reused by every run; the tensors and tables stay referenced)."""

    def __init__(self, plan: Plan, problems, adjoint: bool = False, graph: bool = True):
        self.plan = plan
        self.problems = list(problems)
        self.arr, self._keep = plan._problem_array(self.problems)
        self.flags = (L.ADJOINT if adjoint else 0) | (L.GRAPH if graph else 0)

    def run(self, stream=None) -> None:
        L.check(self.plan._lib.se2conv_chain(self.plan.handle, self.arr, len(self.problems), self.flags,
                                             _stream_handle(stream)))
