"""C ABI checks that need no GPU: symbols, status strings, host-side validation."""
import ctypes
import os
import re

import pytest

import paper_2504_05149_amd as se2
from paper_2504_05149_amd import _lib as L

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    with open(os.path.join(ROOT, "include", "se2conv.h")) as fh:
        text = fh.read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(se2conv_[a-z_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    lib = L.load()
    names = _declared_functions()
    assert "se2conv_apply" in names and "se2conv_chain" in names
    for name in names:
        assert hasattr(lib, name), name
    assert set(names) == set(L.EXPORTED)


def test_status_strings():
    lib = L.load()
    for code in range(6):
        assert lib.se2conv_status_string(code)
    assert lib.se2conv_status_string(99) == b"unknown status"


@pytest.mark.parametrize("shape", [(7, 8, 8), (8, 8, 1), (1024, 8, 8), (8, 600, 8), (8, 8, 513)])
def test_unsupported_sizes(shape):
    with pytest.raises(se2.Se2convError) as e:
        se2.Plan([shape], host_only=True)
    assert e.value.status == L.ERR_UNSUPPORTED_SIZE


@pytest.mark.parametrize("shape", [(31, 31, 31), (33, 41, 43), (101, 53, 17), (50, 32, 35), (10, 8, 5)])
def test_odd_and_prime_sizes_are_accepted(shape):
    # the paper's odd grids L = 2K+1 (Sec. 3.2) and lengths with any prime factor
    se2.Plan([shape], host_only=True).close()


def test_bad_plan_arguments():
    lib = L.load()
    h = ctypes.c_void_p()
    shp = (L.Shape * 1)(L.Shape(32, 32, 32))
    assert lib.se2conv_plan(shp, 0, 0, L.PLAN_HOST_ONLY, ctypes.byref(h)) == L.ERR_INVALID_ARG
    assert lib.se2conv_plan(shp, 1, 7, L.PLAN_HOST_ONLY, ctypes.byref(h)) == L.ERR_INVALID_ARG
    assert lib.se2conv_plan(shp, 1, 0, 0x80, ctypes.byref(h)) == L.ERR_INVALID_ARG
    assert lib.se2conv_plan(shp, 1, 0, L.PLAN_HOST_ONLY, None) == L.ERR_INVALID_ARG


def test_table_sizes_and_kernel_validation():
    p = se2.Plan([(32, 48, 16)], dtype="f32", host_only=True)
    assert p.table_bytes(0, [se2.GaussVM(0.05, 4.0)]) == 8 * (32 + 48 + 16)
    p64 = se2.Plan([(32, 48, 16)], dtype="f64", host_only=True)
    assert p64.table_bytes(0, [se2.GaussVM(0.05, 4.0), se2.GaussVM(0.1, 2.0)]) == 16 * (32 + 48 + 16)
    for bad in [se2.GaussVM(0.0, 4.0), se2.GaussVM(0.05, -1.0), se2.GaussVM(float("nan"), 1.0),
                se2.GaussVM(0.05, 4.0, norm=3)]:
        with pytest.raises(se2.Se2convError) as e:
            p.table_bytes(0, [bad])
        assert e.value.status == L.ERR_INVALID_ARG
    lib = L.load()
    d = L.KernelDesc()
    d.kind = L.K_SAMPLES  # null data pointer
    n = ctypes.c_size_t(0)
    assert lib.se2conv_coeffs(p.handle, 0, ctypes.byref(d), 1, None, ctypes.byref(n), None) == L.ERR_INVALID_ARG
    d.kind = L.K_RADIAL_PROFILE
    d.data = 16
    d.n_knots = 1
    d.r_max = 0.5
    assert lib.se2conv_coeffs(p.handle, 0, ctypes.byref(d), 1, None, ctypes.byref(n), None) == L.ERR_INVALID_ARG
    d.n_knots = 8
    d.r_max = 1.5
    assert lib.se2conv_coeffs(p.handle, 0, ctypes.byref(d), 1, None, ctypes.byref(n), None) == L.ERR_INVALID_ARG
    d.r_max = 0.5
    assert lib.se2conv_coeffs(p.handle, 0, ctypes.byref(d), 1, None, ctypes.byref(n), None) == L.OK
    assert n.value == 8 * 32 * 48 * 16
    d.kind = 9
    assert lib.se2conv_coeffs(p.handle, 0, ctypes.byref(d), 1, None, ctypes.byref(n), None) == L.ERR_INVALID_ARG
    assert lib.se2conv_coeffs(p.handle, 3, ctypes.byref(d), 1, None, ctypes.byref(n), None) == L.ERR_INVALID_ARG


def test_apply_validation_on_host_only_plan():
    lib = L.load()
    p = se2.Plan([(32, 32, 16)], dtype="f32", host_only=True)
    h = p.handle
    fake_table = 4096
    # bad shape index, batch, null and misaligned pointers, overlap, flags
    assert lib.se2conv_apply(h, 1, 256, fake_table, 512, 1, 0, None) == L.ERR_INVALID_ARG
    assert lib.se2conv_apply(h, 0, 256, fake_table, 512, 0, 0, None) == L.ERR_INVALID_ARG
    assert lib.se2conv_apply(h, 0, None, fake_table, 512, 1, 0, None) == L.ERR_INVALID_ARG
    assert lib.se2conv_apply(h, 0, 260, fake_table, 1 << 30, 1, 0, None) == L.ERR_INVALID_ARG
    assert lib.se2conv_apply(h, 0, 1 << 20, fake_table, (1 << 20) + 64, 1, 0, None) == L.ERR_INVALID_ARG
    assert lib.se2conv_apply(h, 0, 1 << 20, fake_table, 1 << 30, 1, 0x80, None) == L.ERR_INVALID_ARG
    # a table this plan did not produce
    assert lib.se2conv_apply(h, 0, 1 << 20, fake_table, 1 << 30, 1, 0, None) == L.ERR_INVALID_ARG
    assert b"not produced by this plan" in lib.se2conv_last_error()
    # in place is allowed (fails only on the table)
    assert lib.se2conv_apply(h, 0, 1 << 20, fake_table, 1 << 20, 1, 0, None) == L.ERR_INVALID_ARG
    # coefficient generation on a host-only plan: validated, then refused as device work
    d = L.KernelDesc()
    d.kind, d.sigma, d.kappa = L.K_GAUSS_VM, 0.05, 4.0
    n = ctypes.c_size_t(1 << 20)
    assert lib.se2conv_coeffs(h, 0, ctypes.byref(d), 1, 1 << 16, ctypes.byref(n), None) == L.ERR_DEVICE


def test_apply_padded_validation_on_host_only_plan():
    lib = L.load()
    p = se2.Plan([(32, 32, 16), (48, 40, 16), (24, 32, 16)], dtype="f32", host_only=True)
    h = p.handle
    fake_table = 4096
    ok_f, ok_out = 1 << 20, 1 << 30
    # shape indices out of range, an output grid coarser than the sampling grid
    assert lib.se2conv_apply_padded(h, 3, ok_f, fake_table, 1, ok_out, 1, 0, None) == L.ERR_INVALID_ARG
    assert lib.se2conv_apply_padded(h, 0, ok_f, fake_table, -1, ok_out, 1, 0, None) == L.ERR_INVALID_ARG
    assert lib.se2conv_apply_padded(h, 0, ok_f, fake_table, 2, ok_out, 1, 0, None) == L.ERR_INVALID_ARG
    assert b"coarser" in lib.se2conv_last_error()
    # batch, null / misaligned pointers, flags, overlap of input and output
    assert lib.se2conv_apply_padded(h, 0, ok_f, fake_table, 1, ok_out, 0, 0, None) == L.ERR_INVALID_ARG
    assert lib.se2conv_apply_padded(h, 0, None, fake_table, 1, ok_out, 1, 0, None) == L.ERR_INVALID_ARG
    assert lib.se2conv_apply_padded(h, 0, ok_f + 4, fake_table, 1, ok_out, 1, 0, None) == L.ERR_INVALID_ARG
    assert lib.se2conv_apply_padded(h, 0, ok_f, fake_table, 1, ok_out, 1, 0x80, None) == L.ERR_INVALID_ARG
    assert lib.se2conv_apply_padded(h, 0, ok_f, fake_table, 1, ok_f + 1024, 1, 0, None) == L.ERR_INVALID_ARG
    assert b"overlap" in lib.se2conv_last_error()
    # valid geometry: refused only because the table is not this plan's
    assert lib.se2conv_apply_padded(h, 0, ok_f, fake_table, 1, ok_out, 1, 0, None) == L.ERR_INVALID_ARG
    assert b"not produced by this plan" in lib.se2conv_last_error()


def test_chain_validation_on_host_only_plan():
    lib = L.load()
    p = se2.Plan([(32, 32, 16)], dtype="f32", host_only=True)
    arr = (L.Problem * 1)()
    tabs = (ctypes.c_void_p * 1)(4096)
    arr[0].shape_idx, arr[0].batch, arr[0].f, arr[0].out = 0, 1, 1 << 20, 1 << 30
    arr[0].tables = ctypes.cast(tabs, ctypes.POINTER(ctypes.c_void_p))
    arr[0].n_tables = 0
    assert lib.se2conv_chain(p.handle, arr, 1, 0, None) == L.ERR_INVALID_ARG
    arr[0].n_tables = 9
    assert lib.se2conv_chain(p.handle, arr, 1, 0, None) == L.ERR_INVALID_ARG
    arr[0].n_tables = 1
    assert lib.se2conv_chain(p.handle, arr, 1, 0, None) == L.ERR_INVALID_ARG  # foreign table
    assert lib.se2conv_chain(p.handle, arr, 0, 0, None) == L.ERR_INVALID_ARG
    assert lib.se2conv_chain(p.handle, arr, 1, L.GRAPH | L.TIMING, None) == L.ERR_INVALID_ARG


def test_pass_times_empty_on_fresh_plan():
    p = se2.Plan([(32, 32, 16)], dtype="f32", host_only=True)
    assert p.pass_times() == []


def test_corrupt_tuning_cache_falls_back_to_defaults(tmp_path, monkeypatch):
    # A tuning cache with malformed lines must not break plan creation.
    import subprocess
    import sys
    cache = tmp_path / "tune.jsonl"
    cache.write_text('{"nx":32,"ny":32,"m":16,"dtype":0,"w":8,"b":2,"x":2048}\n'
                     'garbage line\n{"nx":32,"ny":\n{"nx":32,"ny":32,"m":16,"dtype":0,"w":999,"b":2,"x":2048}\n')
    code = ("import paper_2504_05149_amd as se2; p = se2.Plan([(32, 32, 16)], host_only=True); "
            "print(p.table_bytes(0, [se2.GaussVM(0.05, 4.0)]))")
    env = dict(__import__("os").environ, SE2CONV_TUNE_CACHE=str(cache))
    res = subprocess.run([sys.executable, "-c", code], cwd=ROOT, env=env, capture_output=True, text=True)
    assert res.returncode == 0, res.stderr
    assert res.stdout.strip() == str(8 * (32 + 32 + 16))


def test_fused_entry_points_validate_on_host():
    lib = L.load()
    p = se2.Plan([(64, 64, 16)], dtype="f32", host_only=True)
    h = p.handle
    assert lib.se2conv_fused_supported(None, 0) == 0
    assert lib.se2conv_fused_supported(h, 0) == 0          # host-only plans run nothing
    assert lib.se2conv_fused_supported(h, 3) == 0
    assert lib.se2conv_field_spectra(None, 0, 256, 1, 512, None) == L.ERR_INVALID_ARG
    assert lib.se2conv_field_spectra(h, 2, 256, 1, 512, None) == L.ERR_INVALID_ARG
    assert lib.se2conv_field_spectra(h, 0, 256, 1, 512, None) == L.ERR_DEVICE
    # argument checks come before the device check
    assert lib.se2conv_apply_save(h, 0, 256, 4096, 512, 0, 1 << 30, None) == L.ERR_INVALID_ARG
    assert lib.se2conv_apply_save(h, 0, None, 4096, 512, 1, 1 << 30, None) == L.ERR_INVALID_ARG
    assert lib.se2conv_apply_save(h, 0, 1 << 20, 4096, 1 << 24, 1, 1 << 30, None) == L.ERR_DEVICE
    assert lib.se2conv_backward(h, 0, 1 << 20, 4096, 1 << 30, 0, 1 << 24, 1 << 28, None) == L.ERR_INVALID_ARG
    assert lib.se2conv_backward(h, 0, 1 << 20, 4096, 1 << 30, 1, 1 << 24, 1 << 28, None) == L.ERR_DEVICE
    assert b"host-only" in lib.se2conv_last_error()


def test_coeffs_sum_validation_on_host_only_plan():
    # a weighted sum of kernels is a FULL table; weights must be finite, 1..64 terms,
    # every term validated as in se2conv_coeffs; device work is refused on a host-only plan
    p = se2.Plan([(32, 48, 16)], dtype="f64", host_only=True)
    lib = L.load()
    descs = (L.KernelDesc * 2)()
    for dd, (s, k) in zip(descs, [(0.05, 4.0), (0.03, 9.0)]):
        dd.kind, dd.sigma, dd.kappa = L.K_GAUSS_VM, s, k
    w = (ctypes.c_double * 2)(0.7, 0.3)
    n = ctypes.c_size_t(0)
    assert lib.se2conv_coeffs_sum(p.handle, 0, descs, w, 2, None, ctypes.byref(n), None) == L.OK
    assert n.value == 16 * 32 * 48 * 16
    assert lib.se2conv_coeffs_sum(p.handle, 0, descs, None, 2, None, ctypes.byref(n), None) == L.ERR_INVALID_ARG
    assert lib.se2conv_coeffs_sum(p.handle, 0, descs, w, 0, None, ctypes.byref(n), None) == L.ERR_INVALID_ARG
    assert lib.se2conv_coeffs_sum(p.handle, 0, descs, w, 65, None, ctypes.byref(n), None) == L.ERR_INVALID_ARG
    assert lib.se2conv_coeffs_sum(p.handle, 1, descs, w, 2, None, ctypes.byref(n), None) == L.ERR_INVALID_ARG
    w[1] = float("inf")
    assert lib.se2conv_coeffs_sum(p.handle, 0, descs, w, 2, None, ctypes.byref(n), None) == L.ERR_INVALID_ARG
    w[1] = 0.3
    descs[1].sigma = -1.0
    assert lib.se2conv_coeffs_sum(p.handle, 0, descs, w, 2, None, ctypes.byref(n), None) == L.ERR_INVALID_ARG
    descs[1].sigma = 0.03
    n = ctypes.c_size_t(16 * 32 * 48 * 16)
    assert lib.se2conv_coeffs_sum(p.handle, 0, descs, w, 2, 1 << 16, ctypes.byref(n), None) == L.ERR_DEVICE


def test_table_release_and_counts_on_host_only_plan():
    import ctypes
    plan = se2.Plan([(32, 32, 16)], host_only=True)
    assert plan.counts() == (0, 0)
    lib = L.load()
    # an address the plan never produced
    assert lib.se2conv_table_release(plan.handle, ctypes.c_void_p(0x1000)) == L.ERR_INVALID_ARG
    assert lib.se2conv_table_release(plan.handle, None) == L.ERR_INVALID_ARG
    assert lib.se2conv_table_release(None, ctypes.c_void_p(0x1000)) == L.ERR_INVALID_ARG
    plan.close()


def test_shift_table_validation_on_host_only_plan():
    import ctypes
    plan = se2.Plan([(32, 32, 16)], host_only=True)
    lib = L.load()

    def size(shifts):
        arr = (L.Shift * len(shifts))(*[L.Shift(tx, ty, w, r) for tx, ty, r, w in shifts])
        nb = ctypes.c_size_t(0)
        st = lib.se2conv_shift_table(plan.handle, 0, arr, len(shifts), None, ctypes.byref(nb), None)
        return st, nb.value

    st, nb = size([(0.1, 0.2, 0, 1.0), (0.3, -0.1, 0, 0.5), (0.0, 0.1, 3, 2.0)])
    assert st == L.OK and nb == 2 * 32 * 32 * 16 * 8  # two distinct rolls, FP32 complex
    assert size([(0.1, 0.2, 16, 1.0)])[0] == L.ERR_INVALID_ARG          # roll outside [0, M)
    assert size([(0.1, 0.2, -1, 1.0)])[0] == L.ERR_INVALID_ARG
    assert size([(float("nan"), 0.2, 0, 1.0)])[0] == L.ERR_INVALID_ARG
    assert size([(0.1, 0.2, r, 1.0) for r in range(9)])[0] == L.ERR_INVALID_ARG   # 9 distinct rolls
    assert size([(0.1, 0.2, 0, 1.0)] * 65)[0] == L.ERR_INVALID_ARG                # 65 terms
    # a table the plan never produced is refused by the shifted apply
    tp = (ctypes.c_void_p * 1)(0x2000)
    assert lib.se2conv_apply_shifted(plan.handle, 0, ctypes.c_void_p(0x1000), ctypes.c_void_p(0x3000), tp, 1,
                                     ctypes.c_void_p(0x4000), 1, 0, None) == L.ERR_INVALID_ARG
    plan.close()


def test_table_quarter_validation_on_host_only_plan():
    plan = se2.Plan([(32, 32, 16)], host_only=True)
    lib = L.load()
    nb = ctypes.c_size_t(0)
    # only a FULL table this plan recorded can be folded
    assert lib.se2conv_table_quarter(plan.handle, ctypes.c_void_p(0x1000), None, ctypes.byref(nb),
                                     None) == L.ERR_INVALID_ARG
    assert "not produced by this plan" in lib.se2conv_last_error().decode()
    assert lib.se2conv_table_quarter(plan.handle, None, None, ctypes.byref(nb), None) == L.ERR_INVALID_ARG
    assert lib.se2conv_table_quarter(plan.handle, ctypes.c_void_p(0x1000), None, None, None) == L.ERR_INVALID_ARG
    assert lib.se2conv_table_quarter(None, ctypes.c_void_p(0x1000), None, ctypes.byref(nb),
                                     None) == L.ERR_INVALID_ARG
    plan.close()
