"""Host-side checks of the C ABI: the library loads, exports what include/dts.h declares,
and rejects bad arguments before touching the GPU (no kernel is launched here)."""
import ctypes
import os
import re

import pytest

import paper_1805_04590_amd as dts

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "dts.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(dts_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(dts.library_path()):
        pytest.fail("libdts.so is not built (run python -m paper_1805_04590_amd.build)")
    return dts.library()


def test_library_exports_every_declared_symbol(lib):
    names = declared_functions()
    assert len(names) >= 9
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(dts.EXPORTED_SYMBOLS)


def test_exported_symbols_are_in_dynamic_table():
    import subprocess
    out = subprocess.run(["nm", "-D", "--defined-only", dts.library_path()], capture_output=True,
                         text=True).stdout
    exported = set(re.findall(r"\bT (dts_\w+)", out))
    assert set(declared_functions()) <= exported


def test_strerror_covers_codes(lib):
    for code in (0, -1, -2, -3, -4, -5):
        assert lib.dts_strerror(code)
    assert b"unknown" in lib.dts_strerror(-99)


P = dts._Params


def test_workspace_sizes(lib):
    p = P(8.0, 0.2, 3, 10, 0.99, 0.99)
    small = lib.dts_solve_workspace_bytes(1, 256, 256, 1, ctypes.byref(p))
    big = lib.dts_solve_workspace_bytes(1, 1080, 1920, 1, ctypes.byref(p))
    assert small > 0 and big > small and small % 256 == 0 and big % 256 == 0
    # at least dx, dy and one temporary plane
    assert big >= 3 * 1080 * 1920 * 4
    assert lib.dts_filter_workspace_bytes(1, 256, 256, 1) < small
    assert lib.dts_solve_workspace_bytes(0, 256, 256, 1, ctypes.byref(p)) == 0
    assert lib.dts_solve_workspace_bytes(1, 256, 256, 17, ctypes.byref(p)) == 0
    assert lib.dts_filter_workspace_bytes(1, 256, 256 * 1024, 1) == 0


def _fake(n=1):
    return ctypes.c_void_p(0x1000 * n)


def test_filter_rejects_bad_arguments_without_launching(lib):
    ws = ctypes.c_void_p(0)
    f = lib.dts_filter
    assert f(None, 3, _fake(), _fake(2), 1, 1, 8, 8, 8.0, 0.2, 3, ws, 0, None) == dts.DTS_EINVAL
    assert f(_fake(), 0, _fake(), _fake(2), 1, 1, 8, 8, 8.0, 0.2, 3, ws, 0, None) == dts.DTS_EINVAL
    assert f(_fake(), 17, _fake(), _fake(2), 1, 1, 8, 8, 8.0, 0.2, 3, ws, 0, None) == dts.DTS_EINVAL
    assert f(_fake(), 3, _fake(), _fake(2), 1, 1, 0, 8, 8.0, 0.2, 3, ws, 0, None) == dts.DTS_EINVAL
    assert f(_fake(), 3, _fake(), _fake(2), 1, 1, 8, 8, -1.0, 0.2, 3, ws, 0, None) == dts.DTS_EINVAL
    assert f(_fake(), 3, _fake(), _fake(2), 1, 1, 8, 8, 8.0, 0.0, 3, ws, 0, None) == dts.DTS_EINVAL
    assert f(_fake(), 3, _fake(), _fake(2), 1, 1, 8, 8, 8.0, float("nan"), 3, ws, 0, None) == dts.DTS_EINVAL
    assert f(_fake(), 3, _fake(), _fake(2), 1, 1, 8, 8, 8.0, 0.2, 0, ws, 0, None) == dts.DTS_EINVAL
    assert f(_fake(), 3, _fake(), _fake(2), 1, 1, 8, 40000, 8.0, 0.2, 3, ws, 0, None) == dts.DTS_ENOTSUP
    # valid arguments but no / too small workspace
    assert f(_fake(), 3, _fake(), _fake(2), 1, 1, 8, 8, 8.0, 0.2, 3, ws, 0, None) == dts.DTS_EWORKSPACE
    assert f(_fake(), 3, _fake(), _fake(2), 1, 1, 8, 8, 8.0, 0.2, 3, _fake(3), 64, None) == dts.DTS_EWORKSPACE


def test_solve_rejects_bad_arguments_without_launching(lib):
    ws = ctypes.c_void_p(0)
    s = lib.dts_solve
    good = P(8.0, 0.2, 3, 10, 0.99, 0.99)

    def call(p=good, Cc=1, Ct=1, conf=_fake(3), out=_fake(4), H=8, W=8):
        return s(_fake(), 3, _fake(2), conf, Cc, Ct, 1, H, W, ctypes.byref(p), out, None, ws, 0, None)

    assert call(conf=None) == dts.DTS_EINVAL
    assert call(out=None) == dts.DTS_EINVAL
    assert call(Cc=2, Ct=3) == dts.DTS_EINVAL
    assert call(p=P(8.0, 0.2, 3, -1, 0.99, 0.99)) == dts.DTS_EINVAL
    assert call(p=P(8.0, 0.2, 0, 1, 0.99, 0.99)) == dts.DTS_EINVAL
    assert call(p=P(0.0, 0.2, 3, 1, 0.99, 0.99)) == dts.DTS_EINVAL
    assert call(p=P(8.0, 0.2, 3, 1, float("inf"), 0.99)) == dts.DTS_EINVAL
    assert call() == dts.DTS_EWORKSPACE
    assert call(Cc=3, Ct=3) == dts.DTS_EWORKSPACE
    assert s(_fake(), 3, _fake(2), _fake(3), 1, 1, 1, 8, 8, None, _fake(4), None, ws, 0, None) == dts.DTS_EINVAL


def test_tape_entry_points_reject_missing_buffers_without_launching(lib):
    ws = ctypes.c_void_p(0)
    good = P(8.0, 0.2, 3, 10, 0.99, 0.99)
    st = lib.dts_solve_tape
    # T > 0 needs both the checkpoints and the tape
    assert st(_fake(), 3, _fake(2), _fake(3), 1, 1, 1, 8, 8, ctypes.byref(good), _fake(4), None, _fake(5),
              ws, 0, None) == dts.DTS_EINVAL
    assert st(_fake(), 3, _fake(2), _fake(3), 1, 1, 1, 8, 8, ctypes.byref(good), _fake(4), _fake(5), None,
              ws, 0, None) == dts.DTS_EINVAL
    assert st(_fake(), 3, _fake(2), _fake(3), 1, 1, 1, 8, 8, ctypes.byref(good), _fake(4), _fake(5), _fake(6),
              ws, 0, None) == dts.DTS_EWORKSPACE
    bt = lib.dts_solve_backward_tape
    assert bt(_fake(), 3, _fake(2), _fake(3), 1, 1, 1, 8, 8, ctypes.byref(good), _fake(4), None, _fake(5),
              None, None, None, ws, 0, None) == dts.DTS_EINVAL
    assert bt(_fake(), 3, _fake(2), _fake(3), 1, 1, 1, 8, 8, ctypes.byref(good), _fake(4), _fake(6), _fake(5),
              None, None, None, ws, 0, None) == dts.DTS_EWORKSPACE
    assert st(_fake(), 3, _fake(2), _fake(3), 1, 1, 1, 8, 8, None, _fake(4), None, None, ws, 0, None) == \
        dts.DTS_EINVAL


def test_binding_refuses_cpu_tensors():
    import torch
    g = torch.zeros(3, 8, 8)
    with pytest.raises(ValueError, match="GPU"):
        dts.filter(g, g[:1], 8.0, 0.2)
    with pytest.raises(ValueError, match="GPU"):
        dts.solve(g, g[:1], g[:1], 8.0, 0.2)


def test_batched_variant_table(lib):
    import test_gpu_batched

    n = lib.dts_batched_variant_count()
    assert n == test_gpu_batched.N_BATCH_VARIANTS
    seen = set()
    for v in range(n):
        r, ct, px = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
        assert lib.dts_batched_variant_info(v, ctypes.byref(r), ctypes.byref(ct), ctypes.byref(px)) == 0
        assert r.value * 8 >= 64 and ct.value in (1, 2, 3, 4) and px.value > 0
        seen.add((r.value, ct.value, px.value))
    assert len(seen) == n
    assert lib.dts_batched_variant_info(n, ctypes.byref(r), ctypes.byref(ct), ctypes.byref(px)) != 0


def test_batched_rejects_unsupported_problems(lib):
    """Host-side checks of dts_batched_workspace_bytes (nothing is dereferenced)."""
    P = dts._Problem
    fake = 0x10000

    def table(**kw):
        q = dict(H=64, W=64, Cg=3, Ct=1, Cc=1, sigma_s=8.0, sigma_r=0.2, filter_iters=3, solver_iters=2)
        q.update(kw)
        arr = (P * 1)()
        arr[0] = P(fake, fake, fake, fake, q["H"], q["W"], q["Cg"], q["Ct"], q["Cc"], q["sigma_s"],
                   q["sigma_r"], q["filter_iters"], q["solver_iters"])
        return arr

    assert lib.dts_batched_workspace_bytes(table(), 1, 0) > 0
    assert lib.dts_batched_workspace_bytes(table(W=4096), 1, 0) > 0
    for bad in (dict(W=4097), dict(filter_iters=9), dict(solver_iters=0), dict(Cc=2), dict(Ct=17),
                dict(sigma_r=0.0), dict(H=0)):
        assert lib.dts_batched_workspace_bytes(table(**bad), 1, 0) == 0, bad
    assert lib.dts_batched_workspace_bytes(table(), 1, lib.dts_batched_variant_count()) == 0


def test_variance_confidence_rejects_bad_arguments_without_launching(lib):
    assert lib.dts_variance_confidence_workspace_bytes(1, 8, 8, 8) > 0
    assert lib.dts_variance_confidence_workspace_bytes(1, 8, 8, 9) == 0
    assert lib.dts_variance_confidence_workspace_bytes(0, 8, 8, 1) == 0
    fake = ctypes.c_void_p(0x10000)
    ws = ctypes.c_void_p(0x10000)
    # sigma_c <= 0, too many channels, null output: refused before any launch
    assert lib.dts_variance_confidence(fake, 3, fake, fake, 1, 1, 8, 8, 8.0, 0.2, 3, 0.0, ws, 1 << 20, None) == dts.DTS_EINVAL
    assert lib.dts_variance_confidence(fake, 3, fake, fake, 9, 1, 8, 8, 8.0, 0.2, 3, 0.1, ws, 1 << 20, None) == dts.DTS_EINVAL
    assert lib.dts_variance_confidence(fake, 3, fake, None, 1, 1, 8, 8, 8.0, 0.2, 3, 0.1, ws, 1 << 20, None) == dts.DTS_EINVAL
    assert lib.dts_variance_confidence(fake, 3, fake, fake, 1, 1, 8, 8, 8.0, 0.2, 3, 0.1, ws, 16, None) == dts.DTS_EWORKSPACE


def test_solve_stereo_rejects_bad_arguments_without_launching(lib):
    assert lib.dts_solve_stereo_workspace_bytes(1, 8, 8) > lib.dts_solve_workspace_bytes(1, 8, 8, 1, None)
    assert lib.dts_solve_stereo_workspace_bytes(0, 8, 8) == 0
    fake = ctypes.c_void_p(0x10000)
    p = dts.Params(8.0, 0.2, 3, 5).c()
    ok = lib.dts_solve_stereo_workspace_bytes(1, 8, 8)
    # epsilon <= 0, negative gamma, null output, too-small workspace: refused before any launch
    assert lib.dts_solve_stereo(fake, fake, 3, fake, fake, None, 1, 8, 8, ctypes.byref(p), 0.001, 0.0, fake, fake, ok, None) == dts.DTS_EINVAL
    assert lib.dts_solve_stereo(fake, fake, 3, fake, fake, None, 1, 8, 8, ctypes.byref(p), -1.0, 0.001, fake, fake, ok, None) == dts.DTS_EINVAL
    assert lib.dts_solve_stereo(fake, fake, 3, fake, fake, None, 1, 8, 8, ctypes.byref(p), 0.001, 0.001, None, fake, ok, None) == dts.DTS_EINVAL
    assert lib.dts_solve_stereo(fake, fake, 3, fake, fake, None, 1, 8, 8, ctypes.byref(p), 0.001, 0.001, fake, fake, ok - 256, None) == dts.DTS_EWORKSPACE



def test_support_rejects_bad_arguments_without_launching(lib):
    assert lib.dts_support_workspace_bytes(1, 8, 8) > 0
    assert lib.dts_support_workspace_bytes(0, 8, 8) == 0
    fake = ctypes.c_void_p(0x10000)
    other = ctypes.c_void_p(0x20000)
    ok = lib.dts_support_workspace_bytes(1, 8, 8)
    # null guide or output, bad channels or sigma, N = 0, confidence without an output or
    # aliasing the support, too-small workspace: refused before any launch
    assert lib.dts_support(None, 3, 1, 8, 8, 8.0, 0.2, 3, fake, None, 0, None, fake, ok, None) == dts.DTS_EINVAL
    assert lib.dts_support(fake, 3, 1, 8, 8, 8.0, 0.2, 3, None, None, 0, None, fake, ok, None) == dts.DTS_EINVAL
    assert lib.dts_support(fake, 17, 1, 8, 8, 8.0, 0.2, 3, fake, None, 0, None, fake, ok, None) == dts.DTS_EINVAL
    assert lib.dts_support(fake, 3, 1, 8, 8, 0.0, 0.2, 3, fake, None, 0, None, fake, ok, None) == dts.DTS_EINVAL
    assert lib.dts_support(fake, 3, 1, 8, 8, 8.0, 0.2, 0, fake, None, 0, None, fake, ok, None) == dts.DTS_EINVAL
    assert lib.dts_support(fake, 3, 1, 8, 8, 8.0, 0.2, 3, fake, other, 1, None, fake, ok, None) == dts.DTS_EINVAL
    assert lib.dts_support(fake, 3, 1, 8, 8, 8.0, 0.2, 3, fake, other, 0, other, fake, ok, None) == dts.DTS_EINVAL
    assert lib.dts_support(fake, 3, 1, 8, 8, 8.0, 0.2, 3, fake, other, 1, fake, fake, ok, None) == dts.DTS_EINVAL
    assert lib.dts_support(fake, 3, 1, 8, 8, 8.0, 0.2, 3, fake, None, 0, None, fake, ok - 256, None) == dts.DTS_EWORKSPACE
    assert lib.dts_support(fake, 3, 1, 0, 8, 8.0, 0.2, 3, fake, None, 0, None, fake, ok, None) == dts.DTS_EINVAL


def test_box_window_switch(lib):
    # process-wide launch choice, no device work: on, off, and back to the default
    assert lib.dts_tune_box_window(0) == 0
    assert lib.dts_tune_box_window(1) == 0


def test_box_rejects_bad_arguments_without_launching(lib):
    ok = lib.dts_box_workspace_bytes(1, 8, 8, 1, 3)
    assert ok > 0
    assert lib.dts_box_workspace_bytes(1, 8, 8, 1, 9) == 0      # at most 8 iterations
    assert lib.dts_box_workspace_bytes(1, 8, 8, 17, 3) == 0
    fake = ctypes.c_void_p(0x10000)
    other = ctypes.c_void_p(0x20000)
    # null pointers, aliasing, 9 iterations, a box wider than 255 pixels, too-small workspace
    assert lib.dts_filter_box(None, 3, fake, other, 1, 1, 8, 8, 8.0, 0.2, 3, fake, ok, None) == dts.DTS_EINVAL
    assert lib.dts_filter_box(fake, 3, other, other, 1, 1, 8, 8, 8.0, 0.2, 3, fake, ok, None) == dts.DTS_EINVAL
    assert lib.dts_filter_box(fake, 3, fake, other, 1, 1, 8, 8, 8.0, 0.2, 9, fake, ok, None) == dts.DTS_EINVAL
    big = lib.dts_box_workspace_bytes(1, 8, 8, 1, 1)
    assert lib.dts_filter_box(fake, 3, fake, other, 1, 1, 8, 8, 500.0, 0.2, 1, fake, big, None) == dts.DTS_ENOTSUP
    assert lib.dts_filter_box(fake, 3, fake, other, 1, 1, 8, 8, 8.0, 0.2, 3, fake, ok - 256, None) == dts.DTS_EWORKSPACE
    p = dts.Params(8.0, 0.2, 3, 5).c()
    assert lib.dts_solve_box(fake, 3, fake, fake, 1, 1, 1, 8, 8, ctypes.byref(p), fake, fake, ok, None) == dts.DTS_EINVAL
    assert lib.dts_solve_box(fake, 3, fake, other, 2, 1, 1, 8, 8, ctypes.byref(p), other, fake, ok, None) == dts.DTS_EINVAL
    assert lib.dts_box_codes(fake, 3, 1, 8, 8, 8.0, 0.0, fake, other, None) == dts.DTS_EINVAL
