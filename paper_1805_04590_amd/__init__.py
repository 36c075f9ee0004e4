"""MI355X (gfx950) hot path of the Domain Transform Solver (Bapat & Frahm, ECCV 2018).

Thin ctypes binding over ``libdts.so`` (C ABI declared in ``include/dts.h``).  This module
only marshals arguments: it checks dtypes, devices, shapes and contiguity, sizes and
allocates workspaces with PyTorch (device memory is PyTorch's, the stream is PyTorch's
current stream) and forwards raw device pointers.  Every step of the method runs in the
library's HIP kernels; there is no fallback path, and calls fail loudly when the library
is missing or a tensor is not on the GPU.

Entry points (same names as the C ABI):
  filter(guide, src, sigma_s, sigma_r, filter_iters=3)           edge-aware mean DT(src)
  variance_confidence(guide, z, sigma_s, sigma_r, sigma_c)        Eq. (7) confidence
  solve_stereo(left, right, target, conf, sigma_s, sigma_r, ...)  Eq. (11) disparity refinement
  solve(guide, target, conf, sigma_s, sigma_r, ...)               Eq. (3) gradient descent
  solve_backward(guide, target, conf, checkpoints, grad_out, ...) adjoint of solve
  DTSFunction.apply(guide, target, conf, params)                  autograd wrapper
Tensors are float32, contiguous, shaped [B][C][H][W] (or [C][H][W] for B = 1).
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import torch

__all__ = [
    "DTSError",
    "Params",
    "library",
    "library_path",
    "filter",
    "variance_confidence",
    "solve_stereo",
    "solve",
    "solve_backward",
    "solve_noalloc",
    "DTSFunction",
    "workspace_status",
    "distances",
    "row_pass",
    "col_pass",
    "profile_enable",
    "profile_read",
    "col_variants",
    "tune_col_variant",
    "tune_row_segment",
    "tune_box_window",
    "tune_col_xcd",
    "tune_spin_limit",
    "batched_variants",
    "BatchedSolver",
    "SolveGraph",
    "EXPORTED_SYMBOLS",
]

_PKG = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_PKG, "libdts.so")

DTS_OK = 0
DTS_EINVAL = -1
DTS_EWORKSPACE = -2
DTS_EHIP = -3
DTS_ENOTSUP = -4
DTS_EDEVICE = -5

EXPORTED_SYMBOLS = (
    "dts_filter_workspace_bytes",
    "dts_solve_workspace_bytes",
    "dts_solve_backward_workspace_bytes",
    "dts_filter",
    "dts_solve",
    "dts_solve_backward",
    "dts_solve_tape",
    "dts_solve_backward_tape",
    "dts_solve_noalloc",
    "dts_workspace_status",
    "dts_strerror",
    "dts_last_hip_error",
    "dts_solve_stereo_workspace_bytes",
    "dts_solve_stereo",
    "dts_variance_confidence_workspace_bytes",
    "dts_variance_confidence",
    "dts_support_workspace_bytes",
    "dts_box_workspace_bytes",
    "dts_box_codes",
    "dts_filter_box",
    "dts_solve_box",
    "dts_support",
    "dts_distances",
    "dts_pass_workspace_bytes",
    "dts_row_pass",
    "dts_col_pass",
    "dts_profile_enable",
    "dts_profile_read",
    "dts_col_variant_count",
    "dts_col_variant_info",
    "dts_tune_col_variant",
    "dts_tune_row_segment",
    "dts_tune_box_window",
    "dts_tune_col_xcd",
    "dts_tune_spin_limit",
    "dts_batched_variant_count",
    "dts_batched_variant_info",
    "dts_batched_workspace_bytes",
    "dts_batched_prepare",
    "dts_solve_batched",
)


class DTSError(RuntimeError):
    def __init__(self, code, what):
        self.code = code
        super().__init__(f"{what}: {_strerror(code)} ({code})")


class _Params(ctypes.Structure):
    _fields_ = [
        ("sigma_s", ctypes.c_float),
        ("sigma_r", ctypes.c_float),
        ("filter_iters", ctypes.c_int),
        ("solver_iters", ctypes.c_int),
        ("lam", ctypes.c_float),
        ("step", ctypes.c_float),
    ]


class _Problem(ctypes.Structure):
    _fields_ = [
        ("guide", ctypes.c_void_p),
        ("target", ctypes.c_void_p),
        ("conf", ctypes.c_void_p),
        ("out", ctypes.c_void_p),
        ("H", ctypes.c_int),
        ("W", ctypes.c_int),
        ("Cg", ctypes.c_int),
        ("Ct", ctypes.c_int),
        ("Cc", ctypes.c_int),
        ("sigma_s", ctypes.c_float),
        ("sigma_r", ctypes.c_float),
        ("filter_iters", ctypes.c_int),
        ("solver_iters", ctypes.c_int),
    ]


class _BatchedPlan(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int),
        ("variant", ctypes.c_int),
        ("n_phases", ctypes.c_int),
        ("total_tiles", ctypes.c_int),
        ("grid", ctypes.c_int),
        ("lam", ctypes.c_float),
        ("step", ctypes.c_float),
        ("workspace_bytes", ctypes.c_size_t),
        ("off_inst", ctypes.c_size_t),
        ("off_prefix", ctypes.c_size_t),
        ("off_tickets", ctypes.c_size_t),
    ]


class _KernelStat(ctypes.Structure):
    _fields_ = [
        ("name", ctypes.c_char * 48),
        ("launches", ctypes.c_int),
        ("total_ms", ctypes.c_double),
        ("bytes", ctypes.c_double),
    ]


@dataclass(frozen=True)
class Params:
    """Solver parameters; defaults are the paper's lambda = step = 0.99 (Sec. 4) and three
    filter iterations per edge-aware mean."""
    sigma_s: float
    sigma_r: float
    filter_iters: int = 3
    solver_iters: int = 10
    lam: float = 0.99
    step: float = 0.99

    def c(self):
        return _Params(float(self.sigma_s), float(self.sigma_r), int(self.filter_iters),
                       int(self.solver_iters), float(self.lam), float(self.step))


_lib = None


def library_path():
    return _LIB_PATH


def library():
    """Load libdts.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        raise RuntimeError(f"libdts.so not built at {_LIB_PATH}; run "
                           "`python -m paper_1805_04590_amd.build`")
    lib = ctypes.CDLL(_LIB_PATH)
    P = ctypes.POINTER(_Params)
    vp, fp, i, sz, f = ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int, ctypes.c_size_t, ctypes.c_float
    lib.dts_filter_workspace_bytes.argtypes = [i, i, i, i]
    lib.dts_filter_workspace_bytes.restype = sz
    lib.dts_solve_workspace_bytes.argtypes = [i, i, i, i, P]
    lib.dts_solve_workspace_bytes.restype = sz
    lib.dts_solve_backward_workspace_bytes.argtypes = [i, i, i, i, i, P]
    lib.dts_solve_backward_workspace_bytes.restype = sz
    lib.dts_filter.argtypes = [fp, i, fp, fp, i, i, i, i, f, f, i, vp, sz, vp]
    lib.dts_filter.restype = i
    lib.dts_solve.argtypes = [fp, i, fp, fp, i, i, i, i, i, P, fp, fp, vp, sz, vp]
    lib.dts_solve.restype = i
    lib.dts_solve_backward.argtypes = [fp, i, fp, fp, i, i, i, i, i, P, fp, fp, fp, fp, fp,
                                       vp, sz, vp]
    lib.dts_solve_backward.restype = i
    lib.dts_solve_tape.argtypes = [fp, i, fp, fp, i, i, i, i, i, P, fp, fp, fp, vp, sz, vp]
    lib.dts_solve_tape.restype = i
    lib.dts_solve_backward_tape.argtypes = [fp, i, fp, fp, i, i, i, i, i, P, fp, fp, fp, fp, fp, fp,
                                            vp, sz, vp]
    lib.dts_solve_backward_tape.restype = i
    lib.dts_solve_noalloc.argtypes = [fp, i, fp, fp, i, i, i, i, i, P, fp, fp, vp]
    lib.dts_solve_noalloc.restype = i
    lib.dts_solve_stereo_workspace_bytes.argtypes = [i, i, i]
    lib.dts_solve_stereo_workspace_bytes.restype = sz
    lib.dts_solve_stereo.argtypes = [fp, fp, i, fp, fp, fp, i, i, i, P, f, f, fp, vp, sz, vp]
    lib.dts_solve_stereo.restype = i
    lib.dts_variance_confidence_workspace_bytes.argtypes = [i, i, i, i]
    lib.dts_variance_confidence_workspace_bytes.restype = sz
    lib.dts_variance_confidence.argtypes = [fp, i, fp, fp, i, i, i, i, f, f, i, f, vp, sz, vp]
    lib.dts_variance_confidence.restype = i
    lib.dts_support_workspace_bytes.argtypes = [i, i, i]
    lib.dts_support_workspace_bytes.restype = sz
    lib.dts_support.argtypes = [fp, i, i, i, i, f, f, i, fp, fp, i, fp, vp, sz, vp]
    lib.dts_support.restype = i
    lib.dts_box_workspace_bytes.argtypes = [i, i, i, i, i]
    lib.dts_box_workspace_bytes.restype = sz
    lib.dts_box_codes.argtypes = [fp, i, i, i, i, f, f, vp, vp, vp]
    lib.dts_box_codes.restype = i
    lib.dts_filter_box.argtypes = [fp, i, fp, fp, i, i, i, i, f, f, i, vp, sz, vp]
    lib.dts_filter_box.restype = i
    lib.dts_solve_box.argtypes = [fp, i, fp, fp, i, i, i, i, i, P, fp, vp, sz, vp]
    lib.dts_solve_box.restype = i
    lib.dts_distances.argtypes = [fp, i, i, i, i, f, f, fp, fp, vp]
    lib.dts_distances.restype = i
    lib.dts_pass_workspace_bytes.argtypes = [i, i, i, i]
    lib.dts_pass_workspace_bytes.restype = sz
    lib.dts_row_pass.argtypes = [fp, fp, fp, i, i, i, i, f, i, i, vp]
    lib.dts_row_pass.restype = i
    lib.dts_col_pass.argtypes = [fp, fp, fp, i, i, i, i, f, i, i, vp, sz, vp]
    lib.dts_col_pass.restype = i
    ip = ctypes.POINTER(ctypes.c_int)
    lib.dts_col_variant_count.argtypes = []
    lib.dts_col_variant_count.restype = i
    lib.dts_col_variant_info.argtypes = [i, ip, ip, ip]
    lib.dts_col_variant_info.restype = i
    lib.dts_tune_col_variant.argtypes = [i, i]
    lib.dts_tune_col_variant.restype = i
    lib.dts_tune_row_segment.argtypes = [i]
    lib.dts_tune_row_segment.restype = i
    lib.dts_tune_box_window.argtypes = [i]
    lib.dts_tune_box_window.restype = i
    lib.dts_tune_col_xcd.argtypes = [i]
    lib.dts_tune_col_xcd.restype = i
    lib.dts_tune_spin_limit.argtypes = [i]
    lib.dts_tune_spin_limit.restype = i
    PP = ctypes.POINTER(_Problem)
    BP = ctypes.POINTER(_BatchedPlan)
    lib.dts_batched_variant_count.argtypes = []
    lib.dts_batched_variant_count.restype = i
    lib.dts_batched_variant_info.argtypes = [i, ip, ip, ip]
    lib.dts_batched_variant_info.restype = i
    lib.dts_batched_workspace_bytes.argtypes = [PP, i, i]
    lib.dts_batched_workspace_bytes.restype = sz
    lib.dts_batched_prepare.argtypes = [PP, i, f, f, i, vp, sz, BP, vp]
    lib.dts_batched_prepare.restype = i
    lib.dts_solve_batched.argtypes = [BP, vp, vp]
    lib.dts_solve_batched.restype = i
    lib.dts_profile_enable.argtypes = [i]
    lib.dts_profile_enable.restype = i
    lib.dts_profile_read.argtypes = [ctypes.POINTER(_KernelStat), i]
    lib.dts_profile_read.restype = i
    lib.dts_workspace_status.argtypes = [vp, vp]
    lib.dts_workspace_status.restype = i
    lib.dts_strerror.argtypes = [i]
    lib.dts_strerror.restype = ctypes.c_char_p
    lib.dts_last_hip_error.argtypes = []
    lib.dts_last_hip_error.restype = ctypes.c_char_p
    _lib = lib
    return lib


def _strerror(code):
    try:
        s = library().dts_strerror(int(code)).decode()
        if code == DTS_EHIP:
            s += " [" + library().dts_last_hip_error().decode() + "]"
        return s
    except Exception:  # pragma: no cover - only when the library cannot load at all
        return "error"


def _check(rc, what):
    if rc != DTS_OK:
        raise DTSError(rc, what)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _as4d(t, name):
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch.Tensor")
    if t.device.type != "cuda":
        raise ValueError(f"{name} must be a GPU tensor (got {t.device}); libdts runs on gfx950 only")
    if t.dtype != torch.float32:
        raise TypeError(f"{name} must be float32 (got {t.dtype})")
    if t.dim() == 3:
        t = t.unsqueeze(0)
    if t.dim() != 4:
        raise ValueError(f"{name} must be [B][C][H][W] or [C][H][W]")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return t


def _check_plane(t, name, shape, device):
    if (not isinstance(t, torch.Tensor) or tuple(t.shape) != tuple(shape) or t.device != device
            or t.dtype != torch.float32 or not t.is_contiguous()):
        raise ValueError(f"{name} must be a contiguous float32 {list(shape)} tensor on {device}")


def _check_image(t, name, B, H, W, device, channels=None):
    """t ([B][C][H][W], already through _as4d) matches the call's batch, image size and
    device, and has a channel count in `channels` (any if None)."""
    if t.shape[0] != B or tuple(t.shape[2:]) != (H, W) or t.device != device:
        raise ValueError(f"{name} must be [{B}][C][{H}][{W}] on {device} (got {list(t.shape)} on {t.device})")
    if channels is not None and t.shape[1] not in channels:
        raise ValueError(f"{name} must have {' or '.join(str(c) for c in sorted(set(channels)))} channels")


def _out_like(out, ref, name="out"):
    """The caller's output tensor, checked to be shaped and placed like `ref`."""
    o = _as4d(out, name)
    if o.shape != ref.shape or o.device != ref.device:
        raise ValueError(f"{name} must be {list(ref.shape)} on {ref.device} (got {list(o.shape)} on {o.device})")
    return o


def _finish(ws, internal, check, what):
    """Reads the workspace's device status (a bounded wait that gave up) when asked to, or
    by default when the workspace was allocated here and nobody else could read it."""
    if check or (check is None and internal):
        _check(library().dts_workspace_status(_ptr(ws), _stream()), what + " (device status)")


def _workspace(nbytes, device):
    if nbytes == 0:
        raise DTSError(DTS_EINVAL, "workspace size query")
    return torch.empty(int(nbytes), dtype=torch.uint8, device=device)


def distances(guide, sigma_s, sigma_r):
    """(dx, dy), each [B][H][W]: the transformed distances of Eq. (8)-(9)."""
    g = _as4d(guide, "guide")
    B, Cg, H, W = g.shape
    dx = torch.empty((B, H, W), dtype=torch.float32, device=g.device)
    dy = torch.empty_like(dx)
    _check(library().dts_distances(_ptr(g), Cg, B, H, W, float(sigma_s), float(sigma_r), _ptr(dx),
                                   _ptr(dy), _stream()), "dts_distances")
    return dx, dy


def row_pass(src, dx, sigma_s, iter, filter_iters=3, out=None):
    """One causal+anticausal recursive pass along rows for filter iteration ``iter``."""
    x = _as4d(src, "src")
    B, C, H, W = x.shape
    _check_plane(dx, "dx", (B, H, W), x.device)
    out = torch.empty_like(x) if out is None else _out_like(out, x)
    _check(library().dts_row_pass(_ptr(x), _ptr(out), _ptr(dx), C, B, H, W, float(sigma_s),
                                  int(iter), int(filter_iters), _stream()), "dts_row_pass")
    return out


def col_pass(src, dy, sigma_s, iter, filter_iters=3, out=None, workspace=None, check=None):
    """One causal+anticausal recursive pass along columns for filter iteration ``iter``.
    ``check``: read the workspace's device status afterwards (default: only when the
    workspace is allocated here)."""
    x = _as4d(src, "src")
    B, C, H, W = x.shape
    _check_plane(dy, "dy", (B, H, W), x.device)
    out = torch.empty_like(x) if out is None else _out_like(out, x)
    lib = library()
    internal = workspace is None
    if internal:
        workspace = _workspace(lib.dts_pass_workspace_bytes(B, H, W, C), x.device)
    _check(lib.dts_col_pass(_ptr(x), _ptr(out), _ptr(dy), C, B, H, W, float(sigma_s), int(iter),
                            int(filter_iters), _ptr(workspace), workspace.numel(), _stream()),
           "dts_col_pass")
    _finish(workspace, internal, check, "dts_col_pass")
    return out


def profile_enable(on=True):
    """Start (clearing earlier records) or stop timing every libdts kernel launch."""
    _check(library().dts_profile_enable(1 if on else 0), "dts_profile_enable")


def profile_read():
    """{kernel: {"launches", "total_ms", "avg_ms", "bytes_per_launch"}} of recorded launches."""
    rows = (_KernelStat * 64)()
    n = library().dts_profile_read(rows, 64)
    if n < 0:
        raise DTSError(n, "dts_profile_read")
    out = {}
    for r in rows[:min(n, 64)]:
        out[r.name.decode()] = dict(launches=r.launches, total_ms=r.total_ms,
                                    avg_ms=r.total_ms / max(r.launches, 1),
                                    bytes_per_launch=r.bytes / max(r.launches, 1))
    return out


def col_variants():
    """[(index, group_channels, rows_per_wave, waves)] of the column-pass shapes."""
    lib = library()
    out = []
    for v in range(lib.dts_col_variant_count()):
        ct, r, nw = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
        _check(lib.dts_col_variant_info(v, ctypes.byref(ct), ctypes.byref(r), ctypes.byref(nw)),
               "dts_col_variant_info")
        out.append((v, ct.value, r.value, nw.value))
    return out


def tune_col_variant(group_channels, variant):
    _check(library().dts_tune_col_variant(int(group_channels), int(variant)), "dts_tune_col_variant")


def tune_row_segment(pixels_per_lane):
    _check(library().dts_tune_row_segment(int(pixels_per_lane)), "dts_tune_row_segment")


def tune_box_window(on):
    """Run the box kernel's column passes with h <= 64 as one windowed kernel (default) or
    always through the wide-box kernels."""
    _check(library().dts_tune_box_window(int(bool(on))), "dts_tune_box_window")


def tune_col_xcd(on):
    """Keep every column strip's chunks on one XCD (default) or deal them round-robin."""
    _check(library().dts_tune_col_xcd(1 if on else 0), "dts_tune_col_xcd")


def tune_spin_limit(polls):
    """Bounded waits of the carry exchange: polls > 0 sets the bound, 0 the default, and
    polls < 0 makes every wait give up (to exercise the DTS_EDEVICE path)."""
    _check(library().dts_tune_spin_limit(int(polls)), "dts_tune_spin_limit")


def batched_variants():
    """[(index, rows_per_wave, group_channels, row_tile_pixels)] of the batched kernel's
    shapes."""
    lib = library()
    out = []
    for v in range(lib.dts_batched_variant_count()):
        r, ct, px = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
        _check(lib.dts_batched_variant_info(v, ctypes.byref(r), ctypes.byref(ct), ctypes.byref(px)),
               "dts_batched_variant_info")
        out.append((v, r.value, ct.value, px.value))
    return out


class BatchedSolver:
    """Many independent solves of uneven size in one persistent launch.

    ``problems`` is a list of dicts with GPU tensors ``guide`` [Cg][H][W], ``target``
    [Ct][H][W], ``conf`` [Cc][H][W] and floats ``sigma_s``, ``sigma_r`` plus ints
    ``filter_iters`` (default 3) and ``solver_iters`` (default 10).  Outputs are allocated
    here (``self.outputs``).  ``run()`` enqueues the solve on the current stream and is
    capturable; ``variant=None`` asks the autotuner."""

    def __init__(self, problems, lam=0.99, step=0.99, variant=None, tune_iters=2):
        self.problems = []
        for q in problems:
            g4, t4, c4 = (_as4d(q[k], k) for k in ("guide", "target", "conf"))
            if g4.shape[0] != 1 or t4.shape[0] != 1 or c4.shape[0] != 1:
                raise ValueError("a batched problem holds one image: [C][H][W] (or [1][C][H][W]) tensors")
            g, t, c = g4[0], t4[0], c4[0]
            if g.shape[1:] != t.shape[1:] or c.shape[1:] != t.shape[1:]:
                raise ValueError("guide/target/conf disagree in image size")
            if g.device != t.device or c.device != t.device:
                raise ValueError("guide/target/conf must be on one device")
            self.problems.append(dict(guide=g, target=t, conf=c, sigma_s=float(q["sigma_s"]),
                                      sigma_r=float(q["sigma_r"]),
                                      filter_iters=int(q.get("filter_iters", 3)),
                                      solver_iters=int(q.get("solver_iters", 10))))
        self.lam, self.step = float(lam), float(step)
        self.outputs = [torch.empty_like(q["target"]) for q in self.problems]
        if variant is None:
            from . import autotune
            variant = autotune.batched_variant(self, iters=tune_iters)
        self._prepare(int(variant))

    def _ctable(self):
        arr = (_Problem * len(self.problems))()
        for k, (q, o) in enumerate(zip(self.problems, self.outputs)):
            Cg, H, W = q["guide"].shape
            arr[k] = _Problem(q["guide"].data_ptr(), q["target"].data_ptr(), q["conf"].data_ptr(),
                              o.data_ptr(), H, W, Cg, q["target"].shape[0], q["conf"].shape[0],
                              q["sigma_s"], q["sigma_r"], q["filter_iters"], q["solver_iters"])
        return arr

    def _prepare(self, variant):
        lib = library()
        table = self._ctable()
        nbytes = lib.dts_batched_workspace_bytes(table, len(self.problems), variant)
        if nbytes == 0:
            raise DTSError(DTS_EINVAL, "dts_batched_workspace_bytes")
        self.workspace = torch.empty(int(nbytes), dtype=torch.uint8,
                                     device=self.problems[0]["target"].device)
        self.plan = _BatchedPlan()
        _check(lib.dts_batched_prepare(table, len(self.problems), self.lam, self.step, variant,
                                       _ptr(self.workspace), self.workspace.numel(),
                                       ctypes.byref(self.plan), _stream()),
               "dts_batched_prepare")
        self.variant = variant

    def run(self, check=False):
        """Enqueue the solves; ``check=True`` also waits for them and raises DTSError if a
        bounded wait inside the kernel gave up (not while capturing a graph)."""
        _check(library().dts_solve_batched(ctypes.byref(self.plan), _ptr(self.workspace), _stream()),
               "dts_solve_batched")
        if check:
            self.status()
        return self.outputs

    def status(self):
        return workspace_status(self.workspace)

    def capture(self):
        """A torch.cuda.CUDAGraph (a HIP graph) holding one run(); replay() repeats it."""
        graph = torch.cuda.CUDAGraph()
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            self.run()  # warm-up outside the graph on the capture stream
        torch.cuda.current_stream().wait_stream(side)
        torch.cuda.synchronize()
        with torch.cuda.graph(graph):
            self.run()
        return graph


class SolveGraph:
    """One dts_solve captured into a HIP graph (torch.cuda.CUDAGraph) for repeated solves of
    one shape: the launches of a small image cost more than its passes, and a replay
    issues them all at once.  The graph owns input, output and workspace buffers; copy new
    inputs into ``guide`` / ``target`` / ``conf`` and call ``replay()``, which returns
    ``out``.  Every launch of dts_solve only enqueues work and clears its workspace with
    kernels, so the captured graph holds no memset nodes."""

    def __init__(self, guide, target, conf, sigma_s, sigma_r, filter_iters=3, solver_iters=10, lam=0.99,
                 step=0.99):
        self.guide = _as4d(guide, "guide").clone()
        self.target = _as4d(target, "target").clone()
        self.conf = _as4d(conf, "conf").clone()
        B, Ct, H, W = self.target.shape
        self.args = (float(sigma_s), float(sigma_r), int(filter_iters), int(solver_iters), float(lam), float(step))
        p = Params(*self.args).c()
        self.out = torch.empty_like(self.target)
        self.workspace = _workspace(library().dts_solve_workspace_bytes(B, H, W, Ct, ctypes.byref(p)),
                                    self.target.device)
        self.graph = torch.cuda.CUDAGraph()
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            self._run()  # warm-up outside the graph on the capture stream
        torch.cuda.current_stream().wait_stream(side)
        torch.cuda.synchronize()
        with torch.cuda.graph(self.graph):
            self._run()

    def _run(self):
        solve(self.guide, self.target, self.conf, *self.args, out=self.out, workspace=self.workspace)

    def replay(self):
        self.graph.replay()
        return self.out


def workspace_status(ws):
    """DTS_OK, or raise DTSError(DTS_EDEVICE) if a kernel's bounded wait timed out."""
    _check(library().dts_workspace_status(_ptr(ws), _stream()), "device status")
    return DTS_OK


def filter(guide, src, sigma_s, sigma_r, filter_iters=3, out=None, workspace=None, check=None):
    """DT(src): the edge-aware domain-transform filter guided by ``guide`` (Sec. 3.2).
    ``check``: read the workspace's device status afterwards (default: only when the
    workspace is allocated here)."""
    g = _as4d(guide, "guide")
    x = _as4d(src, "src")
    B, Cs, H, W = x.shape
    _check_image(g, "guide", B, H, W, x.device)
    lib = library()
    out = torch.empty_like(x) if out is None else _out_like(out, x)
    internal = workspace is None
    if internal:
        workspace = _workspace(lib.dts_filter_workspace_bytes(B, H, W, Cs), x.device)
    rc = lib.dts_filter(_ptr(g), g.shape[1], _ptr(x), _ptr(out), Cs, B, H, W, float(sigma_s),
                        float(sigma_r), int(filter_iters), _ptr(workspace), workspace.numel(),
                        _stream())
    _check(rc, "dts_filter")
    _finish(workspace, internal, check, "dts_filter")
    return out if src.dim() == 4 else out[0]


def solve_stereo(left, right, target, conf, sigma_s, sigma_r, filter_iters=3, solver_iters=10,
                 lam=0.99, step=0.99, gamma=0.001, eps=0.001, out=None, workspace=None, check=None,
                 init=None):
    """Disparity refinement of Eq. (11) (Sec. 3.3): smoothness guided by ``left``, a
    Charbonnier target term and the photometric term against ``right``.  left/right
    [B][Cg][H][W] (or [Cg][H][W]); target/conf [B][1][H][W] (or [1][H][W]).  ``init``
    (shaped like target) restarts the descent from that iterate instead of the target."""
    L = _as4d(left, "left")
    R = _as4d(right, "right")
    t = _as4d(target, "target")
    c = _as4d(conf, "conf")
    B, Cg, H, W = L.shape
    if R.shape != L.shape or R.device != L.device:
        raise ValueError("left and right images differ in shape or device")
    if t.shape != (B, 1, H, W) or c.shape != (B, 1, H, W) or t.device != L.device or c.device != L.device:
        raise ValueError("target and conf must be [B][1][H][W] like the images, on their device")
    z0 = None
    if init is not None:
        z0 = _as4d(init, "init")
        if z0.shape != t.shape or z0.device != t.device:
            raise ValueError("init must be shaped like target, on its device")
    lib = library()
    out = torch.empty_like(t) if out is None else _out_like(out, t)
    internal = workspace is None
    if internal:
        nbytes = lib.dts_solve_stereo_workspace_bytes(B, H, W)
        if nbytes == 0:
            raise DTSError(DTS_EINVAL, "dts_solve_stereo_workspace_bytes")
        workspace = _workspace(nbytes, t.device)
    p = Params(sigma_s, sigma_r, filter_iters, solver_iters, lam, step).c()
    rc = lib.dts_solve_stereo(_ptr(L), _ptr(R), Cg, _ptr(t), _ptr(c), _ptr(z0), B, H, W, ctypes.byref(p),
                              float(gamma), float(eps), _ptr(out), _ptr(workspace), workspace.numel(),
                              _stream())
    _check(rc, "dts_solve_stereo")
    _finish(workspace, internal, check, "dts_solve_stereo")
    return out if target.dim() == 4 else out[0]


def variance_confidence(guide, z, sigma_s, sigma_r, sigma_c, filter_iters=3, out=None, workspace=None,
                        check=None):
    """Confidence from the edge-aware variance of z (Eq. (7)): exp(-(DT(z^2) - DT(z)^2) /
    (2 sigma_c^2)) per channel, DT guided by ``guide`` as in ``filter``.  ``out`` may be z."""
    g = _as4d(guide, "guide")
    x = _as4d(z, "z")
    B, C, H, W = x.shape
    _check_image(g, "guide", B, H, W, x.device)
    lib = library()
    out = torch.empty_like(x) if out is None else _out_like(out, x)
    internal = workspace is None
    if internal:
        nbytes = lib.dts_variance_confidence_workspace_bytes(B, H, W, C)
        if nbytes == 0:
            raise DTSError(DTS_EINVAL, "dts_variance_confidence_workspace_bytes")
        workspace = _workspace(nbytes, x.device)
    rc = lib.dts_variance_confidence(_ptr(g), g.shape[1], _ptr(x), _ptr(out), C, B, H, W,
                                     float(sigma_s), float(sigma_r), int(filter_iters),
                                     float(sigma_c), _ptr(workspace), workspace.numel(), _stream())
    _check(rc, "dts_variance_confidence")
    _finish(workspace, internal, check, "dts_variance_confidence")
    return out if z.dim() == 4 else out[0]


def box_codes(guide, sigma_s, sigma_r):
    """(qx, qy), each [B][H][W] int32 holding the uint32 codes round(256 d) that decide box
    membership (``dts_box_codes``)."""
    g = _as4d(guide, "guide")
    B, Cg, H, W = g.shape
    qx = torch.empty((B, H, W), dtype=torch.int32, device=g.device)
    qy = torch.empty_like(qx)
    _check(library().dts_box_codes(_ptr(g), Cg, B, H, W, float(sigma_s), float(sigma_r), _ptr(qx), _ptr(qy),
                                   _stream()), "dts_box_codes")
    return qx, qy


def filter_box(guide, src, sigma_s, sigma_r, filter_iters=3, out=None, workspace=None):
    """Edge-aware mean with the box kernel of Eq. (10) (``dts_filter_box``)."""
    g = _as4d(guide, "guide")
    x = _as4d(src, "src")
    B, C, H, W = x.shape
    _check_image(g, "guide", B, H, W, x.device)
    lib = library()
    out = torch.empty_like(x) if out is None else _out_like(out, x)
    if workspace is None:
        workspace = _workspace(lib.dts_box_workspace_bytes(B, H, W, C, int(filter_iters)), x.device)
    _check(lib.dts_filter_box(_ptr(g), g.shape[1], _ptr(x), _ptr(out), C, B, H, W, float(sigma_s),
                              float(sigma_r), int(filter_iters), _ptr(workspace), workspace.numel(),
                              _stream()), "dts_filter_box")
    return out if src.dim() == 4 else out[0]


def solve_box(guide, target, conf, sigma_s, sigma_r, filter_iters=3, solver_iters=10, lam=0.99, step=0.99,
              out=None, workspace=None):
    """z^T of the Eq. (3) descent with the box form of the edge-aware mean (``dts_solve_box``)."""
    g = _as4d(guide, "guide")
    t = _as4d(target, "target")
    c = _as4d(conf, "conf")
    B, Ct, H, W = t.shape
    _check_image(g, "guide", B, H, W, t.device)
    _check_image(c, "conf", B, H, W, t.device, (1, Ct))
    p = Params(sigma_s, sigma_r, filter_iters, solver_iters, lam, step).c()
    lib = library()
    out = torch.empty_like(t) if out is None else _out_like(out, t)
    if workspace is None:
        workspace = _workspace(lib.dts_box_workspace_bytes(B, H, W, Ct, int(filter_iters)), t.device)
    _check(lib.dts_solve_box(_ptr(g), g.shape[1], _ptr(t), _ptr(c), c.shape[1], Ct, B, H, W, ctypes.byref(p),
                             _ptr(out), _ptr(workspace), workspace.numel(), _stream()), "dts_solve_box")
    return out if target.dim() == 4 else out[0]


def support(guide, sigma_s, sigma_r, filter_iters=3, conf=None, out=None, conf_out=None,
            workspace=None, check=None):
    """Support of the edge-aware kernel relative to a flat region, s in (0, 1] per pixel
    ([B][H][W], or [H][W] for a 3-D guide).  With ``conf`` ([B][Cc][H][W]) also returns the
    support-weighted confidence conf / s (Sec. 3.1, after Eq. (6)) as (s, conf / s);
    ``conf_out`` may be ``conf``.  ``check``: read the workspace's device status afterwards
    (default: only when the workspace is allocated here)."""
    g = _as4d(guide, "guide")
    B, Cg, H, W = g.shape
    lib = library()
    if out is None:
        s_out = torch.empty((B, H, W), dtype=torch.float32, device=g.device)
    else:
        if out.numel() != B * H * W:
            raise ValueError("out must hold [B][H][W] values")
        s_out = _as4d(out.reshape(B, 1, H, W), "out")
    c = co = None
    Cc = 0
    if conf is not None:
        c = _as4d(conf, "conf")
        if c.shape[0] != B or c.shape[2:] != g.shape[2:]:
            raise ValueError("conf and guide disagree in batch or image size")
        Cc = c.shape[1]
        co = torch.empty_like(c) if conf_out is None else _as4d(conf_out, "conf_out")
        if co.shape != c.shape:
            raise ValueError("conf_out must have the shape of conf")
    internal = workspace is None
    if internal:
        nbytes = lib.dts_support_workspace_bytes(B, H, W)
        if nbytes == 0:
            raise DTSError(DTS_EINVAL, "dts_support_workspace_bytes")
        workspace = _workspace(nbytes, g.device)
    rc = lib.dts_support(_ptr(g), Cg, B, H, W, float(sigma_s), float(sigma_r), int(filter_iters),
                         _ptr(s_out), _ptr(c), Cc, _ptr(co), _ptr(workspace), workspace.numel(),
                         _stream())
    _check(rc, "dts_support")
    _finish(workspace, internal, check, "dts_support")
    sv = s_out.reshape(B, H, W) if guide.dim() == 4 else s_out.reshape(H, W)
    if c is None:
        return sv
    return sv, (co if conf.dim() == 4 else co[0])


def solve(guide, target, conf, sigma_s, sigma_r, filter_iters=3, solver_iters=10, lam=0.99,
          step=0.99, checkpoints=False, out=None, workspace=None, check=None, tape=False):
    """z^T of the Eq. (3) gradient descent started at z^0 = target.

    With ``checkpoints=True`` also returns the [T][B][Ct][H][W] tensor of iterates
    z^0..z^{T-1} that ``solve_backward`` consumes.  With ``tape=True`` (implies
    checkpoints) also returns the [T][2N-1][B][Ct][H][W] tensor of every iteration's
    filter-pass outputs (``dts_solve_tape``), which ``solve_backward(tape=...)`` reads
    instead of recomputing.  ``check``: wait for the solve and read the workspace's
    device status (default: only when the workspace is allocated here, since nobody else
    could read it); a caller passing ``workspace`` may read it later with
    ``workspace_status``."""
    g = _as4d(guide, "guide")
    t = _as4d(target, "target")
    c = _as4d(conf, "conf")
    B, Ct, H, W = t.shape
    _check_image(g, "guide", B, H, W, t.device)
    _check_image(c, "conf", B, H, W, t.device, (1, Ct))
    p = Params(sigma_s, sigma_r, filter_iters, solver_iters, lam, step).c()
    lib = library()
    out = torch.empty_like(t) if out is None else _out_like(out, t)
    ck = tp = None
    T = max(int(solver_iters), 0)
    if checkpoints or tape:
        ck = torch.empty((T,) + tuple(t.shape), dtype=torch.float32, device=t.device)
    if tape:
        tp = torch.empty((T, 2 * int(filter_iters) - 1) + tuple(t.shape), dtype=torch.float32,
                         device=t.device)
    internal = workspace is None
    if internal:
        workspace = _workspace(lib.dts_solve_workspace_bytes(B, H, W, Ct, ctypes.byref(p)), t.device)
    ckp = _ptr(ck) if ck is not None and ck.numel() else None
    if tape:
        rc = lib.dts_solve_tape(_ptr(g), g.shape[1], _ptr(t), _ptr(c), c.shape[1], Ct, B, H, W,
                                ctypes.byref(p), _ptr(out), ckp, _ptr(tp) if tp.numel() else None,
                                _ptr(workspace), workspace.numel(), _stream())
        _check(rc, "dts_solve_tape")
    else:
        rc = lib.dts_solve(_ptr(g), g.shape[1], _ptr(t), _ptr(c), c.shape[1], Ct, B, H, W,
                           ctypes.byref(p), _ptr(out), ckp, _ptr(workspace), workspace.numel(), _stream())
        _check(rc, "dts_solve")
    _finish(workspace, internal, check, "dts_solve")
    res = out if target.dim() == 4 else out[0]
    if tape:
        return res, ck, tp
    if checkpoints:
        return res, ck
    return res


def solve_noalloc(guide, target, conf, out, sigma_s, sigma_r, filter_iters=3, solver_iters=10, lam=0.99,
                  step=0.99, checkpoints=None):
    """``dts_solve_noalloc``: z^T into the caller's ``out`` (and the iterates into the caller's
    ``checkpoints``, [T][B][Ct][H][W], if given) with the library's own 64 MiB scratch in
    place of a workspace, so nothing is allocated here either; raises DTSError
    (DTS_ENOTSUP) above that size.  Calls on one device must not overlap."""
    g = _as4d(guide, "guide")
    t = _as4d(target, "target")
    c = _as4d(conf, "conf")
    o = _as4d(out, "out")
    B, Ct, H, W = t.shape
    if g.shape[0] != B or g.shape[2:] != t.shape[2:] or c.shape[0] != B or c.shape[2:] != t.shape[2:]:
        raise ValueError("guide/target/conf disagree in batch or image size")
    if o.shape != t.shape or o.device != t.device:
        raise ValueError("out must be a tensor shaped like target on its device")
    T = int(solver_iters)
    if checkpoints is not None:
        _check_plane(checkpoints, "checkpoints", (T,) + tuple(t.shape), t.device)
    p = Params(sigma_s, sigma_r, filter_iters, solver_iters, lam, step).c()
    rc = library().dts_solve_noalloc(_ptr(g), g.shape[1], _ptr(t), _ptr(c), c.shape[1], Ct, B, H, W,
                                     ctypes.byref(p), _ptr(o),
                                     _ptr(checkpoints) if checkpoints is not None and T else None, _stream())
    _check(rc, "dts_solve_noalloc")
    return out


def solve_backward(guide, target, conf, checkpoints, grad_out, sigma_s, sigma_r, filter_iters=3,
                   solver_iters=10, lam=0.99, step=0.99, need=(True, True, True),
                   workspace=None, check=None, tape=None):
    """(dL/dtarget, dL/dconf, dL/dguide) given dL/dz^T and the checkpoints of ``solve``.
    With ``tape`` (from ``solve(tape=True)``) the filter-pass inputs are read from it
    instead of recomputed (``dts_solve_backward_tape``).  ``check`` as for ``solve``."""
    g = _as4d(guide, "guide")
    t = _as4d(target, "target")
    c = _as4d(conf, "conf")
    go = _as4d(grad_out, "grad_out")
    B, Ct, H, W = t.shape
    _check_image(g, "guide", B, H, W, t.device)
    _check_image(c, "conf", B, H, W, t.device, (1, Ct))
    if go.shape != t.shape or go.device != t.device:
        raise ValueError(f"grad_out must be {list(t.shape)} on {t.device} like the target")
    T = int(solver_iters)
    if checkpoints.shape != (T,) + tuple(t.shape) or checkpoints.dtype != torch.float32 \
            or not checkpoints.is_contiguous() or checkpoints.device != t.device:
        raise ValueError("checkpoints must be the [T][B][Ct][H][W] float32 tensor from solve()")
    if tape is not None and (tape.shape != (T, 2 * int(filter_iters) - 1) + tuple(t.shape)
                             or tape.dtype != torch.float32 or not tape.is_contiguous()
                             or tape.device != t.device):
        raise ValueError("tape must be the [T][2N-1][B][Ct][H][W] float32 tensor from solve(tape=True)")
    p = Params(sigma_s, sigma_r, filter_iters, solver_iters, lam, step).c()
    lib = library()
    gt = torch.empty_like(t) if need[0] else None
    gc = torch.empty_like(c) if need[1] else None
    gg = torch.empty_like(g) if need[2] else None
    internal = workspace is None
    if internal:
        workspace = _workspace(lib.dts_solve_backward_workspace_bytes(
            B, H, W, g.shape[1], Ct, ctypes.byref(p)), t.device)
    if tape is not None:
        rc = lib.dts_solve_backward_tape(_ptr(g), g.shape[1], _ptr(t), _ptr(c), c.shape[1], Ct, B, H, W,
                                         ctypes.byref(p), _ptr(checkpoints) if T else None,
                                         _ptr(tape) if T else None, _ptr(go), _ptr(gt), _ptr(gc), _ptr(gg),
                                         _ptr(workspace), workspace.numel(), _stream())
        _check(rc, "dts_solve_backward_tape")
    else:
        rc = lib.dts_solve_backward(_ptr(g), g.shape[1], _ptr(t), _ptr(c), c.shape[1], Ct, B, H, W,
                                    ctypes.byref(p), _ptr(checkpoints) if T else None, _ptr(go),
                                    _ptr(gt), _ptr(gc), _ptr(gg), _ptr(workspace), workspace.numel(),
                                    _stream())
        _check(rc, "dts_solve_backward")
    _finish(workspace, internal, check, "dts_solve_backward")
    squeeze = target.dim() == 3
    fix = (lambda x: x[0] if (x is not None and squeeze) else x)
    return fix(gt), fix(gc), fix(gg)


class DTSFunction(torch.autograd.Function):
    """z^T = solve(guide, target, conf) with gradients for all three inputs through the
    hand-written adjoint (per-iteration checkpoints, recomputed filter passes).
    ``apply(guide, target, conf, params, check=True, tape=False)``: with ``check`` the
    forward and the backward each wait for their kernels and raise DTSError if a bounded
    wait inside them gave up; ``check=False`` keeps both fully asynchronous.  With
    ``tape`` the forward also keeps every filter pass's output (2N - 1 signals per
    iteration) and the backward reads them instead of recomputing them."""

    @staticmethod
    def forward(ctx, guide, target, conf, params: Params, check=True, tape=False):
        res = solve(guide, target, conf, params.sigma_s, params.sigma_r, params.filter_iters,
                    params.solver_iters, params.lam, params.step, checkpoints=True,
                    check=bool(check), tape=bool(tape))
        if tape:
            z, ck, tp = res
            ctx.save_for_backward(guide, target, conf, ck, tp)
        else:
            z, ck = res
            ctx.save_for_backward(guide, target, conf, ck)
        ctx.params = params
        ctx.check = bool(check)
        ctx.tape = bool(tape)
        return z

    @staticmethod
    def backward(ctx, grad_z):
        saved = ctx.saved_tensors
        guide, target, conf, ck = saved[:4]
        tp = saved[4] if ctx.tape else None
        p = ctx.params
        need = ctx.needs_input_grad[:3]
        gt, gc, gg = solve_backward(guide, target, conf, ck, grad_z.contiguous(), p.sigma_s,
                                    p.sigma_r, p.filter_iters, p.solver_iters, p.lam, p.step,
                                    need=(need[1], need[2], need[0]), check=ctx.check, tape=tp)
        return gg, gt, gc, None, None, None
