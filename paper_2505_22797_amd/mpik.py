"""ctypes binding of the C ABI in include/mpik.h.

Argument marshalling only: every step of the operator runs in the HIP kernels
of libmpik.so.  torch provides device memory (plan and work buffers, inputs,
outputs) and the stream; the library itself never allocates.  The binding
raises if the shared library is missing -- there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os

import torch

_PKG_DIR = os.path.dirname(os.path.abspath(__file__))
# MPIK_LIBRARY selects another build of the library (a file name in this
# package, e.g. libmpik_check.so, or an absolute path); default libmpik.so.
_LIB_PATH = os.path.join(_PKG_DIR, os.environ.get("MPIK_LIBRARY") or "libmpik.so")
CHECK_LIBRARY = os.path.join(_PKG_DIR, "libmpik_check.so")
# (class, check word) of every plan of the bounds-checked build that closed
# with a check failed
CHECK_FAILURES: list[tuple[str, int]] = []

MPI_OK, MPI_ERR_ARG, MPI_ERR_DOMAIN, MPI_ERR_WORKSPACE = 0, -1, -2, -3
MPI_ERR_DTYPE, MPI_ERR_HIP, MPI_ERR_UNSUPPORTED, MPI_ERR_ALLOC = -4, -5, -6, -7
MPI_F32, MPI_F64 = 0, 1
CONV_MODES = {"auto": 0, "direct": 1, "fft": 2}
INTERPS = {"bilinear": 0, "cosine": 1}
CHANNELS = {"xy": 0, "x": 1}

EXPORTS = ("mpi_plan_bytes", "mpi_kernel_build", "mpi_forward", "mpi_adjoint", "mpi_iterate",
           "mpi_plan_info", "mpi_batch_bytes", "mpi_batch_build", "mpi_batch_count", "mpi_batch_offsets",
           "mpi_batch_info", "mpi_batch_forward", "mpi_batch_adjoint", "mpi_batch_pair", "mpi_batch_schedule",
           "mpi_batch_pair_noalloc", "mpi_batch_iterate",
           "mpi_batch_forward_dh", "mpi_batch_residual", "mpi_batch_traj_vjp", "mpi_batch_adjoint_step", "mpi_batch_denoise",
           "mpi_batch_dot", "mpi_batch_unrolled_vjp_bytes", "mpi_batch_unrolled_vjp",
           "mpi_batch_sample_order", "mpi_stage_count", "mpi_stage_name", "mpi_stage_launch",
           "mpi_batch_deconv_bytes", "mpi_batch_trace_conv", "mpi_batch_cg", "mpi_batch_trim_sigma", "mpi_batch_pnp",
           "mpi_batch_core_bytes", "mpi_batch_core_stage", "mpi_batch_field_trace", "mpi_velocity_forward_difference",
           "mpi_scale_trajectory", "mpi_reduce_lissajous", "mpi_vjp_forward", "mpi_vjp_adjoint",
           "mpi_checks_enabled", "mpi_plan_check", "mpi_debug_fail_alloc",
           "mpi_plan_destroy", "mpi_status_str", "mpi_abi_version")
MPI_BUILD_TUNE, MPI_BUILD_COL_SPLIT, MPI_BUILD_COL_WAVE, MPI_BUILD_DERIV = 1, 2, 4, 8
SLICE_FLAGS = {4: 16, 8: 32, 16: 64}        # MPI_BUILD_SLICES_4 / _8 / _16
NOALLOC_SCRATCH_BYTES = 64 << 20     # MPI_NOALLOC_SCRATCH_BYTES: the allocation-free pair's work memory


class MpiError(RuntimeError):
    def __init__(self, status: int, what: str):
        self.status = status
        super().__init__(f"{what}: {status_str(status)} ({status})")


class Problem(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("dtype", ctypes.c_int32), ("h", ctypes.c_double),
                ("radius", ctypes.c_int32), ("conv_mode", ctypes.c_int32), ("interp", ctypes.c_int32),
                ("channels", ctypes.c_int32), ("n_samples", ctypes.c_int64),
                ("r", ctypes.c_void_p), ("v", ctypes.c_void_p), ("grad_x", ctypes.c_double), ("grad_y", ctypes.c_double)]


class IterParams(ctypes.Structure):
    _fields_ = [("n_iter", ctypes.c_int32), ("tau", ctypes.c_double), ("denoise_sigma_px", ctypes.c_double),
                ("denoise_radius", ctypes.c_int32), ("use_graph", ctypes.c_int32)]


class PnpParams(ctypes.Structure):
    _fields_ = [("n_it", ctypes.c_int32), ("cg_max_iter", ctypes.c_int32), ("nu0", ctypes.c_double),
                ("cg_tol", ctypes.c_double), ("clip_percentile", ctypes.c_double),
                ("denoise_sigma_px", ctypes.c_double), ("denoise_radius", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]


_libs: dict[str, ctypes.CDLL] = {}
_current = [_LIB_PATH]


def lib() -> ctypes.CDLL:
    """The library calls go to: libmpik.so unless MPIK_LIBRARY or
    use_library chose another build.  Plans keep the library they were built
    with."""
    path = _current[-1]
    if path not in _libs:
        if not os.path.exists(path):
            raise RuntimeError(f"{path} is missing: build it with `python -m paper_2505_22797_amd.build`")
        _libs[path] = _load(path)
    return _libs[path]


class use_library:
    """Context manager: plans built inside use the library at `path` (e.g.
    CHECK_LIBRARY, the bounds-checked build) for their whole life."""

    def __init__(self, path: str):
        self.path = path

    def __enter__(self):
        _current.append(self.path)
        return lib()

    def __exit__(self, *exc):
        _current.pop()
        return False


def _load(path: str) -> ctypes.CDLL:
    L = ctypes.CDLL(path)
    vp, sz = ctypes.c_void_p, ctypes.c_size_t
    L.mpi_plan_bytes.argtypes = [ctypes.POINTER(Problem), ctypes.POINTER(sz), ctypes.POINTER(sz)]
    L.mpi_kernel_build.argtypes = [ctypes.POINTER(Problem), vp, sz, vp, ctypes.POINTER(vp)]
    L.mpi_forward.argtypes = [vp, vp, vp, vp, sz, vp]
    L.mpi_adjoint.argtypes = [vp, vp, vp, vp, sz, vp]
    L.mpi_iterate.argtypes = [vp, vp, vp, ctypes.POINTER(IterParams), vp, sz, vp]
    L.mpi_plan_info.argtypes = [vp, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32),
                                ctypes.POINTER(ctypes.c_int32)]
    i32p, i64p = ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int64)
    L.mpi_batch_bytes.argtypes = [ctypes.POINTER(Problem), ctypes.c_int, ctypes.c_int, ctypes.POINTER(sz),
                                  ctypes.POINTER(sz)]
    L.mpi_batch_build.argtypes = [ctypes.POINTER(Problem), ctypes.c_int, vp, sz, vp, sz, ctypes.c_int, vp,
                                  ctypes.POINTER(vp)]
    L.mpi_batch_count.argtypes = [vp]
    L.mpi_batch_offsets.argtypes = [vp, i64p, i64p]
    L.mpi_batch_info.argtypes = [vp, ctypes.c_int, i32p, i32p, i32p, i32p]
    L.mpi_batch_forward.argtypes = [vp, vp, vp, vp, sz, vp]
    L.mpi_batch_adjoint.argtypes = [vp, vp, vp, vp, sz, vp]
    L.mpi_batch_pair.argtypes = [vp, vp, vp, vp, vp, sz, vp]
    L.mpi_batch_pair_noalloc.argtypes = [vp, vp, vp, vp, vp]
    L.mpi_batch_schedule.argtypes = [vp, ctypes.c_int32, vp, vp, vp, vp, sz, vp, ctypes.POINTER(ctypes.c_int32)]
    L.mpi_batch_iterate.argtypes = [vp, vp, vp, ctypes.POINTER(IterParams), ctypes.POINTER(ctypes.c_double),
                                    vp, sz, vp]
    L.mpi_batch_forward_dh.argtypes = [vp, vp, vp, vp, sz, vp]
    L.mpi_batch_residual.argtypes = [vp, vp, vp, vp, vp, sz, vp]
    L.mpi_batch_traj_vjp.argtypes = [vp, vp, vp, vp, vp, vp, sz, vp]
    L.mpi_batch_adjoint_step.argtypes = [vp, vp, vp, vp, ctypes.POINTER(ctypes.c_double), vp, sz, vp]
    L.mpi_batch_denoise.argtypes = [vp, vp, vp, ctypes.c_double, ctypes.c_int, vp, sz, vp]
    L.mpi_batch_dot.argtypes = [vp, vp, vp, ctypes.c_int, ctypes.c_int, vp, vp, sz, vp]
    L.mpi_batch_sample_order.argtypes = [vp, ctypes.c_int, vp, vp, vp]
    L.mpi_batch_unrolled_vjp_bytes.argtypes = [vp, ctypes.c_int32, ctypes.POINTER(sz)]
    L.mpi_batch_unrolled_vjp.argtypes = [vp, vp, vp, ctypes.c_int32, ctypes.c_int32, ctypes.c_double,
                                         ctypes.c_int32, ctypes.POINTER(ctypes.c_double), vp, vp, vp, vp, vp, sz,
                                         vp, sz, vp]
    dp = ctypes.POINTER(ctypes.c_double)
    L.mpi_batch_deconv_bytes.argtypes = [vp, ctypes.POINTER(sz)]
    L.mpi_batch_trace_conv.argtypes = [vp, vp, vp, vp, sz, vp]
    L.mpi_batch_cg.argtypes = [vp, vp, vp, dp, ctypes.c_double, ctypes.c_int32, i32p, vp, sz, vp, sz, vp]
    L.mpi_batch_trim_sigma.argtypes = [vp, vp, ctypes.c_double, dp, dp, vp, sz, vp, sz, vp]
    L.mpi_batch_pnp.argtypes = [vp, vp, vp, ctypes.POINTER(PnpParams), i32p, dp, dp, vp, sz, vp, sz, vp]
    L.mpi_batch_core_bytes.argtypes = [vp, ctypes.POINTER(sz)]
    L.mpi_batch_core_stage.argtypes = [vp, vp, vp, ctypes.c_double, ctypes.c_double, ctypes.c_int32, i32p, vp, sz,
                                       vp, sz, vp]
    L.mpi_batch_field_trace.argtypes = [vp, vp, vp, vp]
    L.mpi_velocity_forward_difference.argtypes = [vp, vp, ctypes.c_int64, ctypes.c_double, ctypes.c_int32, vp]
    L.mpi_scale_trajectory.argtypes = [vp, vp, ctypes.c_int64, ctypes.c_double, ctypes.c_double, ctypes.c_int32,
                                       vp, vp, vp]
    L.mpi_reduce_lissajous.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp, sz, vp]
    L.mpi_vjp_forward.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp, sz, vp]
    L.mpi_vjp_adjoint.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp, sz, vp]
    L.mpi_stage_count.argtypes = [vp]
    L.mpi_stage_name.argtypes = [vp, ctypes.c_int]
    L.mpi_stage_name.restype = ctypes.c_char_p
    L.mpi_stage_launch.argtypes = [vp, ctypes.c_int, ctypes.c_int, vp, vp, vp, sz, vp]
    L.mpi_plan_destroy.argtypes = [vp]
    L.mpi_status_str.argtypes = [ctypes.c_int]
    L.mpi_status_str.restype = ctypes.c_char_p
    L.mpi_abi_version.argtypes = []
    L.mpi_checks_enabled.argtypes = []
    L.mpi_plan_check.argtypes = [vp, ctypes.POINTER(ctypes.c_int32), vp]
    L.mpi_debug_fail_alloc.argtypes = [ctypes.c_int32]
    for name in ("mpi_plan_bytes", "mpi_kernel_build", "mpi_forward", "mpi_adjoint", "mpi_iterate",
                 "mpi_plan_info", "mpi_batch_bytes", "mpi_batch_build", "mpi_batch_count", "mpi_batch_offsets",
                 "mpi_batch_info", "mpi_batch_forward", "mpi_batch_adjoint", "mpi_batch_pair",
                 "mpi_batch_pair_noalloc", "mpi_batch_schedule", "mpi_batch_iterate", "mpi_batch_forward_dh", "mpi_batch_residual", "mpi_batch_traj_vjp", "mpi_batch_adjoint_step", "mpi_batch_denoise",
                 "mpi_batch_dot", "mpi_batch_unrolled_vjp_bytes", "mpi_batch_unrolled_vjp",
                 "mpi_batch_sample_order", "mpi_stage_count", "mpi_stage_launch",
                 "mpi_batch_deconv_bytes", "mpi_batch_trace_conv", "mpi_batch_cg", "mpi_batch_trim_sigma",
                 "mpi_batch_pnp", "mpi_batch_core_bytes", "mpi_batch_core_stage", "mpi_batch_field_trace",
                 "mpi_velocity_forward_difference", "mpi_scale_trajectory", "mpi_reduce_lissajous",
                 "mpi_vjp_forward", "mpi_vjp_adjoint",
                 "mpi_checks_enabled", "mpi_plan_check", "mpi_debug_fail_alloc", "mpi_plan_destroy",
                 "mpi_abi_version"):
        getattr(L, name).restype = ctypes.c_int
    return L


def status_str(status: int) -> str:
    return lib().mpi_status_str(int(status)).decode()


def _check(rc: int, what: str):
    if rc != MPI_OK:
        raise MpiError(rc, what)


def _stream(stream) -> int:
    s = stream if stream is not None else torch.cuda.current_stream()
    return int(s.cuda_stream)


def _dtype_code(dt: torch.dtype) -> int:
    if dt == torch.float32:
        return MPI_F32
    if dt == torch.float64:
        return MPI_F64
    raise MpiError(MPI_ERR_DTYPE, f"dtype {dt}")


def problem(n: int, h: float, radius: int, r: torch.Tensor | None, v: torch.Tensor | None,
            n_samples: int | None = None, dtype: torch.dtype = torch.float32,
            conv_mode: str = "auto", interp: str = "bilinear", channels: str = "xy",
            grad=(1.0, 1.0)) -> Problem:
    p = Problem()
    p.n, p.h, p.radius = int(n), float(h), int(radius)
    p.dtype = _dtype_code(r.dtype if r is not None else dtype)
    p.conv_mode = CONV_MODES[conv_mode]
    p.interp = INTERPS[interp]
    p.channels = CHANNELS[channels]
    p.grad_x, p.grad_y = float(grad[0]), float(grad[1])
    p.n_samples = int(r.shape[0] if r is not None else n_samples)
    p.r = r.data_ptr() if r is not None else None
    p.v = v.data_ptr() if v is not None else None
    return p


def plan_bytes(prob: Problem) -> tuple[int, int]:
    pb, wb = ctypes.c_size_t(), ctypes.c_size_t()
    _check(lib().mpi_plan_bytes(ctypes.byref(prob), ctypes.byref(pb), ctypes.byref(wb)), "mpi_plan_bytes")
    return pb.value, wb.value


class Plan:
    """A built plan for one problem: kernel table/spectra and sample binning in
    device memory owned by this object, plus a reusable work buffer."""

    def __init__(self, n: int, h: float, radius: int, r: torch.Tensor, v: torch.Tensor,
                 conv_mode: str = "auto", stream=None, interp: str = "bilinear", channels: str = "xy",
                 grad=(1.0, 1.0)):
        self._L = lib()
        if not (r.is_cuda and v.is_cuda):
            raise ValueError("r and v must be device tensors")
        if r.dtype != v.dtype or r.shape != v.shape or r.ndim != 2 or r.shape[1] != 2:
            raise ValueError("r and v must be matching (T, 2) tensors")
        r = r.contiguous()
        v = v.contiguous()
        self.n, self.h, self.dtype, self.device = int(n), float(h), r.dtype, r.device
        self.n_samples = int(r.shape[0])
        self.interp = interp
        prob = problem(n, h, radius, r, v, conv_mode=conv_mode, interp=interp, channels=channels, grad=grad)
        pb, wb = plan_bytes(prob)
        self.plan_mem = torch.empty(pb, dtype=torch.uint8, device=r.device)
        self.work = torch.empty(wb, dtype=torch.uint8, device=r.device)
        handle = ctypes.c_void_p()
        _check(self._L.mpi_kernel_build(ctypes.byref(prob), self.plan_mem.data_ptr(), pb, _stream(stream),
                                      ctypes.byref(handle)), "mpi_kernel_build")
        self._h = handle
        rad, m, mode = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        _check(self._L.mpi_plan_info(self._h, ctypes.byref(rad), ctypes.byref(m), ctypes.byref(mode)), "mpi_plan_info")
        self.radius, self.fft_size = rad.value, m.value
        self.conv_mode = "fft" if mode.value == 2 else "direct"

    def _vec(self, t: torch.Tensor, shape, name):
        if t.dtype != self.dtype or t.device != self.device or tuple(t.shape) != tuple(shape) or not t.is_contiguous():
            raise ValueError(f"{name} must be a contiguous {self.dtype} tensor of shape {tuple(shape)} on {self.device}")
        return t

    def forward(self, c: torch.Tensor, s: torch.Tensor | None = None, stream=None) -> torch.Tensor:
        self._vec(c, (self.n, self.n), "c")
        if s is None:
            s = torch.empty((self.n_samples, 2), dtype=self.dtype, device=self.device)
        self._vec(s, (self.n_samples, 2), "s")
        _check(self._L.mpi_forward(self._h, c.data_ptr(), s.data_ptr(), self.work.data_ptr(), self.work.numel(),
                                 _stream(stream)), "mpi_forward")
        return s

    def adjoint(self, s: torch.Tensor, c: torch.Tensor | None = None, stream=None) -> torch.Tensor:
        self._vec(s, (self.n_samples, 2), "s")
        if c is None:
            c = torch.empty((self.n, self.n), dtype=self.dtype, device=self.device)
        self._vec(c, (self.n, self.n), "c")
        _check(self._L.mpi_adjoint(self._h, s.data_ptr(), c.data_ptr(), self.work.data_ptr(), self.work.numel(),
                                 _stream(stream)), "mpi_adjoint")
        return c

    def pair(self, c: torch.Tensor, s: torch.Tensor | None = None, g: torch.Tensor | None = None, stream=None):
        """s = A c and g = A^T s in one call (mpi_batch_pair on this one-problem plan)."""
        self._vec(c, (self.n, self.n), "c")
        if s is None:
            s = torch.empty((self.n_samples, 2), dtype=self.dtype, device=self.device)
        if g is None:
            g = torch.empty((self.n, self.n), dtype=self.dtype, device=self.device)
        self._vec(s, (self.n_samples, 2), "s")
        self._vec(g, (self.n, self.n), "g")
        _check(self._L.mpi_batch_pair(self._h, c.data_ptr(), s.data_ptr(), g.data_ptr(), self.work.data_ptr(),
                                    self.work.numel(), _stream(stream)), "mpi_batch_pair")
        return s, g

    def iterate(self, s: torch.Tensor, c: torch.Tensor, n_iter: int, tau: float,
                denoise_sigma_px: float = 0.0, denoise_radius: int = 2, use_graph: bool = True,
                stream=None) -> torch.Tensor:
        """In place on c: c <- D(c - tau A^T (A c - s)), n_iter times."""
        self._vec(s, (self.n_samples, 2), "s")
        self._vec(c, (self.n, self.n), "c")
        ip = IterParams(int(n_iter), float(tau), float(denoise_sigma_px), int(denoise_radius), int(bool(use_graph)))
        _check(self._L.mpi_iterate(self._h, s.data_ptr(), c.data_ptr(), ctypes.byref(ip), self.work.data_ptr(),
                                 self.work.numel(), _stream(stream)), "mpi_iterate")
        return c

    def stages(self) -> list[str]:
        n = self._L.mpi_stage_count(self._h)
        return [self._L.mpi_stage_name(self._h, k).decode() for k in range(n)]

    def launch_stage(self, stage: int, reps: int, c: torch.Tensor, s: torch.Tensor, stream=None):
        """Enqueue `reps` launches of one kernel of the forward/transpose sequence."""
        self._vec(c, (self.n, self.n), "c")
        self._vec(s, (self.n_samples, 2), "s")
        _check(self._L.mpi_stage_launch(self._h, int(stage), int(reps), c.data_ptr(), s.data_ptr(),
                                      self.work.data_ptr(), self.work.numel(), _stream(stream)), "mpi_stage_launch")

    def sample_order(self, stream=None):
        """(time index, base cell i0 | j0 << 16) of the samples in the order
        the plan holds them (int32 device tensors)."""
        order = torch.empty(self.n_samples, dtype=torch.int32, device=self.device)
        cell = torch.empty_like(order)
        _check(self._L.mpi_batch_sample_order(self._h, 0, order.data_ptr(), cell.data_ptr(), _stream(stream)),
               "mpi_batch_sample_order")
        return order, cell

    def check_word(self, stream=None) -> int:
        """OR of the problems' bounds-check words (nonzero only in the
        bounds-checked build, when a kernel met an index out of range)."""
        w = ctypes.c_int32()
        _check(self._L.mpi_plan_check(self._h, ctypes.byref(w), _stream(stream)), "mpi_plan_check")
        return w.value

    def close(self):
        if getattr(self, "_h", None):
            if self._L.mpi_checks_enabled():
                w = ctypes.c_int32()
                if self._L.mpi_plan_check(self._h, ctypes.byref(w), None) == MPI_OK and w.value:
                    CHECK_FAILURES.append((type(self).__name__, w.value))
            self._L.mpi_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Many independent problems in one plan; every stage is one launch over
    the whole batch.  Concentrations and signals of all problems live
    concatenated in one flat tensor each (see `c_offsets`, `s_offsets`)."""

    def __init__(self, specs, dtype=torch.float32, tune: bool = True, columns: str | None = None,
                 deriv: bool = False, stream=None, interp: str = "bilinear", channels: str = "xy",
                 grad=(1.0, 1.0), slices: int | None = None):
        """specs: list of (n, h, radius, r, v[, conv_mode[, interp]]) with r, v device (T, 2).
        columns: None (by batch size), "split" or "wave": shape of the column-FFT kernels.
        deriv: also build the dK/dh tables (for forward_dh) and the weight slopes.
        interp: "bilinear" or "cosine", for specs that do not name one.
        channels ("xy" or "x") and grad (the selection-field gradient) apply to every problem.
        slices (4, 8 or 16): the direct path's wave slices per tile, forced for every problem."""
        self._L = lib()
        keep = []
        arr = (Problem * len(specs))()
        for i, sp in enumerate(specs):
            n, h, radius, r, v = sp[:5]
            mode = sp[5] if len(sp) > 5 else "auto"
            ip = sp[6] if len(sp) > 6 else interp
            r = r.contiguous()
            v = v.contiguous()
            if r.dtype != dtype or v.dtype != dtype:
                raise ValueError("every problem of a batch shares the dtype")
            keep += [r, v]
            arr[i] = problem(n, h, radius, r, v, conv_mode=mode, interp=ip, channels=channels, grad=grad)
        self.interps = [sp[6] if len(sp) > 6 else interp for sp in specs]
        self.count = len(specs)
        self.dtype = dtype
        self.device = specs[0][3].device
        self.ns = [int(sp[0]) for sp in specs]
        self.ts = [int(sp[3].shape[0]) for sp in specs]
        flags = (MPI_BUILD_TUNE if tune else 0) | (MPI_BUILD_DERIV if deriv else 0) | {
            None: 0, "split": MPI_BUILD_COL_SPLIT, "wave": MPI_BUILD_COL_WAVE}[columns] | (
            SLICE_FLAGS[slices] if slices else 0)
        pb, wb = ctypes.c_size_t(), ctypes.c_size_t()
        _check(self._L.mpi_batch_bytes(arr, self.count, flags, ctypes.byref(pb), ctypes.byref(wb)), "mpi_batch_bytes")
        self.plan_mem = torch.empty(pb.value, dtype=torch.uint8, device=self.device)
        self.work = torch.empty(wb.value, dtype=torch.uint8, device=self.device)
        handle = ctypes.c_void_p()
        _check(self._L.mpi_batch_build(arr, self.count, self.plan_mem.data_ptr(), pb.value, self.work.data_ptr(),
                                     wb.value, flags, _stream(stream), ctypes.byref(handle)), "mpi_batch_build")
        self._h = handle
        co = (ctypes.c_int64 * (self.count + 1))()
        so = (ctypes.c_int64 * (self.count + 1))()
        _check(self._L.mpi_batch_offsets(self._h, co, so), "mpi_batch_offsets")
        self.c_offsets = list(co)
        self.s_offsets = list(so)
        self.info = []
        for b in range(self.count):
            rad, m, mode, sl = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
            _check(self._L.mpi_batch_info(self._h, b, ctypes.byref(rad), ctypes.byref(m), ctypes.byref(mode),
                                        ctypes.byref(sl)), "mpi_batch_info")
            self.info.append(dict(radius=rad.value, fft_size=m.value,
                                  conv_mode="fft" if mode.value == 2 else "direct", slices=sl.value))

    def stages(self) -> list[str]:
        n = self._L.mpi_stage_count(self._h)
        return [self._L.mpi_stage_name(self._h, k).decode() for k in range(n)]

    def launch_stage(self, stage: int, reps: int, c_all: torch.Tensor, s_all: torch.Tensor, stream=None):
        """Enqueue `reps` launches of one kernel of the forward/transpose sequence."""
        self._flat(c_all, self.c_offsets[-1], "c_all")
        self._flat(s_all, self.s_offsets[-1], "s_all")
        _check(self._L.mpi_stage_launch(self._h, int(stage), int(reps), c_all.data_ptr(), s_all.data_ptr(),
                                      self.work.data_ptr(), self.work.numel(), _stream(stream)), "mpi_stage_launch")

    def c_views(self, c_all):
        return [c_all[self.c_offsets[b]:self.c_offsets[b + 1]].view(self.ns[b], self.ns[b]) for b in range(self.count)]

    def s_views(self, s_all):
        return [s_all[self.s_offsets[b]:self.s_offsets[b + 1]].view(self.ts[b], 2) for b in range(self.count)]

    def _flat(self, t, n, name):
        if t.dtype != self.dtype or t.device != self.device or t.numel() != n or not t.is_contiguous():
            raise ValueError(f"{name} must be a contiguous {self.dtype} tensor of {n} elements")
        return t

    def forward(self, c_all, s_all=None, stream=None):
        self._flat(c_all, self.c_offsets[-1], "c_all")
        if s_all is None:
            s_all = torch.empty(self.s_offsets[-1], dtype=self.dtype, device=self.device)
        self._flat(s_all, self.s_offsets[-1], "s_all")
        _check(self._L.mpi_batch_forward(self._h, c_all.data_ptr(), s_all.data_ptr(), self.work.data_ptr(),
                                       self.work.numel(), _stream(stream)), "mpi_batch_forward")
        return s_all

    def adjoint(self, s_all, c_all=None, stream=None):
        self._flat(s_all, self.s_offsets[-1], "s_all")
        if c_all is None:
            c_all = torch.empty(self.c_offsets[-1], dtype=self.dtype, device=self.device)
        self._flat(c_all, self.c_offsets[-1], "c_all")
        _check(self._L.mpi_batch_adjoint(self._h, s_all.data_ptr(), c_all.data_ptr(), self.work.data_ptr(),
                                       self.work.numel(), _stream(stream)), "mpi_batch_adjoint")
        return c_all

    def pair(self, c_all, s_all=None, g_all=None, stream=None):
        """s_all = A c_all and g_all = A^T s_all in one call (mpi_batch_pair)."""
        self._flat(c_all, self.c_offsets[-1], "c_all")
        if s_all is None:
            s_all = torch.empty(self.s_offsets[-1], dtype=self.dtype, device=self.device)
        if g_all is None:
            g_all = torch.empty(self.c_offsets[-1], dtype=self.dtype, device=self.device)
        self._flat(s_all, self.s_offsets[-1], "s_all")
        self._flat(g_all, self.c_offsets[-1], "g_all")
        _check(self._L.mpi_batch_pair(self._h, c_all.data_ptr(), s_all.data_ptr(), g_all.data_ptr(),
                                    self.work.data_ptr(), self.work.numel(), _stream(stream)), "mpi_batch_pair")
        return s_all, g_all

    def schedule(self, ranges: int = -1, c_all=None, s_all=None, g_all=None, stream=None) -> int:
        """Problem ranges per FFT-size group: -1 reports the count in use, a
        positive count sets it.  0 (choosing it by timing) is switched off in
        the library and raises MpiError (MPI_ERR_UNSUPPORTED).  Results never
        depend on the count."""
        chosen = ctypes.c_int32()
        ptrs = [0, 0, 0]
        if ranges == 0:
            if c_all is None:
                c_all = torch.zeros(self.c_offsets[-1], dtype=self.dtype, device=self.device)
            if s_all is None:
                s_all = torch.empty(self.s_offsets[-1], dtype=self.dtype, device=self.device)
            if g_all is None:
                g_all = torch.empty(self.c_offsets[-1], dtype=self.dtype, device=self.device)
            self._flat(c_all, self.c_offsets[-1], "c_all")
            self._flat(s_all, self.s_offsets[-1], "s_all")
            self._flat(g_all, self.c_offsets[-1], "g_all")
            ptrs = [c_all.data_ptr(), s_all.data_ptr(), g_all.data_ptr()]
        _check(self._L.mpi_batch_schedule(self._h, int(ranges), *ptrs, self.work.data_ptr(), self.work.numel(),
                                          _stream(stream), ctypes.byref(chosen)), "mpi_batch_schedule")
        return chosen.value

    def pair_noalloc(self, c_all, s_all, g_all, stream=None):
        """As pair(), through the allocation-free entry (mpi_batch_pair_noalloc):
        the library's fixed per-GPU array serves as the work memory, so the
        outputs must be given.  Calls overlapping on one GPU race."""
        self._flat(c_all, self.c_offsets[-1], "c_all")
        self._flat(s_all, self.s_offsets[-1], "s_all")
        self._flat(g_all, self.c_offsets[-1], "g_all")
        _check(self._L.mpi_batch_pair_noalloc(self._h, c_all.data_ptr(), s_all.data_ptr(), g_all.data_ptr(),
                                            _stream(stream)), "mpi_batch_pair_noalloc")
        return s_all, g_all

    def iterate(self, s_all, c_all, n_iter, taus, denoise_sigma_px=0.0, denoise_radius=2, use_graph=True,
                stream=None):
        self._flat(s_all, self.s_offsets[-1], "s_all")
        self._flat(c_all, self.c_offsets[-1], "c_all")
        tarr = (ctypes.c_double * self.count)(*[float(t) for t in taus])
        ip = IterParams(int(n_iter), 0.0, float(denoise_sigma_px), int(denoise_radius), int(bool(use_graph)))
        _check(self._L.mpi_batch_iterate(self._h, s_all.data_ptr(), c_all.data_ptr(), ctypes.byref(ip), tarr,
                                       self.work.data_ptr(), self.work.numel(), _stream(stream)), "mpi_batch_iterate")
        return c_all

    # ---- derivative building blocks
    def forward_dh(self, x_all, s_all=None, stream=None):
        self._flat(x_all, self.c_offsets[-1], "x_all")
        if s_all is None:
            s_all = torch.empty(self.s_offsets[-1], dtype=self.dtype, device=self.device)
        self._flat(s_all, self.s_offsets[-1], "s_all")
        _check(self._L.mpi_batch_forward_dh(self._h, x_all.data_ptr(), s_all.data_ptr(), self.work.data_ptr(),
                                          self.work.numel(), _stream(stream)), "mpi_batch_forward_dh")
        return s_all

    def residual(self, c_all, y_all, out=None, stream=None):
        """A c - y, time order."""
        self._flat(c_all, self.c_offsets[-1], "c_all")
        self._flat(y_all, self.s_offsets[-1], "y_all")
        if out is None:
            out = torch.empty(self.s_offsets[-1], dtype=self.dtype, device=self.device)
        _check(self._L.mpi_batch_residual(self._h, c_all.data_ptr(), y_all.data_ptr(), out.data_ptr(),
                                        self.work.data_ptr(), self.work.numel(), _stream(stream)),
               "mpi_batch_residual")
        return out

    def traj_vjp(self, x_all, y_all, stream=None):
        self._flat(x_all, self.c_offsets[-1], "x_all")
        self._flat(y_all, self.s_offsets[-1], "y_all")
        g_r = torch.empty(self.s_offsets[-1], dtype=self.dtype, device=self.device)
        g_v = torch.empty_like(g_r)
        _check(self._L.mpi_batch_traj_vjp(self._h, x_all.data_ptr(), y_all.data_ptr(), g_r.data_ptr(), g_v.data_ptr(),
                                        self.work.data_ptr(), self.work.numel(), _stream(stream)),
               "mpi_batch_traj_vjp")
        return g_r, g_v

    def _vjp(self, fn, name, a, a_n, b, b_n, out_n, stream):
        self._flat(a, a_n, "input")
        self._flat(b, b_n, "upstream gradient")
        out = torch.empty(out_n, dtype=self.dtype, device=self.device)
        g_h = torch.empty(self.count, dtype=torch.float64, device=self.device)
        g_r = torch.empty(self.s_offsets[-1], dtype=self.dtype, device=self.device)
        g_v = torch.empty_like(g_r)
        _check(fn(self._h, a.data_ptr(), b.data_ptr(), out.data_ptr(), g_h.data_ptr(), g_r.data_ptr(),
                  g_v.data_ptr(), self.work.data_ptr(), self.work.numel(), _stream(stream)), name)
        return out, g_h, g_r, g_v

    def vjp_forward(self, c_all, gs_all, stream=None):
        """For s = A c: (A^T gs, <(dA/dh) c, gs> per problem, the sample
        position and velocity gradients of <gs, A c>)."""
        return self._vjp(self._L.mpi_vjp_forward, "mpi_vjp_forward", c_all, self.c_offsets[-1], gs_all,
                         self.s_offsets[-1], self.c_offsets[-1], stream)

    def vjp_adjoint(self, y_all, gc_all, stream=None):
        """For c' = A^T y: (A gc, <(dA/dh) gc, y> per problem, the sample
        position and velocity gradients of <y, A gc>)."""
        return self._vjp(self._L.mpi_vjp_adjoint, "mpi_vjp_adjoint", y_all, self.s_offsets[-1], gc_all,
                         self.c_offsets[-1], self.s_offsets[-1], stream)

    def adjoint_step(self, s_all, c_in, taus, c_out=None, stream=None):
        self._flat(s_all, self.s_offsets[-1], "s_all")
        self._flat(c_in, self.c_offsets[-1], "c_in")
        if c_out is None:
            c_out = torch.empty_like(c_in)
        tarr = (ctypes.c_double * self.count)(*[float(t) for t in taus])
        _check(self._L.mpi_batch_adjoint_step(self._h, s_all.data_ptr(), c_in.data_ptr(), c_out.data_ptr(), tarr,
                                            self.work.data_ptr(), self.work.numel(), _stream(stream)),
               "mpi_batch_adjoint_step")
        return c_out

    def denoise(self, u_all, sigma_px=0.5, radius=2, c_out=None, stream=None):
        self._flat(u_all, self.c_offsets[-1], "u_all")
        if c_out is None:
            c_out = torch.empty_like(u_all)
        _check(self._L.mpi_batch_denoise(self._h, u_all.data_ptr(), c_out.data_ptr(), float(sigma_px), int(radius),
                                       self.work.data_ptr(), self.work.numel(), _stream(stream)), "mpi_batch_denoise")
        return c_out

    def dot(self, a, b, space="signal", comp="both", out=None, stream=None):
        """Per-problem float64 dot products (device tensor of `count`)."""
        n = self.s_offsets[-1] if space == "signal" else self.c_offsets[-1]
        self._flat(a, n, "a")
        self._flat(b, n, "b")
        if out is None:
            out = torch.empty(self.count, dtype=torch.float64, device=self.device)
        _check(self._L.mpi_batch_dot(self._h, a.data_ptr(), b.data_ptr(), 0 if space == "signal" else 1,
                                   {"x": 0, "y": 1, "both": 2}[comp], out.data_ptr(), self.work.data_ptr(),
                                   self.work.numel(), _stream(stream)), "mpi_batch_dot")
        return out

    def unrolled_vjp(self, s_all, checkpoints, n_iter, every, taus, gbar, denoise_sigma_px=0.0, denoise_radius=2,
                     stream=None):
        """Reverse sweep of `n_iter` iteration steps from the checkpoints (a
        tensor of ceil(n_iter/every) concatenated concentration vectors).
        gbar (dL/dc_K) is overwritten with dL/dc_0.  Returns (g_h float64 per
        problem, g_r, g_v per sample in time order)."""
        self._flat(s_all, self.s_offsets[-1], "s_all")
        self._flat(gbar, self.c_offsets[-1], "gbar")
        nseg = (int(n_iter) + int(every) - 1) // int(every)
        self._flat(checkpoints, nseg * self.c_offsets[-1], "checkpoints")
        vb = ctypes.c_size_t()
        _check(self._L.mpi_batch_unrolled_vjp_bytes(self._h, int(every), ctypes.byref(vb)),
               "mpi_batch_unrolled_vjp_bytes")
        if getattr(self, "_vjp_work", None) is None or self._vjp_work.numel() < vb.value:
            self._vjp_work = torch.empty(vb.value, dtype=torch.uint8, device=self.device)
        g_h = torch.empty(self.count, dtype=torch.float64, device=self.device)
        g_r = torch.empty(self.s_offsets[-1], dtype=self.dtype, device=self.device)
        g_v = torch.empty_like(g_r)
        tarr = (ctypes.c_double * self.count)(*[float(t) for t in taus])
        _check(self._L.mpi_batch_unrolled_vjp(self._h, s_all.data_ptr(), checkpoints.data_ptr(), int(n_iter),
                                            int(every), float(denoise_sigma_px), int(denoise_radius), tarr,
                                            gbar.data_ptr(), g_h.data_ptr(), g_r.data_ptr(), g_v.data_ptr(),
                                            self.work.data_ptr(), self.work.numel(), self._vjp_work.data_ptr(),
                                            self._vjp_work.numel(), _stream(stream)), "mpi_batch_unrolled_vjp")
        return g_h, g_r, g_v

    # ---- the Deconvolution Stage (trace-kernel convolution, CG, ZeroShot-PnP)
    def _deconv_work(self):
        if getattr(self, "_dwork", None) is None:
            nb = ctypes.c_size_t()
            _check(self._L.mpi_batch_deconv_bytes(self._h, ctypes.byref(nb)), "mpi_batch_deconv_bytes")
            self._dwork = torch.empty(nb.value, dtype=torch.uint8, device=self.device)
        return self._dwork

    def trace_conv(self, x_all, out=None, stream=None):
        """C_b x_b for every problem (the trace-kernel convolution)."""
        self._flat(x_all, self.c_offsets[-1], "x_all")
        if out is None:
            out = torch.empty_like(x_all)
        _check(self._L.mpi_batch_trace_conv(self._h, x_all.data_ptr(), out.data_ptr(), self.work.data_ptr(),
                                          self.work.numel(), _stream(stream)), "mpi_batch_trace_conv")
        return out

    def cg(self, rhs_all, nus, tol=1e-3, max_iter=10000, x_out=None, stream=None):
        """CG on (C^T C + nu_b I) x = rhs from x = 0; returns (x, steps per problem)."""
        self._flat(rhs_all, self.c_offsets[-1], "rhs_all")
        if x_out is None:
            x_out = torch.empty_like(rhs_all)
        dw = self._deconv_work()
        nu = (ctypes.c_double * self.count)(*[float(v) for v in nus])
        it = (ctypes.c_int32 * self.count)()
        _check(self._L.mpi_batch_cg(self._h, rhs_all.data_ptr(), x_out.data_ptr(), nu, float(tol), int(max_iter), it,
                                  self.work.data_ptr(), self.work.numel(), dw.data_ptr(), dw.numel(), _stream(stream)),
               "mpi_batch_cg")
        return x_out, list(it)

    def trim_sigma(self, x_all, pct=5.0, stream=None):
        """In place: trim x below its pct-th percentile (pct < 0: no trim);
        returns (percentiles, sigmas) per problem."""
        self._flat(x_all, self.c_offsets[-1], "x_all")
        dw = self._deconv_work()
        q = (ctypes.c_double * self.count)()
        sg = (ctypes.c_double * self.count)()
        _check(self._L.mpi_batch_trim_sigma(self._h, x_all.data_ptr(), float(pct), q, sg, self.work.data_ptr(),
                                          self.work.numel(), dw.data_ptr(), dw.numel(), _stream(stream)),
               "mpi_batch_trim_sigma")
        return list(q), list(sg)

    def pnp(self, u_all, n_it=9, nu0=1e-5, tol=1e-3, max_iter=10000, clip_pct=5.0, sigma_px=0.5, radius=2,
            rho_out=None, stream=None):
        """ZeroShot-PnP deconvolution of the trace images; returns (rho, info)
        with per-pass CG steps, noise estimates and Tikhonov weights."""
        self._flat(u_all, self.c_offsets[-1], "u_all")
        if rho_out is None:
            rho_out = torch.empty_like(u_all)
        dw = self._deconv_work()
        prm = PnpParams(int(n_it), int(max_iter), float(nu0), float(tol), float(-1.0 if clip_pct is None else clip_pct),
                        float(0.0 if sigma_px is None else sigma_px), int(radius), 0)
        m = (n_it + 1) * self.count
        it, sg, nu = (ctypes.c_int32 * m)(), (ctypes.c_double * m)(), (ctypes.c_double * m)()
        _check(self._L.mpi_batch_pnp(self._h, u_all.data_ptr(), rho_out.data_ptr(), ctypes.byref(prm), it, sg, nu,
                                   self.work.data_ptr(), self.work.numel(), dw.data_ptr(), dw.numel(),
                                   _stream(stream)), "mpi_batch_pnp")
        B = self.count
        info = {"cg_steps": [[it[k * B + b] for k in range(n_it + 1)] for b in range(B)],
                "sigma": [[sg[k * B + b] for k in range(n_it + 1)] for b in range(B)],
                "nu": [[nu[k * B + b] for k in range(n_it + 1)] for b in range(B)]}
        return rho_out, info

    # ---- the Core Stage (variational field reconstruction) and the trace image
    def field_views(self, field_all):
        """Per-problem [3, N, N] views (channels xx, xy, yy) of a field buffer."""
        return [field_all[3 * self.c_offsets[b]:3 * self.c_offsets[b + 1]].view(3, n, n)
                for b, n in enumerate(self.ns)]

    def core_stage(self, s_all, gamma=1e-3, tol=1e-3, max_iter=10000, field_out=None, stream=None):
        """The field minimising the Core Stage functional for every problem;
        returns (field, CG steps per problem)."""
        self._flat(s_all, self.s_offsets[-1], "s_all")
        if field_out is None:
            field_out = torch.empty(3 * self.c_offsets[-1], dtype=self.dtype, device=self.device)
        self._flat(field_out, 3 * self.c_offsets[-1], "field_out")
        if getattr(self, "_cwork", None) is None:
            nb = ctypes.c_size_t()
            _check(self._L.mpi_batch_core_bytes(self._h, ctypes.byref(nb)), "mpi_batch_core_bytes")
            self._cwork = torch.empty(nb.value, dtype=torch.uint8, device=self.device)
        it = (ctypes.c_int32 * self.count)()
        _check(self._L.mpi_batch_core_stage(self._h, s_all.data_ptr(), field_out.data_ptr(), float(gamma), float(tol),
                                          int(max_iter), it, self.work.data_ptr(), self.work.numel(),
                                          self._cwork.data_ptr(), self._cwork.numel(), _stream(stream)),
               "mpi_batch_core_stage")
        return field_out, list(it)

    def field_trace(self, field_all, u_out=None, stream=None):
        """u = A_xx + A_yy per problem (concentration-shaped)."""
        self._flat(field_all, 3 * self.c_offsets[-1], "field_all")
        if u_out is None:
            u_out = torch.empty(self.c_offsets[-1], dtype=self.dtype, device=self.device)
        _check(self._L.mpi_batch_field_trace(self._h, field_all.data_ptr(), u_out.data_ptr(), _stream(stream)),
               "mpi_batch_field_trace")
        return u_out

    def reduce_lissajous(self, g_r, g_v, rho_all, nu_all, stream=None):
        """Per-problem amplitude gradients (float64 device tensors of `count`):
        dL/dax = sum_k g_r,x rho_x + g_v,x nu_x and dL/day likewise, from the
        per-sample gradients and the unit shapes (mpi_reduce_lissajous)."""
        n = self.s_offsets[-1]
        for t, name in ((g_r, "g_r"), (g_v, "g_v"), (rho_all, "rho_all"), (nu_all, "nu_all")):
            self._flat(t, n, name)
        gax = torch.empty(self.count, dtype=torch.float64, device=self.device)
        gay = torch.empty(self.count, dtype=torch.float64, device=self.device)
        _check(self._L.mpi_reduce_lissajous(self._h, g_r.data_ptr(), g_v.data_ptr(), rho_all.data_ptr(),
                                          nu_all.data_ptr(), gax.data_ptr(), gay.data_ptr(), self.work.data_ptr(),
                                          self.work.numel(), _stream(stream)), "mpi_reduce_lissajous")
        return gax, gay

    def sample_order(self, b, stream=None):
        """(time index, base cell i0 | j0 << 16) of problem b's samples in the
        order the plan holds them (int32 device tensors)."""
        order = torch.empty(self.ts[b], dtype=torch.int32, device=self.device)
        cell = torch.empty_like(order)
        _check(self._L.mpi_batch_sample_order(self._h, int(b), order.data_ptr(), cell.data_ptr(), _stream(stream)),
               "mpi_batch_sample_order")
        return order, cell

    def check_word(self, stream=None) -> int:
        """OR of the problems' bounds-check words (nonzero only in the
        bounds-checked build, when a kernel met an index out of range)."""
        w = ctypes.c_int32()
        _check(self._L.mpi_plan_check(self._h, ctypes.byref(w), _stream(stream)), "mpi_plan_check")
        return w.value

    def close(self):
        if getattr(self, "_h", None):
            if self._L.mpi_checks_enabled():
                w = ctypes.c_int32()
                if self._L.mpi_plan_check(self._h, ctypes.byref(w), None) == MPI_OK and w.value:
                    CHECK_FAILURES.append((type(self).__name__, w.value))
            self._L.mpi_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def velocity_forward_difference(r: torch.Tensor, dt: float, out: torch.Tensor | None = None, stream=None):
    """v_k = (r_{k+1} - r_k) / dt on the device (the last sample repeats the
    previous difference)."""
    if r.ndim != 2 or r.shape[1] != 2 or not r.is_cuda or not r.is_contiguous():
        raise ValueError("r must be a contiguous (T, 2) device tensor")
    if out is None:
        out = torch.empty_like(r)
    _check(lib().mpi_velocity_forward_difference(r.data_ptr(), out.data_ptr(), r.shape[0], float(dt),
                                                 _dtype_code(r.dtype), _stream(stream)),
           "mpi_velocity_forward_difference")
    return out


def scale_trajectory(rho: torch.Tensor, nu: torch.Tensor, ax: float, ay: float, stream=None):
    """r = (ax rho_x, ay rho_y), v = (ax nu_x, ay nu_y) on the device
    (mpi_scale_trajectory): the trajectory of amplitudes (ax, ay) over
    unit-amplitude shapes rho, nu, each product in float64 rounded once."""
    for t, name in ((rho, "rho"), (nu, "nu")):
        if t.ndim != 2 or t.shape[1] != 2 or not t.is_cuda or not t.is_contiguous():
            raise ValueError(f"{name} must be a contiguous (T, 2) device tensor")
    if nu.shape != rho.shape or nu.dtype != rho.dtype:
        raise ValueError("rho and nu must have the same shape and dtype")
    r = torch.empty_like(rho)
    v = torch.empty_like(nu)
    _check(lib().mpi_scale_trajectory(rho.data_ptr(), nu.data_ptr(), rho.shape[0], float(ax), float(ay),
                                      _dtype_code(rho.dtype), r.data_ptr(), v.data_ptr(), _stream(stream)),
           "mpi_scale_trajectory")
    return r, v

