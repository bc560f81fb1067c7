"""C-ABI checks that need no GPU: the library loads, exports every function the
header declares, and rejects bad descriptors on the host before any device
work is enqueued."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mpik.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(mpi_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def mpik():
    from paper_2505_22797_amd import mpik as m
    m.lib()
    return m


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("mpi_kernel_build", "mpi_forward", "mpi_adjoint", "mpi_iterate", "mpi_plan_bytes"):
        assert required in names


def test_library_exports_every_declared_symbol(mpik):
    lib = mpik.lib()
    for name in declared_functions():
        assert hasattr(lib, name), name
    assert set(mpik.EXPORTS) == set(declared_functions())


def test_abi_version_and_status_strings(mpik):
    assert mpik.lib().mpi_abi_version() == 2
    seen = set()
    for code in (0, -1, -2, -3, -4, -5, -6, -7):
        s = mpik.status_str(code)
        assert s and s != "unknown status"
        seen.add(s)
    assert len(seen) == 8
    assert mpik.status_str(-99) == "unknown status"


def _prob(mpik, **kw):
    base = dict(n=64, h=0.01, radius=31, r=None, v=None, n_samples=1000)
    base.update(kw)
    return mpik.problem(base["n"], base["h"], base["radius"], None, None, n_samples=base["n_samples"],
                        conv_mode=base.get("conv_mode", "auto"))


def test_plan_bytes_valid(mpik):
    pb, wb = mpik.plan_bytes(_prob(mpik))
    assert pb > 0 and wb > 0 and pb % 256 == 0 and wb % 256 == 0
    # the FFT path needs its column buffers, the direct path does not
    pf, wf = mpik.plan_bytes(_prob(mpik, conv_mode="fft"))
    pd, wd = mpik.plan_bytes(_prob(mpik, conv_mode="direct"))
    assert wf > wd


def _batch_bytes(mpik, probs, flags=0):
    arr = (mpik.Problem * len(probs))(*probs)
    pb, wb = ctypes.c_size_t(), ctypes.c_size_t()
    assert mpik.lib().mpi_batch_bytes(arr, len(probs), flags, ctypes.byref(pb), ctypes.byref(wb)) == 0
    return pb.value, wb.value


def test_batch_bytes_share_kernel_tables(mpik):
    """Problems with the same N, R, h, gradient and requested path keep one
    copy of the kernel tables: the plan shrinks by exactly the duplicated
    spectra and twiddles (FFT path) or taps (direct path), 256-byte aligned;
    the work memory, per problem, does not."""
    al = lambda x: (x + 255) // 256 * 256
    for kw, table in ((dict(n=64, radius=63, conv_mode="fft"), al(3 * 65 * 65 * 4) + al(128 * 2 * 4)),
                      (dict(n=40, radius=9, conv_mode="direct"), al(3 * 19 * 20 * 4))):
        same = [_prob(mpik, n_samples=t, **kw) for t in (1000, 1500, 800)]
        distinct = [_prob(mpik, n_samples=t, h=h, **kw) for t, h in ((1000, 0.01), (1500, 0.0101), (800, 0.0102))]
        ps, ws = _batch_bytes(mpik, same)
        pd, wd = _batch_bytes(mpik, distinct)
        assert ws == wd and pd - ps == 2 * table, (kw, pd - ps, table)
        # a problem that asks for another path keeps tables of its own: those of
        # its single plan, which differ from the shared ones by its plan's size
        mixed = same[:2] + [_prob(mpik, n_samples=800, **dict(kw, conv_mode="auto"))]
        own = table + _batch_bytes(mpik, mixed[2:])[0] - _batch_bytes(mpik, same[2:])[0]
        assert _batch_bytes(mpik, mixed)[0] == ps + own, kw


@pytest.mark.parametrize("field,value,code", [
    ("n", 1, -1), ("n", 2000, -1), ("h", 0.0, -1), ("h", float("nan"), -1), ("radius", -1, -1),
    ("n_samples", 0, -1), ("dtype", 7, -4), ("conv_mode", 9, -1), ("interp", 2, -1), ("interp", -1, -1),
    ("channels", 2, -1), ("grad_x", float("inf"), -1), ("grad_y", 0.0, -1),
])
def test_plan_bytes_rejects(mpik, field, value, code):
    p = _prob(mpik)
    setattr(p, field, value)
    pb, wb = ctypes.c_size_t(), ctypes.c_size_t()
    assert mpik.lib().mpi_plan_bytes(ctypes.byref(p), ctypes.byref(pb), ctypes.byref(wb)) == code


def test_channels_and_gradients_accepted(mpik):
    pb, wb = ctypes.c_size_t(), ctypes.c_size_t()
    for ch, gx, gy in ((1, 1.39, -3.16), (0, 0.0, 0.0), (0, -1.0, -1.0)):
        p = _prob(mpik)
        p.channels, p.grad_x, p.grad_y = ch, gx, gy
        assert mpik.lib().mpi_plan_bytes(ctypes.byref(p), ctypes.byref(pb), ctypes.byref(wb)) == 0


def test_both_interpolators_accepted(mpik):
    pb, wb = ctypes.c_size_t(), ctypes.c_size_t()
    sizes = []
    for interp in (0, 1):
        p = _prob(mpik)
        p.interp = interp
        assert mpik.lib().mpi_plan_bytes(ctypes.byref(p), ctypes.byref(pb), ctypes.byref(wb)) == 0
        sizes.append((pb.value, wb.value))
    assert sizes[0] == sizes[1]


def test_unsupported_sizes(mpik):
    # an FFT larger than the LDS line buffers
    p = _prob(mpik, n=1024, radius=1023, conv_mode="fft")
    pb, wb = ctypes.c_size_t(), ctypes.c_size_t()
    assert mpik.lib().mpi_plan_bytes(ctypes.byref(p), ctypes.byref(pb), ctypes.byref(wb)) == -6


def test_build_argument_errors_need_no_gpu(mpik):
    L = mpik.lib()
    p = _prob(mpik)
    out = ctypes.c_void_p()
    # null r / v / plan memory and a too-small plan are rejected on the host
    assert L.mpi_kernel_build(ctypes.byref(p), None, 1 << 20, None, ctypes.byref(out)) == -1
    p.r = 256
    p.v = 512
    assert L.mpi_kernel_build(ctypes.byref(p), 4096, 16, None, ctypes.byref(out)) == -3
    assert L.mpi_kernel_build(ctypes.byref(p), 4097, 1 << 30, None, ctypes.byref(out)) == -1   # misaligned
    assert out.value is None
    assert L.mpi_kernel_build(ctypes.byref(p), 4096, 1 << 30, None, None) == -1


def test_apply_argument_errors_need_no_gpu(mpik):
    L = mpik.lib()
    assert L.mpi_forward(None, 256, 256, 256, 1 << 20, None) == -1
    assert L.mpi_adjoint(None, 256, 256, 256, 1 << 20, None) == -1
    assert L.mpi_iterate(None, 256, 256, None, 256, 1 << 20, None) == -1
    assert L.mpi_batch_pair(None, 256, 256, 512, 256, 1 << 20, None) == -1
    assert L.mpi_batch_schedule(None, 2, None, None, None, None, 0, None, None) == -1
    assert L.mpi_plan_destroy(None) == -1
    assert L.mpi_plan_info(None, None, None, None) == -1


def test_trajectory_amplitude_entries_reject_bad_arguments(mpik):
    """mpi_scale_trajectory and mpi_reduce_lissajous check their arguments on
    the host: null or aliased pointers, sample counts, dtypes, a null plan."""
    L = mpik.lib()
    assert L.mpi_scale_trajectory(None, 512, 10, 1.0, 1.0, 0, 1024, 2048, None) == -1
    assert L.mpi_scale_trajectory(256, 512, 0, 1.0, 1.0, 0, 1024, 2048, None) == -1
    assert L.mpi_scale_trajectory(256, 512, 1 << 26, 1.0, 1.0, 0, 1024, 2048, None) == -1
    assert L.mpi_scale_trajectory(256, 512, 10, float("nan"), 1.0, 0, 1024, 2048, None) == -1
    assert L.mpi_scale_trajectory(256, 512, 10, 1.0, 1.0, 3, 1024, 2048, None) == -4
    assert L.mpi_scale_trajectory(256, 512, 10, 1.0, 1.0, 0, 1024, 1024, None) == -1     # r == v
    assert L.mpi_scale_trajectory(256, 512, 10, 1.0, 1.0, 0, 256, 2048, None) == -1      # r == rho
    assert L.mpi_scale_trajectory(256, 512, 10, 1.0, 1.0, 1, 1028, 2048, None) == -1     # misaligned
    assert L.mpi_reduce_lissajous(None, 256, 512, 768, 1024, 1280, 1536, 4096, 1 << 20, None) == -1
    assert L.mpi_vjp_forward(None, 256, 512, 768, 1024, 1280, 1536, 4096, 1 << 20, None) == -1
    assert L.mpi_vjp_adjoint(None, 256, 512, 768, 1024, 1280, 1536, 4096, 1 << 20, None) == -1


def test_size_limits(mpik):
    """The edges that the GPU limit tests run at are accepted, one past each is rejected."""
    pb, wb = ctypes.c_size_t(), ctypes.c_size_t()

    def code(**kw):
        p = _prob(mpik, **{k: v for k, v in kw.items() if k in ("n", "radius", "conv_mode")})
        for k, v in kw.items():
            if k not in ("n", "radius", "conv_mode"):
                setattr(p, k, v)
        return mpik.lib().mpi_plan_bytes(ctypes.byref(p), ctypes.byref(pb), ctypes.byref(wb))

    assert code(n=1024, radius=7, conv_mode="direct", n_samples=(1 << 26) - 1) == 0
    assert code(n=1024, radius=7, conv_mode="direct", n_samples=1 << 26) == -1
    assert code(n=1025, radius=7, conv_mode="direct") == -1
    assert code(n=512, radius=511, conv_mode="fft") == 0          # M = 1024, float32
    assert code(n=513, radius=7, conv_mode="fft") == -6           # the FFT path stops at 512^2
    assert code(n=400, radius=112, conv_mode="fft", dtype=1) == 0  # M = 512, float64
    assert code(n=400, radius=113, conv_mode="fft", dtype=1) == -6


def test_injected_allocation_failure_in_the_sizing(mpik):
    """The test hook fails the k-th host allocation of the plan sizing: every
    k up to the number of allocations there makes the call return
    MPI_ERR_ALLOC, and the next one lets it through with the sizes of an
    unhooked call.  A build fails the same way at the sizing and at the plan
    object, before any device call."""
    L = mpik.lib()
    probs = (mpik.Problem * 3)(*[_prob(mpik, n=n) for n in (32, 64, 128)])
    pb, wb = ctypes.c_size_t(), ctypes.c_size_t()
    assert L.mpi_batch_bytes(probs, 3, 0, ctypes.byref(pb), ctypes.byref(wb)) == 0
    ref = (pb.value, wb.value)
    try:
        k = 1
        while True:
            assert L.mpi_debug_fail_alloc(k) == 0
            pb.value = wb.value = 0
            rc = L.mpi_batch_bytes(probs, 3, 0, ctypes.byref(pb), ctypes.byref(wb))
            if rc == 0:
                break
            assert rc == mpik.MPI_ERR_ALLOC, (k, rc)
            k += 1
            assert k < 64
        assert k > 1, "the sizing reached no allocation point"
        assert (pb.value, wb.value) == ref
        sizing_points = k - 1
        # the build: the sizing's points, then the plan object, all before any device call
        p = _prob(mpik)
        p.r, p.v = 256, 512
        out = ctypes.c_void_p()
        for k in (1, sizing_points, sizing_points + 1):
            assert L.mpi_debug_fail_alloc(k) == 0
            assert L.mpi_kernel_build(ctypes.byref(p), 4096, 1 << 30, None, ctypes.byref(out)) == mpik.MPI_ERR_ALLOC
            assert out.value is None
    finally:
        L.mpi_debug_fail_alloc(0)
    assert L.mpi_debug_fail_alloc(-1) == mpik.MPI_ERR_ARG
    assert L.mpi_batch_bytes(probs, 3, 0, ctypes.byref(pb), ctypes.byref(wb)) == 0


def test_bounds_checks_only_in_the_checked_build(mpik):
    """libmpik_check.so is the build with kernel bounds checks; the others
    compile them away."""
    checked = os.path.basename(mpik._LIB_PATH) == "libmpik_check.so"
    assert mpik.lib().mpi_checks_enabled() == int(checked)
    assert mpik.lib().mpi_plan_check(None, None, None) == mpik.MPI_ERR_ARG
    if not checked and os.path.exists(mpik.CHECK_LIBRARY):
        with mpik.use_library(mpik.CHECK_LIBRARY) as L:
            assert L.mpi_checks_enabled() == 1


def test_slice_flags_are_exclusive(mpik):
    """One MPI_BUILD_SLICES_* flag at most; each alone sizes a plan."""
    L = mpik.lib()
    probs = (mpik.Problem * 2)(*[_prob(mpik, n=32, radius=7, conv_mode="direct"), _prob(mpik, n=48, radius=15)])
    pb, wb = ctypes.c_size_t(), ctypes.c_size_t()
    for f in (16, 32, 64):
        assert L.mpi_batch_bytes(probs, 2, f, ctypes.byref(pb), ctypes.byref(wb)) == 0
    assert L.mpi_batch_bytes(probs, 2, 16 | 64, ctypes.byref(pb), ctypes.byref(wb)) == mpik.MPI_ERR_ARG
