"""Host-side checks of the C-ABI library (no GPU needed): it loads and
exports every entry point that include/fio.h declares."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fio.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(fio3?_[a-z_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ("fio_plan", "fio_apply", "fio_apply_adjoint", "fio_destroy", "fio_last_error"):
        assert must in names


def test_library_exports_every_declared_symbol():
    import torch  # noqa: F401  (load torch's HIP runtime first, as the binding does)
    import paper_0809_0719_amd as fio
    path = fio.library_path()
    if not os.path.exists(path):
        pytest.fail(f"{path} not built: run __graft_entry__.build()")
    lib = ctypes.CDLL(path)
    for name in declared_functions():
        assert hasattr(lib, name), name
    assert sorted(fio.EXPORTED_SYMBOLS) == declared_functions()


def test_argument_errors_need_no_device():
    # validation happens before any device call
    import torch  # noqa: F401
    import paper_0809_0719_amd as fio
    lib = fio.load_library()
    h = ctypes.c_void_p()
    ph = fio._cphase(fio.Phase())
    assert lib.fio_plan(100, 9, ctypes.byref(ph), ctypes.byref(h)) == -1     # N not a power of two
    assert b"power of two" in lib.fio_last_error()
    assert lib.fio_plan(64, 2, ctypes.byref(ph), ctypes.byref(h)) == -1      # q too small
    assert lib.fio_plan(64, 17, ctypes.byref(ph), ctypes.byref(h)) == -1     # q too large
    bad = fio._cphase(fio.Phase(a1=-1.0))
    assert lib.fio_plan(64, 9, ctypes.byref(bad), ctypes.byref(h)) == -1
    assert lib.fio_apply(None, None, None, 1, fio.C64, None) == -1
    assert lib.fio_apply_adjoint(None, None, None, 1, fio.C64, None) == -1
    assert lib.fio_destroy(None) == 0


def test_batch_and_q_selection_argument_errors_need_no_device():
    import torch  # noqa: F401
    import paper_0809_0719_amd as fio
    lib = fio.load_library()
    h = ctypes.c_void_p()
    plans = (ctypes.c_void_p * 2)(None, None)
    assert lib.fio_batch_create(plans, 0, 4, ctypes.byref(h)) == -1           # no plans
    assert lib.fio_batch_create(plans, 2, 0, ctypes.byref(h)) == -1           # no streams
    assert lib.fio_batch_create(plans, 2, 4, ctypes.byref(h)) == -1           # NULL plans
    assert b"NULL" in lib.fio_last_error()
    assert lib.fio_batch_apply(None, None, None, None) == -1
    assert lib.fio_batch_destroy(None) == -1
    assert lib.fio_direct_rows(None, None, None, 1, None, None) == -1
    ph = fio._cphase(fio.Phase())
    opts = fio._COpts(-1, -1, fio.C64, 1, fio.CONTRACT_FP)
    q, err = ctypes.c_int(), ctypes.c_double()
    assert lib.fio_select_q(64, ctypes.byref(ph), ctypes.byref(opts), 1e-4, 9, 5, 64, 0, ctypes.byref(q),
                            ctypes.byref(err), None) == -1                     # qmin > qmax
    assert lib.fio_select_q(64, ctypes.byref(ph), ctypes.byref(opts), 0.0, 3, 9, 64, 0, ctypes.byref(q),
                            ctypes.byref(err), None) == -1                     # tol <= 0
    assert lib.fio_select_q(100, ctypes.byref(ph), ctypes.byref(opts), 1e-4, 3, 9, 64, 0, ctypes.byref(q),
                            ctypes.byref(err), None) == -1                     # N not a power of two


@pytest.mark.gpu
def test_apply_rejects_dtype_mismatch_and_overlapping_ranges_before_any_launch():
    """fio_apply / fio_apply_adjoint check the caller's dtype against the
    plan's and reject input and output byte ranges that share a byte --
    equal pointers, or one starting inside the other -- before any launch
    (the plan at N = 16 launches nothing when it is made either)."""
    import torch
    import paper_0809_0719_amd as fio
    lib = fio.load_library()
    N, nr = 16, 3
    plan = fio.Plan(N, 4, fio.Phase(), dtype=torch.complex64, nrhs_max=nr)
    buf = torch.zeros(4 * nr * N * N, dtype=torch.complex64, device="cuda")
    p0 = buf.data_ptr()
    plane = N * N * 8
    for fn in (lib.fio_apply, lib.fio_apply_adjoint):
        assert fn(plan._h, p0, p0 + nr * plane, nr, fio.C128, None) == -1
        assert b"dtype" in lib.fio_last_error()
        assert fn(plan._h, p0, p0, nr, fio.C64, None) == -1
        assert fn(plan._h, p0, p0 + plane, nr, fio.C64, None) == -1          # u starts inside f
        assert fn(plan._h, p0 + (nr * plane) // 2, p0, nr, fio.C64, None) == -1   # f starts inside u
        assert b"overlap" in lib.fio_last_error()
        assert fn(plan._h, p0, p0 + nr * plane, 0, fio.C64, None) == -1
    torch.cuda.synchronize()
    assert not buf.any()   # nothing was launched


@pytest.mark.gpu
def test_binding_checks_output_tensors():
    """Plan.apply / Plan.adjoint / Batch write through the output's data
    pointer, so a wrong shape, dtype, device, layout or an output that shares
    memory with the input is refused before the library is called."""
    import torch
    import paper_0809_0719_amd as fio
    N = 16
    plan = fio.Plan(N, 4, fio.Phase(), dtype=torch.complex64, nrhs_max=2)
    f = torch.zeros(2, N, N, dtype=torch.complex64, device="cuda")
    bad = [torch.empty(1, N, N, dtype=torch.complex64, device="cuda"),           # too small
           torch.empty(2, N, N, dtype=torch.complex128, device="cuda"),          # dtype
           torch.empty(2, N, N, dtype=torch.complex64),                          # host
           torch.empty(2, N, 2 * N, dtype=torch.complex64, device="cuda")[:, :, ::2],   # strided
           f]                                                                    # aliases the input
    for out in bad:
        for call in (plan.apply, plan.adjoint):
            with pytest.raises(ValueError):
                call(f, out=out)
    batch = fio.Batch([fio.Plan(N, 4, fio.Phase(), dtype=torch.complex64)], nstreams=1)
    with pytest.raises(ValueError):
        batch.apply([f[0]], [torch.empty(N, N + 1, dtype=torch.complex64, device="cuda")])
    torch.cuda.synchronize()
