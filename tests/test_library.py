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
    assert lib.fio_apply(None, None, None, 1, None) == -1
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
