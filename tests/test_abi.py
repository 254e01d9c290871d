"""The C-ABI library loads and exports every function declared in include/lhdm.h;
host-side argument checks run without a GPU (no compute call is made)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    inc = os.path.join(ROOT, "include")
    src = "\n".join(open(os.path.join(inc, f)).read() for f in sorted(os.listdir(inc)) if f.endswith(".h"))
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[a-z_0-9]+\s*\*?\s*([a-z_0-9]+)\s*\(", src, flags=re.M)
    return sorted(set(n for n in names if n.startswith(("lhdm_", "lh_"))))


@pytest.fixture(scope="module")
def lib():
    from paper_2108_05345_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        import __graft_entry__
        __graft_entry__.build()
    return _lib.load()


def test_header_declares_the_boundary():
    names = _declared_functions()
    for required in ("lhdm_solve", "lh_solve", "lhdm_solve_batched", "lhdm_backward"):
        assert required in names


def test_library_exports_every_declared_symbol(lib):
    names = _declared_functions()
    assert len(names) >= 10
    for name in names:
        assert hasattr(lib, name), name


def test_binding_signatures_cover_the_header(lib):
    from paper_2108_05345_amd import _lib
    assert set(_declared_functions()) == set(_lib.SIGNATURES)


def test_struct_layouts():
    from paper_2108_05345_amd import _lib
    assert ctypes.sizeof(_lib.LhdmParams) == 48
    assert ctypes.sizeof(_lib.LhdmInfo) == 40


def test_default_params(lib):
    from paper_2108_05345_amd import _lib
    p = _lib.LhdmParams()
    lib.lhdm_default_params(ctypes.byref(p))
    # Section 5: tau1 = 0.6, delta = 0.9, tau2 = 0.15, kmax = 32
    assert (p.tau1, p.tau2, p.delta, p.kmax) == (0.6, 0.15, 0.9, 32)
    assert p.kkt_tol == 1e-9


def test_status_strings(lib):
    for code in (0, 1, 2, 3, -1, -2, -3, -4):
        assert lib.lhdm_status_string(code)


def test_argument_validation_without_gpu(lib):
    from paper_2108_05345_amd import _lib
    p = _lib.LhdmParams()
    lib.lhdm_default_params(ctypes.byref(p))
    fake = 256  # never dereferenced: validation fails first
    # m < 1
    assert lib.lhdm_solve(None, 0, 5, fake, 1, fake, ctypes.byref(p), fake, None, None, None, None, 0) == -1
    # lda < m
    assert lib.lhdm_solve(None, 5, 5, fake, 4, fake, ctypes.byref(p), fake, None, None, None, None, 0) == -1
    # NULL A
    assert lib.lhdm_solve(None, 5, 5, None, 5, fake, ctypes.byref(p), fake, None, None, None, None, 0) == -1
    # bad parameters
    for field, bad in (("tau1", 0.0), ("tau2", 1.5), ("delta", 0.0), ("kmax", 0), ("kmax", 65)):
        q = _lib.LhdmParams()
        lib.lhdm_default_params(ctypes.byref(q))
        setattr(q, field, bad)
        assert lib.lhdm_solve(None, 5, 5, fake, 5, fake, ctypes.byref(q), fake, None, None, None, None, 0) == -1
    assert lib.lh_solve(None, 5, 5, fake, 5, fake, -1.0, 0, fake, None, None, None, None, 0) == -1
    mm = (ctypes.c_int32 * 1)(0)
    nn = (ctypes.c_int32 * 1)(4)
    off = (ctypes.c_int64 * 1)(0)
    assert lib.lhdm_solve_batched(None, 1, mm, nn, off, fake, off, fake, off, fake, None, ctypes.byref(p), 0,
                                  None, None, 0) == -1
    assert lib.lhdm_backward(None, 0, mm, nn, off, fake, off, fake, off, fake, fake, fake, fake, fake,
                             None, 0) == -1


def test_workspace_queries(lib):
    from paper_2108_05345_amd import _lib
    p = _lib.LhdmParams()
    lib.lhdm_default_params(ctypes.byref(p))
    assert lib.lhdm_workspace_bytes(64, 128, ctypes.byref(p)) > 64 * 64 * 8
    assert lib.lhdm_workspace_bytes(0, 128, ctypes.byref(p)) == 0
    mm = (ctypes.c_int32 * 2)(32, 64)
    nn = (ctypes.c_int32 * 2)(80, 130)
    assert lib.lhdm_batched_workspace_bytes(2, mm, nn, ctypes.byref(p)) > 0
    assert lib.lhdm_backward_workspace_bytes(2, mm, nn) >= 8 * (32 * 32 + 64 * 64)


def test_signed_entry_rejects_bad_sizes_before_device_work(lib):
    from paper_2108_05345_amd import _lib
    p = _lib.LhdmParams()
    lib.lhdm_default_params(ctypes.byref(p))
    assert lib.lhdm_solve_signed(None, 0, 5, None, 1, None, ctypes.byref(p), 1, None, None, None, None, None,
                                 0) == _lib.LHDM_EINVAL
    assert lib.lhdm_signed_workspace_bytes(0, 5, ctypes.byref(p)) == 0


def test_theorem4_flag_is_checked_on_the_host(lib):
    from paper_2108_05345_amd import _lib
    p = _lib.LhdmParams()
    lib.lhdm_default_params(ctypes.byref(p))
    p.flags = 4   # LHDM_FLAG_NO_JLOOP with tau1 = 0.6: invalid
    assert lib.lhdm_solve(None, 4, 4, None, 4, None, ctypes.byref(p), None, None, None, None, None,
                          0) == _lib.LHDM_EINVAL
