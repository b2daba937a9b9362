"""The C-ABI library loads and exports every entry point of include/mgfem.h
(CPU only: no compute call is made)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mgfem.h")
LIB = os.path.join(ROOT, "paper_2505_05105_amd", "libmgfem.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(mgfem_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        from paper_2505_05105_amd import build
        build.build()
    return ctypes.CDLL(LIB)


def test_every_declared_symbol_is_exported(lib):
    names = declared_functions()
    assert len(names) >= 14
    for name in names:
        assert hasattr(lib, name), name


def test_binding_declares_the_same_names():
    from paper_2505_05105_amd import _lib
    assert sorted(_lib.EXPORTED) == declared_functions()


def test_host_only_calls(lib):
    """Calls that touch no device: defaults, status strings, argument checks."""
    from paper_2505_05105_amd import _lib
    p = _lib.default_params()
    assert (p.gamma, p.snap_alpha, p.nu1, p.nu2, p.eta, p.coarsest_n) == (2.0, 1.75, 2, 1, 4, 4)
    assert _lib.status_string(_lib.ERR_EMPTY_DOMAIN) == "empty domain"
    h = ctypes.c_void_p()
    # null psi is rejected before any device work
    rc = _lib.lib().mgfem_setup(None, 64, ctypes.byref(p), None, ctypes.byref(h))
    assert rc == _lib.ERR_INVALID_ARG and not h.value
    # gamma <= 1 loses coercivity (section 4.4) and is rejected
    bad = _lib.default_params(gamma=1.0)
    rc = _lib.lib().mgfem_setup(ctypes.c_void_p(16), 64, ctypes.byref(bad), None, ctypes.byref(h))
    assert rc == _lib.ERR_INVALID_ARG
    assert "gamma" in _lib.last_error(None)
    # N must be coarsest_n times a power of two
    rc = _lib.lib().mgfem_setup(ctypes.c_void_p(16), 96, ctypes.byref(p), None, ctypes.byref(h))
    assert rc == _lib.ERR_INVALID_ARG
    assert _lib.lib().mgfem_level_n(None, 0) == -1
    # history queries reject a null handle and a negative capacity
    cnt = ctypes.c_int32(7)
    assert _lib.lib().mgfem_step_cycles(None, None, 0, ctypes.byref(cnt)) == _lib.ERR_INVALID_ARG
    assert _lib.lib().mgfem_residual_l2(None, None, 0, ctypes.byref(cnt)) == _lib.ERR_INVALID_ARG
    # inner_cycles outside 1..16 is rejected for mixed precision, before any device work
    for k in (0, 17):
        bad = _lib.default_params(precision=_lib.PREC_MIXED, inner_cycles=k)
        rc = _lib.lib().mgfem_setup(ctypes.c_void_p(16), 64, ctypes.byref(bad), None, ctypes.byref(h))
        assert rc == _lib.ERR_INVALID_ARG and "inner_cycles" in _lib.last_error(None)
