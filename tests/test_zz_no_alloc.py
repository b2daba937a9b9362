"""The allocation-free misfit call against mgfem_misfit, through the C ABI.

mgfem_misfit_noalloc keeps its partial sums in the library's static device
array instead of allocated memory.  Two calls in a row on two handles, the
second with the smaller grid, and the first handle again: J and dJ/du equal
those of mgfem_misfit (dJ/du bit for bit: the same rows in the same order;
J to rounding, its sum runs in another order), and the device's free memory
does not change across the calls.
"""
import ctypes as C

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2505_05105_amd as mg
    return mg


def _case(mg, N, seed):
    p = W.flower_mms(N)
    s = mg.Solver(p.psi, N)
    rng = np.random.default_rng(seed)
    dev = "cuda:0"
    u = torch.tensor(p.u_exact + 0.01 * rng.standard_normal(p.u_exact.shape), device=dev)
    ut = torch.tensor(W.adjoint_target(N), device=dev)
    return s, u, ut


def _both(mg, s, u, ut):
    from paper_2505_05105_amd import _lib
    L = _lib.lib()
    n = u.numel()
    y0 = torch.full((n,), 7.0, dtype=torch.float64, device=u.device)
    y1 = torch.full((n,), -7.0, dtype=torch.float64, device=u.device)
    J0, J1 = C.c_double(0.0), C.c_double(0.0)
    _lib.check(L.mgfem_misfit(s.handle, u.data_ptr(), ut.data_ptr(), C.byref(J0), y0.data_ptr()), s.handle)
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    _lib.check(L.mgfem_misfit_noalloc(s.handle, u.data_ptr(), ut.data_ptr(), C.byref(J1), y1.data_ptr()),
               s.handle)
    torch.cuda.synchronize()
    free1 = torch.cuda.mem_get_info()[0]
    # J without dJ/du as well
    J2 = C.c_double(0.0)
    _lib.check(L.mgfem_misfit_noalloc(s.handle, u.data_ptr(), ut.data_ptr(), C.byref(J2), None), s.handle)
    return J0.value, J1.value, J2.value, y0, y1, free0, free1


def test_noalloc_misfit_equals_misfit_on_consecutive_calls():
    mg = _gpu()
    big = _case(mg, 512, 1)
    small = _case(mg, 128, 2)
    for s, u, ut in (big, small, big):
        print(f"noalloc misfit: N={s.N}", flush=True)
        J0, J1, J2, y0, y1, free0, free1 = _both(mg, s, u, ut)
        assert J0 > 0.0
        assert J1 == pytest.approx(J0, rel=1e-12, abs=0.0)
        assert J2 == J1
        assert torch.equal(y0, y1)
        assert free1 == free0


def test_noalloc_misfit_rejects_bad_arguments():
    mg = _gpu()
    from paper_2505_05105_amd import _lib
    L = _lib.lib()
    s, u, ut = _case(mg, 64, 3)
    J = C.c_double(0.0)
    assert L.mgfem_misfit_noalloc(s.handle, None, ut.data_ptr(), C.byref(J), None) == _lib.ERR_INVALID_ARG
    assert L.mgfem_misfit_noalloc(s.handle, u.data_ptr(), ut.data_ptr(), None, None) == _lib.ERR_INVALID_ARG
    assert L.mgfem_misfit_noalloc(None, u.data_ptr(), ut.data_ptr(), C.byref(J), None) == _lib.ERR_INVALID_ARG
