"""GPU parity of the batched form (one persistent launch for many problems):
every problem against the oracle, and against the single-problem solver."""
import numpy as np
import pytest

import workloads as W
from oracle import assembly as oasm
from oracle import multigrid as omg

from helpers import rel_max

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2505_05105_amd as mg
    return mg


def test_batched_matches_oracle_per_problem():
    mg = _gpu()
    probs = W.batched_draws(count=8, seed=0, sizes=(32, 64, 128))
    bs = mg.BatchedSolver([p.psi for p in probs], [p.N for p in probs])
    assert bs.tile in (0, 32, 64, 128, 256)
    for tol in (1e-10, 1e-12):
        us, hists = bs.solve([p.f for p in probs], [p.g for p in probs], tol=tol, max_cycles=80)
        assert bs.last_status == 0
        for p, u, h in zip(probs, us, hists):
            d = oasm.assemble(p.psi, p.N)
            F = d.rhs(p.f, p.g)
            ref = omg.solve(omg.build_hierarchy(d), F, tol=1e-14, max_cycles=100)
            assert h[-1] <= tol * h[0]
            assert h[0] == pytest.approx(np.abs(F).max(), rel=1e-12)
            ug = u.cpu().numpy()
            assert np.all(ug[~d.active] == 0)
            # single-problem FP64 solve at the same tolerance sets the error scale
            s = mg.Solver(p.psi, p.N)
            u64, _ = s.solve(p.f, p.g, tol=tol, max_cycles=80)
            err64 = rel_max(u64.cpu().numpy(), ref.u)
            assert rel_max(ug, ref.u) < 10 * err64 + 1e-13


def test_batched_fixed_cycles_equal_single_mixed():
    """Same cycles in float32 as the single-problem mixed solver (the batched
    form updates in place over global memory, the single form in LDS tiles):
    equal up to float32 rounding."""
    mg = _gpu()
    probs = W.batched_draws(count=3, seed=4, sizes=(64, 128))
    bs = mg.BatchedSolver([p.psi for p in probs], [p.N for p in probs])
    us, _ = bs.solve([p.f for p in probs], [p.g for p in probs], tol=-1.0, max_cycles=3)
    for p, u in zip(probs, us):
        s = mg.Solver(p.psi, p.N, precision=mg.PREC_MIXED)
        um, _ = s.solve(p.f, p.g, tol=-1.0, max_cycles=3)
        assert rel_max(u.cpu().numpy(), um.cpu().numpy()) < 1e-4


def test_single_problem_calls_reject_a_batched_handle():
    """A batched handle has no levels of its own: every call of one problem
    returns INVALID_ARG before it launches anything (and the handle still
    solves afterwards)."""
    mg = _gpu()
    import ctypes as C
    from paper_2505_05105_amd import _lib
    L = _lib.lib()
    probs = W.batched_draws(count=2, seed=1, sizes=(32, 64))
    bs = mg.BatchedSolver([p.psi for p in probs], [p.N for p in probs])
    n = (probs[0].N + 1) ** 2
    a = torch.zeros(n, dtype=torch.float64, device="cuda:0")
    b = torch.zeros_like(a)
    hist = (C.c_double * 8)()
    nc = C.c_int32(0)
    J = C.c_double(0.0)
    h, pa, pb = bs.handle, a.data_ptr(), b.data_ptr()
    calls = {
        "mgfem_solve": lambda: L.mgfem_solve(h, pa, pa, 1e-10, 5, 0, pb, hist, C.byref(nc)),
        "mgfem_solve_mixed_bc": lambda: L.mgfem_solve_mixed_bc(h, pa, pa, None, 1e-10, 5, 0, pb, hist,
                                                               C.byref(nc)),
        "mgfem_adjoint": lambda: L.mgfem_adjoint(h, pa, 1e-10, 5, None, pb, None, hist, C.byref(nc)),
        "mgfem_adjoint_neumann": lambda: L.mgfem_adjoint_neumann(h, pa, pb),
        "mgfem_misfit": lambda: L.mgfem_misfit(h, pa, pa, C.byref(J), pb),
        "mgfem_smooth": lambda: L.mgfem_smooth(h, 0, pa, pb, 1, 0),
        "mgfem_export": lambda: L.mgfem_export(h, _lib.EXPORT_A, 0, pb),
    }
    for name, call in calls.items():
        assert call() == _lib.ERR_INVALID_ARG, name
    torch.cuda.synchronize()
    us, hists = bs.solve([p.f for p in probs], [p.g for p in probs], tol=1e-10, max_cycles=80)
    assert bs.last_status == 0


def _batched_env(mg, probs, path, **params):
    import os
    old = os.environ.get("MGFEM_BATCH_PATH")
    os.environ["MGFEM_BATCH_PATH"] = path
    try:
        return mg.BatchedSolver([p.psi for p in probs], [p.N for p in probs], **params)
    finally:
        if old is None:
            del os.environ["MGFEM_BATCH_PATH"]
        else:
            os.environ["MGFEM_BATCH_PATH"] = old


class _env:
    """Set environment variables for the duration of a with-block."""

    def __init__(self, **kv):
        self.kv, self.old = kv, {}

    def __enter__(self):
        import os
        for k, v in self.kv.items():
            self.old[k] = os.environ.get(k)
            os.environ[k] = v

    def __exit__(self, *exc):
        import os
        for k, v in self.old.items():
            if v is None:
                del os.environ[k]
            else:
                os.environ[k] = v


def _single_mixed(mg, p, **params):
    """The single-problem mixed solver with its coarse map on the first
    single-workgroup level, as batch members have it (a single solver
    otherwise extends the map to the levels above while they are small)."""
    with _env(MGFEM_NO_MAP_EXTENSION="1"):
        return mg.Solver(p.psi, p.N, precision=mg.PREC_MIXED, **params)


@pytest.mark.parametrize("inner", [1, 2])
def test_tiled_batch_path_equals_single_mixed_solves(inner):
    """The tiled batch path runs each problem's steps with the kernels of the
    single-problem mixed solve (all problems of a step in one launch), so
    after fixed cycles every problem's iterate and max-norm history equal
    that solver's bit for bit, also with several float32 cycles per float64
    step; and to the tolerance every problem converges with the single
    solver's cycle count."""
    mg = _gpu()
    probs = W.batched_draws(count=12, seed=6, sizes=(64, 128, 256, 512))
    bs = _batched_env(mg, probs, "tiled", inner_cycles=inner)
    assert bs.tile == 0
    us, hists = bs.solve([p.f for p in probs], [p.g for p in probs], tol=-1.0, max_cycles=3)
    for p, u, h in zip(probs, us, hists):
        s = _single_mixed(mg, p, inner_cycles=inner)
        um, hm = s.solve(p.f, p.g, tol=-1.0, max_cycles=3)
        assert np.array_equal(h, hm), (p.N, h, hm)
        assert torch.equal(u, um), p.N
    # both forms with every step at the full count (each shortens its last
    # steps by its own rule otherwise: the batch by the problems' largest need)
    with _env(MGFEM_FIXED_INNER="1"):
        us, hists = bs.solve([p.f for p in probs], [p.g for p in probs], tol=1e-10, max_cycles=80)
    assert bs.last_status == 0
    for p, u, h in zip(probs, us, hists):
        s = _single_mixed(mg, p, inner_cycles=inner)
        with _env(MGFEM_FIXED_INNER="1"):
            um, hm = s.solve(p.f, p.g, tol=1e-10, max_cycles=80)
        assert len(h) == len(hm) and torch.equal(u, um), p.N


def test_persistent_batch_path_still_solves():
    mg = _gpu()
    probs = W.batched_draws(count=6, seed=7, sizes=(32, 64, 128))
    bs = _batched_env(mg, probs, "persistent")
    assert bs.tile in (32, 64, 128, 256)
    us, hists = bs.solve([p.f for p in probs], [p.g for p in probs], tol=1e-10, max_cycles=80)
    assert bs.last_status == 0
    for p, u, h in zip(probs, us, hists):
        d = oasm.assemble(p.psi, p.N)
        ref = omg.solve(omg.build_hierarchy(d), d.rhs(p.f, p.g), tol=1e-14, max_cycles=100)
        assert h[-1] <= 1e-10 * h[0]
        assert rel_max(u.cpu().numpy(), ref.u) < 1e-8
