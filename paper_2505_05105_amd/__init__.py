"""Ghost-FEM multigrid on MI355X (gfx950): Python binding of libmgfem.so.

PyTorch provides device memory and streams only; every step of setup, solve
and adjoint runs in the library's HIP kernels (see include/mgfem.h).

    solver = Solver(psi, N)                  # psi: (N+1)^2 nodal level set
    u, hist = solver.solve(f, g, tol=1e-10)  # u: torch float64 on the GPU
    u = GhostFEMSolve.apply(f, g, solver)    # differentiable in f and g

    l2 = solver.residual_l2()                # ||F - A u_m||_2 beside the max-norm hist

    solver = Solver(psi, N, chi=chi)         # Neumann where chi > 0 (mixed boundaries)
    u, hist = solver.solve(f, gD, gN=gN)
    u = GhostFEMSolveMixed.apply(f, gD, gN, solver)   # differentiable in f, g_D and g_N

    batch = BatchedSolver(psis, Ns)          # many problems, one persistent launch
    us, hists = batch.solve(fs, gs, tol=1e-10)
"""
from __future__ import annotations

import ctypes as C

import numpy as np
import torch

from . import _lib
from ._lib import (COARSE_GALERKIN, COARSE_REDISCRETISED, CYCLE_TWO_GRID, CYCLE_V, CYCLE_W,  # noqa: F401
                   PREC_FP64, PREC_MIXED, STAB_FIXED, STAB_GLOBAL, STAB_LOCAL_EIG, STAB_PAPER, MgfemError,
                   default_params)

__all__ = ["Solver", "BatchedSolver", "GhostFEMSolve", "GhostFEMSolveMixed", "MgfemError", "default_params"]

CELL_TYPES = ("external", "triangle", "quadrilateral", "pentagon", "internal",
              "saddle_split", "saddle_hexagon")


def _dev(x, device, n=None):
    """A contiguous float64 tensor on `device` (copied from numpy if needed)."""
    if isinstance(x, np.ndarray):
        x = torch.from_numpy(np.ascontiguousarray(x, dtype=np.float64))
    if not isinstance(x, torch.Tensor):
        raise TypeError("expected a numpy array or a torch tensor")
    x = x.to(device=device, dtype=torch.float64).contiguous().reshape(-1)
    if n is not None and x.numel() != n:
        raise ValueError(f"expected {n} values, got {x.numel()}")
    return x


class Solver:
    """One level set, one hierarchy (mgfem_setup / mgfem_destroy).  With chi,
    the nodal Neumann indicator, mixed boundaries (mgfem_setup_mixed_bc)."""

    def __init__(self, psi, N, device="cuda:0", chi=None, **params):
        self.N = int(N)
        self.n = (self.N + 1) ** 2
        self.device = torch.device(device)
        self.params = default_params(**params)
        self.stream = torch.cuda.current_stream(self.device)
        self._psi = _dev(psi, self.device, self.n)
        h = C.c_void_p()
        L = _lib.lib()
        if chi is None:
            rc = L.mgfem_setup(self._psi.data_ptr(), self.N, C.byref(self.params),
                               C.c_void_p(self.stream.cuda_stream), C.byref(h))
        else:
            chi_t = _dev(chi, self.device, self.n)
            rc = L.mgfem_setup_mixed_bc(self._psi.data_ptr(), chi_t.data_ptr(), self.N,
                                        C.byref(self.params), C.c_void_p(self.stream.cuda_stream),
                                        C.byref(h))
        _lib.check(rc, None)
        self.handle = h
        self.last_cycles = 0

    # -- queries -------------------------------------------------------------
    def info(self) -> dict:
        inf = _lib.Info()
        _lib.check(_lib.lib().mgfem_query(self.handle, C.byref(inf)), self.handle)
        out = {f: getattr(inf, f) for f, _ in _lib.Info._fields_}
        out["n_cells_by_type"] = dict(zip(CELL_TYPES, list(inf.n_cells_by_type)))
        return out

    def residual_l2(self):
        """||F - A u_m||_2, m = 0..cycles, of the last solve or adjoint."""
        cnt = C.c_int32(0)
        _lib.check(_lib.lib().mgfem_residual_l2(self.handle, None, 0, C.byref(cnt)), self.handle)
        out = np.zeros(cnt.value)
        if cnt.value:
            _lib.check(_lib.lib().mgfem_residual_l2(self.handle, out.ctypes.data_as(C.POINTER(C.c_double)),
                                                    cnt.value, C.byref(cnt)), self.handle)
        return out

    def step_cycles(self):
        """V-cycles run by each iteration of the last solve or adjoint (mixed
        precision: the float32 cycles of each float64 step)."""
        cnt = C.c_int32(0)
        _lib.check(_lib.lib().mgfem_step_cycles(self.handle, None, 0, C.byref(cnt)), self.handle)
        out = np.zeros(cnt.value, dtype=np.int32)
        if cnt.value:
            _lib.check(_lib.lib().mgfem_step_cycles(self.handle, out.ctypes.data_as(C.POINTER(C.c_int32)),
                                                    cnt.value, C.byref(cnt)), self.handle)
        return out

    def level_n(self, level):
        return _lib.lib().mgfem_level_n(self.handle, level)

    @property
    def n_levels(self):
        return self.info()["n_levels"]

    def export(self, what, level=0):
        Nl = self.level_n(level)
        if Nl < 0:
            raise ValueError("level out of range")
        sizes = {_lib.EXPORT_PSI: (self.N + 1) ** 2, _lib.EXPORT_CELL_TYPE: self.N ** 2,
                 _lib.EXPORT_CELL_LAMBDA: self.N ** 2, _lib.EXPORT_A: 9 * (Nl + 1) ** 2,
                 _lib.EXPORT_M: 9 * (Nl + 1) ** 2, _lib.EXPORT_G: 9 * (Nl + 1) ** 2,
                 _lib.EXPORT_NODE_FLAGS: (Nl + 1) ** 2, _lib.EXPORT_RHS: (self.N + 1) ** 2,
                 _lib.EXPORT_GN: 9 * (Nl + 1) ** 2}
        out = torch.empty(sizes[what], dtype=torch.float64, device=self.device)
        _lib.check(_lib.lib().mgfem_export(self.handle, what, level, out.data_ptr()), self.handle)
        return out

    # -- solves --------------------------------------------------------------
    def solve(self, f, g, tol=1e-10, max_cycles=50, u0=None, out=None, raise_on_fail=True, gN=None):
        """Returns (u, hist) with hist[m] = ||F - A u_m||_inf, m = 0..cycles.
        g is the Dirichlet data, gN the Neumann data (mixed boundaries)."""
        f = _dev(f, self.device, self.n)
        g = _dev(g, self.device, self.n)
        gN = None if gN is None else _dev(gN, self.device, self.n)
        flags = 0
        if out is None:
            out = torch.empty(self.n, dtype=torch.float64, device=self.device)
        if u0 is not None:
            out.copy_(_dev(u0, self.device, self.n))
            flags = _lib.SOLVE_WARM_START
        hist = np.zeros(max_cycles + 1)
        ncyc = C.c_int32(0)
        hp = hist.ctypes.data_as(C.POINTER(C.c_double))
        if gN is None:
            rc = _lib.lib().mgfem_solve(self.handle, f.data_ptr(), g.data_ptr(), float(tol),
                                        int(max_cycles), flags, out.data_ptr(), hp, C.byref(ncyc))
        else:
            rc = _lib.lib().mgfem_solve_mixed_bc(self.handle, f.data_ptr(), g.data_ptr(), gN.data_ptr(),
                                                 float(tol), int(max_cycles), flags, out.data_ptr(), hp,
                                                 C.byref(ncyc))
        self.last_status = rc
        self.last_cycles = ncyc.value
        if raise_on_fail:
            _lib.check(rc, self.handle, allow=(_lib.OK, _lib.ERR_NOT_CONVERGED))
        return out, hist[: ncyc.value + 1]

    def adjoint(self, dJdu, tol=1e-10, max_cycles=50):
        """Returns (dJ/df, dJ/dg, lam, hist) from the transposed cycles."""
        dJdu = _dev(dJdu, self.device, self.n)
        lam = torch.empty(self.n, dtype=torch.float64, device=self.device)
        df = torch.empty_like(lam)
        dg = torch.empty_like(lam)
        hist = np.zeros(max_cycles + 1)
        ncyc = C.c_int32(0)
        rc = _lib.lib().mgfem_adjoint(self.handle, dJdu.data_ptr(), float(tol), int(max_cycles),
                                      lam.data_ptr(), df.data_ptr(), dg.data_ptr(),
                                      hist.ctypes.data_as(C.POINTER(C.c_double)), C.byref(ncyc))
        _lib.check(rc, self.handle, allow=(_lib.OK, _lib.ERR_NOT_CONVERGED))
        return df, dg, lam, hist[: ncyc.value + 1]

    def neumann_gradient(self, lam):
        """dJ/dg_N = GN^T lam for the lam returned by adjoint()."""
        lam = _dev(lam, self.device, self.n)
        out = torch.empty(self.n, dtype=torch.float64, device=self.device)
        _lib.check(_lib.lib().mgfem_adjoint_neumann(self.handle, lam.data_ptr(), out.data_ptr()),
                   self.handle)
        return out

    def misfit(self, u, ut):
        """J = 1/2 (u - u_t)^T M (u - u_t) and dJ/du = M (u - u_t)."""
        u = _dev(u, self.device, self.n)
        ut = _dev(ut, self.device, self.n)
        J = C.c_double(0.0)
        g = torch.empty(self.n, dtype=torch.float64, device=self.device)
        _lib.check(_lib.lib().mgfem_misfit(self.handle, u.data_ptr(), ut.data_ptr(), C.byref(J),
                                           g.data_ptr()), self.handle)
        return J.value, g

    def smooth(self, level, x, b, steps=1, reverse=False):
        """Apply smoothing steps of one level in place on x (device float64)."""
        _lib.check(_lib.lib().mgfem_smooth(self.handle, level, x.data_ptr(), b.data_ptr(), steps,
                                           1 if reverse else 0), self.handle)
        return x

    def level_counts(self, level):
        a, s, c = C.c_int64(), C.c_int64(), C.c_int64()
        _lib.check(_lib.lib().mgfem_level_counts(self.handle, level, C.byref(a), C.byref(s), C.byref(c)),
                   self.handle)
        return {"n_active": a.value, "n_stored": s.value, "n_cut": c.value}

    def profile(self, enable=True, repeat=1):
        """Enable HIP-event timing of the profiled kernel class (resets the
        counters); repeat > 1 times each profiled launch repeated back to back."""
        _lib.check(_lib.lib().mgfem_profile(self.handle, (max(1, int(repeat)) if enable else 0)), self.handle)

    def profile_read(self, kernel_class=0):
        n, ms, b = C.c_int64(), C.c_double(), C.c_double()
        _lib.check(_lib.lib().mgfem_profile_read(self.handle, kernel_class, C.byref(n), C.byref(ms),
                                                 C.byref(b)), self.handle)
        return {"launches": n.value, "total_ms": ms.value, "alg_bytes": b.value}

    def close(self):
        if getattr(self, "handle", None):
            _lib.lib().mgfem_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _float64_solver(solver):
    if solver.params.precision != PREC_FP64:
        raise ValueError("the backward pass is the transposed float64 k-cycle map, the exact gradient of a "
                         "float64 solve only: use a float64 solver (or Solver.adjoint directly)")


class GhostFEMSolve(torch.autograd.Function):
    """u = B_k (M f + G g) with k float64 cycles; backward applies the exact
    transposed k-cycle map: dL/df = M lam, dL/dg = G^T lam, lam = B_k^T dL/du
    (the gradient of the map the forward ran, not of the converged discrete
    solution).  Needs a float64 solver."""

    @staticmethod
    def forward(ctx, f, g, solver, tol=1e-10, max_cycles=50):
        _float64_solver(solver)
        u, hist = solver.solve(f.detach(), g.detach(), tol=tol, max_cycles=max_cycles)
        ctx.solver = solver
        ctx.cycles = len(hist) - 1
        return u

    @staticmethod
    def backward(ctx, grad_u):
        df, dg, _, _ = ctx.solver.adjoint(grad_u.contiguous(), tol=-1.0, max_cycles=ctx.cycles)
        return df, dg, None, None, None


class GhostFEMSolveMixed(torch.autograd.Function):
    """Mixed boundaries: u = B_k (M f + G g_D + GN g_N) with k float64 cycles
    on a solver set up with an indicator; backward gives dL/df = M lam,
    dL/dg_D = G^T lam and dL/dg_N = GN^T lam (mgfem_adjoint_neumann).  Needs
    a float64 solver."""

    @staticmethod
    def forward(ctx, f, gD, gN, solver, tol=1e-10, max_cycles=50):
        _float64_solver(solver)
        u, hist = solver.solve(f.detach(), gD.detach(), tol=tol, max_cycles=max_cycles, gN=gN.detach())
        ctx.solver = solver
        ctx.cycles = len(hist) - 1
        return u

    @staticmethod
    def backward(ctx, grad_u):
        df, dg, lam, _ = ctx.solver.adjoint(grad_u.contiguous(), tol=-1.0, max_cycles=ctx.cycles)
        return df, dg, ctx.solver.neumann_gradient(lam), None, None, None


class BatchedSolver:
    """Many independent problems solved together (mgfem_setup_batched)."""

    def __init__(self, psis, Ns, device="cuda:0", **params):
        self.Ns = [int(n) for n in Ns]
        self.device = torch.device(device)
        self.params = default_params(**params)
        self.stream = torch.cuda.current_stream(self.device)
        self._psi = [_dev(p, self.device, (n + 1) ** 2) for p, n in zip(psis, self.Ns)]
        cnt = len(self.Ns)
        ptrs = (C.c_void_p * cnt)(*[t.data_ptr() for t in self._psi])
        ns = (C.c_int32 * cnt)(*self.Ns)
        h = C.c_void_p()
        rc = _lib.lib().mgfem_setup_batched(cnt, ptrs, ns, C.byref(self.params),
                                            C.c_void_p(self.stream.cuda_stream), C.byref(h))
        _lib.check(rc, None)
        self.handle = h

    def solve(self, fs, gs, tol=1e-10, max_cycles=50, outs=None):
        cnt = len(self.Ns)
        fs = [_dev(f, self.device, (n + 1) ** 2) for f, n in zip(fs, self.Ns)]
        gs = [_dev(g, self.device, (n + 1) ** 2) for g, n in zip(gs, self.Ns)]
        if outs is None:
            outs = [torch.empty((n + 1) ** 2, dtype=torch.float64, device=self.device) for n in self.Ns]
        hist = np.zeros(cnt * (max_cycles + 1))
        ncyc = (C.c_int32 * cnt)()
        P = C.c_void_p * cnt
        rc = _lib.lib().mgfem_solve_batched(self.handle, P(*[t.data_ptr() for t in fs]),
                                            P(*[t.data_ptr() for t in gs]), float(tol), int(max_cycles),
                                            P(*[t.data_ptr() for t in outs]),
                                            hist.ctypes.data_as(C.POINTER(C.c_double)), ncyc)
        self.last_status = rc
        _lib.check(rc, self.handle, allow=(_lib.OK, _lib.ERR_NOT_CONVERGED))
        hist = hist.reshape(cnt, max_cycles + 1)
        return outs, [hist[i, : ncyc[i] + 1] for i in range(cnt)]

    @property
    def tile(self):
        """The autotuner's choice: 0 the tiled path, else the persistent kernel's footprint width."""
        return _lib.lib().mgfem_batched_tile(self.handle)

    def last_ms(self):
        """Device time of the last batched solve."""
        inf = _lib.Info()
        _lib.check(_lib.lib().mgfem_query(self.handle, C.byref(inf)), self.handle)
        return inf.setup_ms

    def close(self):
        if getattr(self, "handle", None):
            _lib.lib().mgfem_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
