"""dsweep: diagonal-sweeping source-transfer DDM for the PML Helmholtz equation on MI355X.

Python binding of libdsweep.so.  Argument marshalling only: every step of the
method runs in the library's HIP kernels; PyTorch provides device memory and
the current stream.  Every call needs the built library and a GPU; there is no
fallback.

    plan = Plan(n=(1024, 1024), h=1/1024, omega=2*pi*40, pml=20, overlap=10,
                parts=(8, 8), m=m_cuda, precision="c64", max_rhs=16)
    x, iters, relres = plan.gmres(b, tol=1e-6, maxit=60)
"""
from __future__ import annotations

import ctypes as C
from typing import Optional, Sequence, Tuple

import torch

from . import _lib
from ._lib import DSD_C64, DSD_C128, DSD_OK, DsweepError, check

__all__ = ["Plan", "HelmholtzMisfit", "DsweepError", "load_library"]


def load_library():
    return _lib.load()


def _stream_ptr():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dev(t: torch.Tensor, dtype, name: str) -> torch.Tensor:
    if not t.is_cuda or t.dtype != dtype or not t.is_contiguous():
        raise ValueError(f"{name} must be a contiguous CUDA tensor of dtype {dtype}")
    return t


class Plan:
    """Partition, local operators and factors for one (medium, omega) pair."""

    def __init__(self, n: Sequence[int], h: float, omega: float, pml: int, overlap: int,
                 parts: Sequence[int], m: torch.Tensor, precision: str = "c64",
                 max_rhs: int = 1, rhs_per_group: int = 0, sigma0_delta: float = 60.0,
                 schedule: str = "dag", local_solver: str = "auto", dense_top: int = 0,
                 sweep_order: str = "default", nd_leaf: int = 0, nd_top_cells: int = 0,
                 nd_wide: int = 0, nd_wave_steps: int = 0, nd_fuse: int = 0):
        self._lib = _lib.load()
        dim = len(n)
        if dim not in (2, 3) or len(parts) != dim:
            raise ValueError("n and parts must have 2 or 3 entries")
        p = _lib.Params()
        p.dim = dim
        for a in range(3):
            p.n[a] = int(n[a]) if a < dim else 1
            p.parts[a] = int(parts[a]) if a < dim else 1
        p.h, p.pml, p.overlap = float(h), int(pml), int(overlap)
        p.sigma0_delta = float(sigma0_delta)
        p.precision = {"c64": DSD_C64, "c128": DSD_C128}[precision]
        p.max_rhs, p.rhs_per_group = int(max_rhs), int(rhs_per_group)
        p.schedule = {"dag": 0, "sequential": 1, "additive": 2}[schedule]
        p.local_solver = {"auto": 0, "chain": 1, "bcr": 2, "chain-steps": 3, "nd": 4}[local_solver]
        p.dense_top = int(dense_top)
        p.sweep_order = {"default": 0, "l1": 1}[sweep_order]
        p.nd_leaf, p.nd_top_cells, p.nd_wide = int(nd_leaf), int(nd_top_cells), int(nd_wide)
        p.nd_wave_steps, p.nd_fuse = int(nd_wave_steps), int(nd_fuse)
        self.params = p
        self.n, self.dim, self.pml, self.omega = tuple(int(k) for k in n), dim, int(pml), omega
        self.precision, self.max_rhs = precision, int(max_rhs)
        self.gshape = tuple(k + 2 * pml for k in reversed(self.n))
        m = _dev(m, torch.float64, "m")
        if tuple(m.shape) != tuple(reversed(self.n)):
            raise ValueError(f"m must have shape {tuple(reversed(self.n))}")
        h_ = C.c_void_p()
        check(self._lib.dsd_plan_create(C.byref(p), float(omega), C.c_void_p(m.data_ptr()),
                                        _stream_ptr(), C.byref(h_)), "dsd_plan_create")
        self._h = h_

    def close(self):
        if getattr(self, "_h", None):
            self._lib.dsd_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ------------------------------------------------------------- queries
    def info(self) -> dict:
        ng, ns, fb, wb = C.c_longlong(), C.c_int(), C.c_longlong(), C.c_longlong()
        check(self._lib.dsd_plan_info(self._h, C.byref(ng), C.byref(ns), C.byref(fb),
                                      C.byref(wb)), "dsd_plan_info")
        return {"n_global": ng.value, "n_subdomains": ns.value, "factor_bytes": fb.value,
                "workspace_bytes": wb.value}

    def pivots(self) -> dict:
        """dsd_plan_pivots: the largest max|pivot| / min|pivot| of the factorisation's
        block inversions and its subdomain."""
        r, sub = C.c_double(), C.c_int()
        check(self._lib.dsd_plan_pivots(self._h, C.byref(r), C.byref(sub)), "dsd_plan_pivots")
        return {"ratio": r.value, "subdomain": sub.value}

    def subdomain_grid(self, sub: int) -> Tuple[Tuple[int, ...], Tuple[int, ...]]:
        dims, g0 = (C.c_int * 3)(), (C.c_int * 3)()
        check(self._lib.dsd_subdomain_grid(self._h, int(sub), dims, g0), "dsd_subdomain_grid")
        return tuple(dims[: self.dim]), tuple(g0[: self.dim])

    def _batch(self, t: torch.Tensor, name: str) -> int:
        _dev(t, torch.complex128, name)
        if tuple(t.shape[1:]) != self.gshape:
            raise ValueError(f"{name} must have shape (nrhs, *{self.gshape})")
        return t.shape[0]

    # -------------------------------------------------------------- solves
    def local_solve(self, sub: int, r: torch.Tensor) -> torch.Tensor:
        dims, _ = self.subdomain_grid(sub)
        _dev(r, torch.complex128, "r")
        if tuple(r.shape[1:]) != tuple(reversed(dims)):
            raise ValueError(f"r must have shape (nrhs, *{tuple(reversed(dims))})")
        u = torch.empty_like(r)
        check(self._lib.dsd_local_solve(self._h, int(sub), C.c_void_p(r.data_ptr()),
                                        C.c_void_p(u.data_ptr()), r.shape[0], _stream_ptr()),
              "dsd_local_solve")
        return u

    def local_solve_noalloc(self, sub: int, r: torch.Tensor, u: torch.Tensor) -> torch.Tensor:
        """dsd_local_solve_noalloc: the same local solve with the library's static
        device scratch (no allocation in the call); the caller passes the output."""
        dims, _ = self.subdomain_grid(sub)
        _dev(r, torch.complex128, "r")
        _dev(u, torch.complex128, "u")
        if tuple(r.shape[1:]) != tuple(reversed(dims)) or u.shape != r.shape:
            raise ValueError(f"r and u must have shape (nrhs, *{tuple(reversed(dims))})")
        check(self._lib.dsd_local_solve_noalloc(self._h, int(sub), C.c_void_p(r.data_ptr()),
                                                C.c_void_p(u.data_ptr()), r.shape[0],
                                                _stream_ptr()), "dsd_local_solve_noalloc")
        return u

    def sweep_apply(self, f: torch.Tensor, out: Optional[torch.Tensor] = None) -> torch.Tensor:
        k = self._batch(f, "f")
        u = torch.empty_like(f) if out is None else out
        check(self._lib.dsd_sweep_apply(self._h, C.c_void_p(f.data_ptr()),
                                        C.c_void_p(u.data_ptr()), k, _stream_ptr()),
              "dsd_sweep_apply")
        return u

    def apply_operator(self, x: torch.Tensor) -> torch.Tensor:
        k = self._batch(x, "x")
        y = torch.empty_like(x)
        check(self._lib.dsd_apply_operator(self._h, C.c_void_p(x.data_ptr()),
                                           C.c_void_p(y.data_ptr()), k, _stream_ptr()),
              "dsd_apply_operator")
        return y

    def _krylov(self, fn, b, tol, maxit, restart, name):
        k = self._batch(b, "b")
        x = torch.empty_like(b)
        iters, rel = (C.c_int * k)(), (C.c_double * k)()
        rc = fn(self._h, C.c_void_p(b.data_ptr()), C.c_void_p(x.data_ptr()), k, float(tol),
                int(maxit), int(restart), iters, rel, _stream_ptr())
        check(rc, name, allow_not_converged=True)
        return x, list(iters), list(rel), rc == _lib.DSD_OK

    def gmres(self, b: torch.Tensor, tol: float = 1e-6, maxit: int = 100, restart: int = 0):
        """Solve M x = b; returns (x, iterations per RHS, true relres per RHS, converged)."""
        return self._krylov(self._lib.dsd_gmres_solve, b, tol, maxit, restart, "dsd_gmres_solve")

    def ddm_iterate(self, f: torch.Tensor, iters: int):
        """The sweeps as a stand-alone iterative solver: x_{k+1} = x_k + DDM(f - M x_k)
        from x_0 = 0; returns (x, relative residual history of shape (iters + 1, k))."""
        k = self._batch(f, "f")
        x = torch.empty_like(f)
        hist = (C.c_double * ((int(iters) + 1) * k))()
        check(self._lib.dsd_ddm_iterate(self._h, C.c_void_p(f.data_ptr()), C.c_void_p(x.data_ptr()),
                                        k, int(iters), hist, _stream_ptr()), "dsd_ddm_iterate")
        return x, [list(hist[i * k:(i + 1) * k]) for i in range(int(iters) + 1)]

    def adjoint_solve(self, b: torch.Tensor, tol: float = 1e-6, maxit: int = 100,
                      restart: int = 0):
        """Solve M^H x = b with the same factors."""
        return self._krylov(self._lib.dsd_adjoint_solve, b, tol, maxit, restart,
                            "dsd_adjoint_solve")

    # ----------------------------------------------------------------- FWI
    def fwi_forward(self, f: torch.Tensor, receivers: torch.Tensor, tol=1e-6, maxit=100,
                    allow_not_converged=False):
        """d = P u_s for every source.  Raises DsweepError (DSD_NOT_CONVERGED) if a
        forward solve missed tol within maxit, unless allow_not_converged; the
        flag of the last call is kept in ``last_converged``."""
        k = self._batch(f, "f")
        _dev(receivers, torch.int64, "receivers")
        d = torch.empty((k, receivers.numel()), dtype=torch.complex128, device=f.device)
        rc = self._lib.dsd_fwi_forward(self._h, C.c_void_p(f.data_ptr()), k,
                                       C.c_void_p(receivers.data_ptr()), receivers.numel(),
                                       float(tol), int(maxit), C.c_void_p(d.data_ptr()),
                                       _stream_ptr())
        check(rc, "dsd_fwi_forward", allow_not_converged=allow_not_converged)
        self.last_converged = rc == DSD_OK
        return d

    def fwi_gradient(self, f: torch.Tensor, receivers: torch.Tensor, d_obs: torch.Tensor,
                     tol=1e-6, maxit=100, allow_not_converged=False):
        """Misfit 1/2 sum |P u - d|^2 and its gradient w.r.t. m = 1/c^2 (physical cells).
        Raises DsweepError (DSD_NOT_CONVERGED) if a forward or adjoint solve missed
        tol within maxit, unless allow_not_converged; the flag of the last call is
        kept in ``last_converged``."""
        k = self._batch(f, "f")
        _dev(receivers, torch.int64, "receivers")
        _dev(d_obs, torch.complex128, "d_obs")
        g = torch.empty(tuple(reversed(self.n)), dtype=torch.float64, device=f.device)
        J = C.c_double()
        rc = self._lib.dsd_fwi_gradient(self._h, C.c_void_p(f.data_ptr()), k,
                                        C.c_void_p(receivers.data_ptr()), receivers.numel(),
                                        C.c_void_p(d_obs.data_ptr()), float(tol), int(maxit),
                                        C.c_void_p(g.data_ptr()), C.byref(J), None,
                                        _stream_ptr())
        check(rc, "dsd_fwi_gradient", allow_not_converged=allow_not_converged)
        self.last_converged = rc == DSD_OK
        return J.value, g

    # -------------------------------------------------------------- timing
    def autotune(self, nrhs: Optional[int] = None, reps: int = 2) -> dict:
        """Time the candidate launch shapes of the subdomain solves and keep the fastest."""
        k = self.max_rhs if nrhs is None else int(nrhs)
        kg, cw, cm, ms = C.c_int(), C.c_int(), C.c_int(), C.c_double()
        check(self._lib.dsd_autotune(self._h, k, int(reps), C.byref(kg), C.byref(cw), C.byref(cm),
                                     C.byref(ms), _stream_ptr()), "dsd_autotune")
        return {"rhs_per_group": kg.value, "cg_wide": cw.value, "cg_mid": cm.value,
                "ms_per_application": ms.value, "shape": self.solve_shape}

    @property
    def solve_shape(self) -> tuple:
        """Launch shape of the subdomain solves (13 ints: RHS per workgroup, then the
        cyclic-reduction level policy); set it to reuse an autotuned shape."""
        v = (C.c_int * 13)()
        check(self._lib.dsd_get_solve_shape(self._h, v), "dsd_get_solve_shape")
        return tuple(v)

    @solve_shape.setter
    def solve_shape(self, shape):
        v = (C.c_int * 13)(*[int(x) for x in shape])
        check(self._lib.dsd_set_solve_shape(self._h, v), "dsd_set_solve_shape")

    def use_graph(self, on: bool = True):
        """Run preconditioner applications as captured HIP graphs."""
        check(self._lib.dsd_set_graph(self._h, int(bool(on))), "dsd_set_graph")

    @property
    def local_solver(self) -> str:
        return {1: "chain", 2: "bcr", 3: "chain-steps",
                4: "nd"}[self._lib.dsd_plan_local_solver(self._h)]

    def timing(self, on: bool):
        check(self._lib.dsd_timing_enable(self._h, int(bool(on))), "dsd_timing_enable")

    def timing_read(self) -> dict:
        ms, n, b, o = C.c_double(), C.c_longlong(), C.c_double(), C.c_double()
        check(self._lib.dsd_timing_read(self._h, C.byref(ms), C.byref(n), C.byref(b),
                                        C.byref(o)), "dsd_timing_read")
        fl = C.c_double()
        check(self._lib.dsd_timing_flops(self._h, C.byref(fl)), "dsd_timing_flops")
        return {"solve_ms": ms.value, "solve_launches": n.value, "solve_bytes": b.value,
                "solve_flops": fl.value}


class HelmholtzMisfit(torch.autograd.Function):
    """J(m) = 1/2 sum_s ||P u_s - d_s||^2 with M(m) u_s = f_s.

    forward(m, f, receivers, d_obs, plan_kwargs, tol, maxit) -> scalar tensor.
    The gradient dJ/dm comes from the adjoint solves M^H lam_s = P^T(P u_s - d_s)
    with the same complex-symmetric factors; it is computed together with J
    (one factorisation) and returned by backward.  A forward or adjoint solve
    that misses tol within maxit raises DsweepError (DSD_NOT_CONVERGED) instead
    of returning a gradient of unconverged fields.
    """

    @staticmethod
    def forward(ctx, m, f, receivers, d_obs, plan_kwargs, tol=1e-6, maxit=100):
        plan = Plan(m=m.detach().contiguous(), max_rhs=f.shape[0], **plan_kwargs)
        try:
            J, g = plan.fwi_gradient(f, receivers, d_obs, tol=tol, maxit=maxit)
        finally:
            plan.close()
        ctx.save_for_backward(g)
        return torch.tensor(J, dtype=torch.float64, device=m.device)

    @staticmethod
    def backward(ctx, grad_out):
        (g,) = ctx.saved_tensors
        return grad_out * g, None, None, None, None, None, None
