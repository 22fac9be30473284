"""Differentiable solves: p = A(kappa)^{-1} f with a hand-written adjoint.

``FVOperator`` wraps the library's finite-volume operator (assembly of the
two-point-flux matrix from base-mesh faces and the kappa-gradient kernel);
``PoissonSolve`` is a torch.autograd.Function whose backward solves
A lambda = dL/dp with the same symmetric reduced solve (A = A^T, Q_s = Q_s^T)
and returns dL/df = lambda and dL/dkappa from face products.  Marshalling
only: assembly, setup, solves and the gradient run in libmsp.so.
"""
from __future__ import annotations

import ctypes

import numpy as np
import scipy.sparse as sp

from . import _lib
from ._lib import MSP_NOT_CONVERGED, MspError, check, lib
from .solver import Solver


def _p(a, t):
    return a.ctypes.data_as(ctypes.POINTER(t))


class FVOperator:
    """Base-mesh face geometry (any object with cell_a, cell_b, kind, axis,
    area, dist_a, dist_b arrays) and the symmetry map img (n_b x 2^s)."""

    def __init__(self, faces, img, device: int = 0):
        self._keep = dict(
            ca=np.ascontiguousarray(faces.cell_a, dtype=np.int64), cb=np.ascontiguousarray(faces.cell_b, dtype=np.int64),
            kind=np.ascontiguousarray(faces.kind, dtype=np.int8), axis=np.ascontiguousarray(faces.axis, dtype=np.int8),
            area=np.ascontiguousarray(faces.area, dtype=np.float64),
            da=np.ascontiguousarray(faces.dist_a, dtype=np.float64),
            db=np.ascontiguousarray(faces.dist_b, dtype=np.float64))
        k = self._keep
        F = _lib.msp_faces(k["ca"].size, _p(k["ca"], ctypes.c_int64), _p(k["cb"], ctypes.c_int64),
                           _p(k["kind"], ctypes.c_int8), _p(k["axis"], ctypes.c_int8), _p(k["area"], ctypes.c_double),
                           _p(k["da"], ctypes.c_double), _p(k["db"], ctypes.c_double))
        self.img = np.ascontiguousarray(img, dtype=np.int64)
        self.n_b, S = self.img.shape
        self.s = S.bit_length() - 1
        self.n = self.n_b * S
        smap = _lib.msp_symmap(self.s, self.n_b, _p(self.img, ctypes.c_int64))
        self._h = ctypes.c_void_p()
        check(lib.msp_fv_create(ctypes.byref(F), ctypes.byref(smap), device, ctypes.byref(self._h)))

    def assemble(self, kappa_base: np.ndarray) -> sp.csr_matrix:
        kap = np.ascontiguousarray(kappa_base, dtype=np.float64)
        nnz = ctypes.c_int64()
        check(lib.msp_fv_nnz(self._h, ctypes.byref(nnz)))
        rp = np.empty(self.n + 1, np.int64)
        ci = np.empty(nnz.value, np.int32)
        va = np.empty(nnz.value)
        vp = lambda a: a.ctypes.data_as(ctypes.c_void_p)  # noqa: E731
        check(lib.msp_fv_assemble(self._h, vp(kap), vp(rp), vp(ci), vp(va)))
        return sp.csr_matrix((va, ci, rp), shape=(self.n, self.n))

    def nnz(self) -> int:
        v = ctypes.c_int64()
        check(lib.msp_fv_nnz(self._h, ctypes.byref(v)))
        return v.value

    def assemble_device(self, kappa, out=None, stream=None):
        """The values of ``assemble``'s matrix for kappa (torch, n_b, on the
        device), computed on the device in its positions: a float64 tensor of
        nnz values (``out`` if given)."""
        import torch
        kap = kappa.detach().to(torch.float64).contiguous()
        if out is None:
            out = torch.empty(self.nnz(), dtype=torch.float64, device=kap.device)
        if out.numel() != self.nnz() or out.dtype != torch.float64 or not out.is_contiguous():
            raise ValueError("out must be a contiguous float64 tensor of nnz values")
        st = stream if stream is not None else torch.cuda.current_stream(kap.device)
        check(lib.msp_fv_assemble_device(self._h, ctypes.c_void_p(kap.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                                         ctypes.c_void_p(st.cuda_stream)))
        return out

    def kappa_grad(self, kappa, lam, p, stream=None):
        """dL/dkappa (torch, n_b) from lambda and p (torch, (n,) or (n, m))."""
        import torch
        lam2 = lam.reshape(self.n, -1).t().contiguous()
        p2 = p.reshape(self.n, -1).t().contiguous()
        kap = kappa.contiguous().to(torch.float64)
        out = torch.empty(self.n_b, dtype=torch.float64, device=lam.device)
        st = stream if stream is not None else torch.cuda.current_stream(lam.device)
        check(lib.msp_fv_kappa_grad(self._h, ctypes.c_void_p(kap.data_ptr()), lam2.shape[0],
                                    ctypes.c_void_p(lam2.data_ptr()), ctypes.c_void_p(p2.data_ptr()),
                                    ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(st.cuda_stream)))
        return out

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            lib.msp_fv_free(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class DifferentiablePoisson:
    """Holds the operator and a solver for the last kappa seen.

    resetup = "host": every new kappa gets a fresh solver (host assembly and
    setup).  resetup = "device": the first kappa sets the solver up on the
    host; for later ones the matrix is assembled on the device and the
    solver's values are recomputed there on the first setup's structure
    (msp_fv_assemble_device, msp_refresh), which is much faster for the small
    kappa steps of an optimisation.  A backward for a forward whose kappa
    has since been replaced is then an error (the solver holds the new
    values).  Three policies bound what the kept structure costs:
    ``max_split_drift`` (a fraction of the base cells): a device re-setup
    whose reduction-level split a fresh setup would change on more cells than
    that (msp_stats.split_drift) is followed at once by a fresh host setup for
    the same kappa; ``max_split_drift1`` (a fraction of the level-1 points):
    the same for level 1's split of the new A_1 (msp_stats.split_drift1),
    which moves long before the reduction level's does (with
    ``drift1_action="rebuild_below"`` the solver keeps its re-set-up reduction
    level and rebuilds the levels below it on the host, msp_rebuild_below,
    instead of a fresh setup); ``max_iteration_growth`` (a ratio): once a solve on a
    re-set-up solver takes more than that times the iterations of the first
    solve after the last fresh setup, the next kappa gets a fresh host setup
    (the coarser levels and the kept interpolation patterns can cost
    iterations while the reduction level's split stays)."""

    def __init__(self, faces, img, device: int = 0, resetup: str = "host", max_split_drift=None,
                 max_iteration_growth=None, max_split_drift1=None, drift1_action: str = "fresh",
                 **solver_opts):
        if resetup not in ("host", "device"):
            raise ValueError("resetup must be 'host' or 'device'")
        if drift1_action not in ("fresh", "rebuild_below"):
            raise ValueError("drift1_action must be 'fresh' or 'rebuild_below'")
        self.op = FVOperator(faces, img, device)
        self.opts = dict(solver_opts, device=device)
        self.resetup = resetup
        self.max_split_drift = max_split_drift
        self.max_split_drift1 = max_split_drift1
        self.drift1_action = drift1_action
        self.rebuilds = 0
        self._base_version = 0     # solver version of the last fresh setup or rebuild
        self.max_iteration_growth = max_iteration_growth
        self.fresh_setups = 0
        self._fresh_iters = None   # iterations of the first solve after the last fresh setup
        self._grown = False
        self._kappa = None
        self._vals = None
        self.solver = None

    def solver_for(self, kappa):
        """The solver for this kappa (rebuilt when kappa changes).  With host
        re-setups the previous solver is not closed here: an autograd graph
        recorded with it may still need it for its backward solve, and it is
        freed when the last reference goes."""
        import torch
        kap = kappa.detach().to(torch.float64)
        if self._kappa is not None and self._kappa.device == kap.device and torch.equal(kap, self._kappa):
            return self.solver
        fresh = True
        if self.resetup == "device" and self.solver is not None and not self._grown:
            self._vals = self.op.assemble_device(kap, out=self._vals)
            self.solver.refresh(self._vals)
            st = self.solver.stats
            over0 = self.max_split_drift is not None and st.split_drift > self.max_split_drift * self.op.n_b
            over1 = (self.max_split_drift1 is not None and st.nlev > 2
                     and st.split_drift1 > self.max_split_drift1 * st.rows[1])
            fresh = over0 or over1
            if over1 and not over0 and self.drift1_action == "rebuild_below":
                self.solver.rebuild_below(self._vals)
                self.rebuilds += 1
                self._fresh_iters = None
                self._base_version = self.solver.version
                fresh = False
        if fresh:
            A = self.op.assemble(kap.cpu().numpy())
            self.solver = Solver(A, self.op.img, **self.opts)
            self.fresh_setups += 1
            self._fresh_iters = None
            self._base_version = 0
            self._grown = False
        self._kappa = kap.clone()
        return self.solver

    def __call__(self, f, kappa):
        return PoissonSolve.apply(f, kappa, self)

    def _observe(self, sv):
        """Iteration count of a solve with the current solver (the growth policy)."""
        if sv is not self.solver:
            return
        its = sv.last.iters
        if self._fresh_iters is None and sv.version == self._base_version:
            self._fresh_iters = its
        elif (self.max_iteration_growth is not None and self._fresh_iters is not None
              and sv.version > self._base_version
              and its > self.max_iteration_growth * self._fresh_iters):
            self._grown = True


def _converged_solve(sv, rhs, what):
    """A solve whose result feeds a gradient: an unconverged one is an error."""
    import warnings
    with warnings.catch_warnings():
        warnings.simplefilter("ignore", RuntimeWarning)
        x = sv.solve(rhs)
    if sv.status != MSP_NOT_CONVERGED:
        return x
    raise MspError(MSP_NOT_CONVERGED, f"{what} solve did not reach the tolerance in {sv.last.iters} iterations")


def _torch_function():
    import torch

    class PoissonSolve(torch.autograd.Function):
        """p = A(kappa)^{-1} f; backward: lambda = A^{-1} g, dL/df = lambda,
        dL/dkappa = face-product gradient (library kernel)."""

        @staticmethod
        def forward(ctx, f, kappa, dp):
            sv = dp.solver_for(kappa)
            p = _converged_solve(sv, f.contiguous(), "forward")
            dp._observe(sv)
            ctx.dp = dp
            ctx.sv = sv
            ctx.version = sv.version
            ctx.save_for_backward(p, kappa)
            return p

        @staticmethod
        def backward(ctx, g):
            p, kappa = ctx.saved_tensors
            if ctx.sv.version != ctx.version:
                raise RuntimeError("the solver of this forward was re-set up for another kappa since: run the "
                                   "backward first, or use resetup='host'")
            lam = _converged_solve(ctx.sv, g.contiguous(), "adjoint")
            gk = ctx.dp.op.kappa_grad(kappa, lam, p) if ctx.needs_input_grad[1] else None
            return lam, gk, None

    return PoissonSolve


class _Lazy:
    _fn = None

    def __getattr__(self, name):
        if _Lazy._fn is None:
            _Lazy._fn = _torch_function()
        return getattr(_Lazy._fn, name)


PoissonSolve = _Lazy()
