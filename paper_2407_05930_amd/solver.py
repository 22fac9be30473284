"""Python front end of the C interface: ``Solver(A, img, ...)`` then
``solve(b)``.  Marshalling only; every step of the solve runs in the
library's HIP kernels.  Device arrays are torch tensors."""
from __future__ import annotations

import ctypes
import warnings
from typing import Optional

import numpy as np

from . import _lib
from ._lib import check, lib


def _ptr(a: np.ndarray, ctype):
    return a.ctypes.data_as(ctypes.POINTER(ctype))


def _csr(A):
    """The matrix as contiguous arrays (kept alive by the caller) and its msp_csr."""
    indptr = np.ascontiguousarray(A.indptr, dtype=np.int64)
    indices = np.ascontiguousarray(A.indices, dtype=np.int32)
    data = np.ascontiguousarray(A.data, dtype=np.float64)
    csr = _lib.msp_csr(indptr.size - 1, _ptr(indptr, ctypes.c_int64), _ptr(indices, ctypes.c_int32),
                       _ptr(data, ctypes.c_double))
    return (indptr, indices, data), csr


def default_opts() -> _lib.msp_opts:
    o = _lib.msp_opts()
    check(lib.msp_default_opts(ctypes.byref(o)))
    return o


def make_opts(**kw) -> _lib.msp_opts:
    o = default_opts()
    for key, val in kw.items():
        if key == "precision":
            val = _lib.PRECISION[val] if isinstance(val, str) else val
        elif key == "pc":
            val = _lib.PC[val] if isinstance(val, str) else val
        elif key == "k":
            key = "lrc_k"
        if not hasattr(o, key):
            raise TypeError(f"unknown option {key}")
        setattr(o, key, val)
    return o


def _warn_not_converged(rc, what):
    if rc == _lib.MSP_NOT_CONVERGED:
        warnings.warn(f"{what}: maximum iteration count reached before the tolerance (MSP_NOT_CONVERGED); "
                      "the result is the last iterate", RuntimeWarning, stacklevel=3)


class Solver:
    """Setup from the full symmetric matrix ``A`` (scipy CSR or anything with
    indptr/indices/data) and the symmetry map ``img`` (n_b x 2^s, row of
    image a of base cell i); options as in ``msp_opts`` (``k`` = LRC rank,
    ``precision`` in {"fp64", "mixed", "mixed_bf16g", "mixed_bf16"}, ``pc`` in
    {"amgr", "fsai", "none", "amgr_sub", "amgs"}, ``device`` = -1 for a host-only setup)."""

    def __init__(self, A, img, **opts):
        img = np.ascontiguousarray(img, dtype=np.int64)
        if img.ndim != 2:
            raise ValueError("img must be (n_b, 2^s)")
        n_b, S = img.shape
        s = S.bit_length() - 1
        if 1 << s != S:
            raise ValueError("img must have 2^s columns")
        arrays, csr = _csr(A)
        self.n, self.n_b, self.s = csr.n, n_b, s
        smap = _lib.msp_symmap(s, n_b, _ptr(img, ctypes.c_int64))
        self.opts = make_opts(**opts)
        self._ctx = ctypes.c_void_p()
        check(lib.msp_setup(ctypes.byref(csr), ctypes.byref(smap), ctypes.byref(self.opts),
                            ctypes.byref(self._ctx)))
        self.last = _lib.msp_stats()
        self.version = 0   # incremented by every refresh

    @classmethod
    def from_copies(cls, A, sub, **opts):
        """Setup of AMGR in the original basis for a domain made of copies of
        one subdomain (msp_setup_copies): ``sub`` is (n_b, copies), the row of
        base unknown i in copy a.  The context solves the whole system in its
        own ordering; ``export_outer`` reports the interface over all n
        unknowns."""
        sub = np.ascontiguousarray(sub, dtype=np.int64)
        if sub.ndim != 2:
            raise ValueError("sub must be (n_b, copies)")
        arrays, csr = _csr(A)
        self = cls.__new__(cls)
        self.n, self.n_b, self.s = csr.n, csr.n, 0
        cmap = _lib.msp_copies(sub.shape[1], sub.shape[0], _ptr(sub, ctypes.c_int64))
        self.opts = make_opts(**opts)
        self._ctx = ctypes.c_void_p()
        check(lib.msp_setup_copies(ctypes.byref(csr), ctypes.byref(cmap), ctypes.byref(self.opts),
                                   ctypes.byref(self._ctx)))
        self.last = _lib.msp_stats()
        self.version = 0   # incremented by every refresh
        return self

    def refresh(self, values, stream=None):
        """Numeric re-setup on the device (msp_refresh) for a matrix with the
        setup matrix's sparsity: ``values`` are its nonzeros in the CSR order
        of the matrix given at setup (a float64 CUDA tensor, or a host array
        that is copied to the device first)."""
        import torch
        if not torch.is_tensor(values):
            values = torch.from_numpy(np.ascontiguousarray(values, dtype=np.float64)).cuda()
        if values.dtype != torch.float64 or not values.is_cuda or not values.is_contiguous():
            raise ValueError("values must be a contiguous float64 CUDA tensor")
        st = stream if stream is not None else torch.cuda.current_stream(values.device)
        self.version += 1
        check(lib.msp_refresh(self._ctx, ctypes.c_void_p(values.data_ptr()), ctypes.c_void_p(st.cuda_stream)))

    def rebuild_below(self, values=None, stream=None):
        """Rebuild every level below the reduction level on the host from the
        current level-1 operator (msp_rebuild_below): for a solver whose
        re-setups have moved the coarser splits (``stats.split_drift1``).  The
        reduction level, with its current values, is kept; the solver then
        holds the new context (``version`` is incremented, as by refresh).
        ``values``: the float64 CUDA tensor of the last refresh (or of the
        setup matrix), from which the device computes the per-subsystem
        values and the corrections instead of the host."""
        new = ctypes.c_void_p()
        vp, sp = None, None
        if values is not None:
            import torch
            if values.dtype != torch.float64 or not values.is_cuda or not values.is_contiguous():
                raise ValueError("values must be a contiguous float64 CUDA tensor")
            st = stream if stream is not None else torch.cuda.current_stream(values.device)
            vp, sp = ctypes.c_void_p(values.data_ptr()), ctypes.c_void_p(st.cuda_stream)
        check(lib.msp_rebuild_below(self._ctx, vp, sp, ctypes.byref(new)))
        lib.msp_free(self._ctx)
        self._ctx = new
        self.version += 1

    # ------------------------------------------------------------------ solves
    def solve(self, b, stream=None):
        """Solve A x = b for a torch tensor b on the context's GPU, shape (n,)
        or (n, m), float64.  Returns x with b's shape.  The library takes and
        writes n x m column-major arrays: a b already column-major (the
        transpose of a contiguous (m, n) tensor) is passed without a copy, and
        x is returned as the column-major view the library wrote.  ``stream``
        is a torch.cuda.Stream (default: the current stream)."""
        import torch
        vec = b.dim() == 1
        B = b.reshape(self.n, -1)
        m = B.shape[1]
        bt = B.t().contiguous()                       # (m, n) = n x m column-major
        if bt.dtype != torch.float64 or not bt.is_cuda:
            raise ValueError("b must be a float64 CUDA tensor")
        xt = torch.empty_like(bt)
        st = stream if stream is not None else torch.cuda.current_stream(bt.device)
        rc = check(lib.msp_solve_device(self._ctx, m, ctypes.c_void_p(bt.data_ptr()),
                                        ctypes.c_void_p(xt.data_ptr()), ctypes.c_void_p(st.cuda_stream),
                                        ctypes.byref(self.last)))
        self.status = rc
        _warn_not_converged(rc, "Solver.solve")
        x = xt.t()
        return x.reshape(-1) if vec else x

    def solve_host(self, b: np.ndarray) -> np.ndarray:
        vec = b.ndim == 1
        B = np.asarray(b, dtype=np.float64).reshape(self.n, -1)
        m = B.shape[1]
        bt = np.ascontiguousarray(B.T)
        xt = np.empty_like(bt)
        rc = check(lib.msp_solve(self._ctx, m, bt.ctypes.data_as(ctypes.c_void_p),
                                 xt.ctypes.data_as(ctypes.c_void_p), ctypes.byref(self.last)))
        self.status = rc
        _warn_not_converged(rc, "Solver.solve_host")
        return xt.T.reshape(-1) if vec else np.ascontiguousarray(xt.T)

    # ------------------------------------------------------------------ introspection
    @property
    def stats(self):
        st = _lib.msp_stats()
        check(lib.msp_get_stats(self._ctx, ctypes.byref(st)))
        return st

    def num_levels(self) -> int:
        v = ctypes.c_int32()
        check(lib.msp_num_levels(self._ctx, ctypes.byref(v)))
        return v.value

    def export_level(self, lev: int) -> dict:
        """Host copy of level ``lev``: cf mask, A, P, G (scipy CSR), omega."""
        import scipy.sparse as sp
        n, nA, nP, nG = (ctypes.c_int64() for _ in range(4))
        check(lib.msp_level_sizes(self._ctx, lev, ctypes.byref(n), ctypes.byref(nA), ctypes.byref(nP),
                                  ctypes.byref(nG)))
        n, nA, nP, nG = n.value, nA.value, nP.value, nG.value
        cf = np.zeros(n, dtype=np.int8)
        Arp, Aci, Av = np.zeros(n + 1, np.int64), np.zeros(nA, np.int32), np.zeros(nA)
        has_p = nP > 0
        Prp, Pci, Pv = np.zeros(n + 1, np.int64), np.zeros(nP, np.int32), np.zeros(nP)
        Grp, Gci, Gv = np.zeros(n + 1, np.int64), np.zeros(nG, np.int32), np.zeros(nG)
        om = ctypes.c_double()
        vp = lambda a: a.ctypes.data_as(ctypes.c_void_p)  # noqa: E731
        check(lib.msp_export_level(self._ctx, lev, vp(cf), vp(Arp), vp(Aci), vp(Av),
                                   vp(Prp) if has_p else None, vp(Pci) if has_p else None,
                                   vp(Pv) if has_p else None, vp(Grp) if nG else None,
                                   vp(Gci) if nG else None, vp(Gv) if nG else None, ctypes.byref(om)))
        out = dict(A=sp.csr_matrix((Av, Aci, Arp), shape=(n, n)), omega=om.value)
        if has_p:
            nc = int(cf.sum())
            out["cf"] = cf.astype(bool)
            out["P"] = sp.csr_matrix((Pv, Pci, Prp), shape=(n, nc))
            out["G"] = sp.csr_matrix((Gv, Gci, Grp), shape=(n, n))
        return out

    def export_sub_level(self, lev: int, a: int) -> dict:
        """pc = "amgr_sub": level ``lev`` >= 1 of subsystem ``a`` -- A, P, G on
        the shared level's patterns (scipy CSR) with this subsystem's values,
        and its damping."""
        shared = self.export_level(lev)
        vp = lambda x: x.ctypes.data_as(ctypes.c_void_p)  # noqa: E731
        Av = np.zeros(shared["A"].nnz)
        Pv = np.zeros(shared["P"].nnz) if "P" in shared else None
        Gv = np.zeros(shared["G"].nnz) if "G" in shared else None
        om = ctypes.c_double()
        check(lib.msp_export_sub_level(self._ctx, lev, a, vp(Av), vp(Pv) if Pv is not None else None,
                                       vp(Gv) if Gv is not None else None, ctypes.byref(om)))
        import scipy.sparse as sp

        def like(M, v):
            return sp.csr_matrix((v, M.indices.copy(), M.indptr.copy()), shape=M.shape)

        out = dict(A=like(shared["A"], Av), omega=om.value)
        if Pv is not None:
            out["cf"] = shared["cf"]
            out["P"] = like(shared["P"], Pv)
            out["G"] = like(shared["G"], Gv)
        return out

    def export_outer(self):
        S = 1 << self.s
        sigma = np.zeros(self.n_b * S)
        iface = np.zeros(self.n_b, dtype=np.int8)
        check(lib.msp_export_outer(self._ctx, sigma.ctypes.data_as(ctypes.c_void_p),
                                   iface.ctypes.data_as(ctypes.c_void_p)))
        return sigma.reshape(self.n_b, S), iface.astype(bool)

    def export_amgs(self, which: str):
        """AMGS blocks and factors ("B", "C1", "GK", "SG1", "GS1") as scipy CSR,
        in the library's inner-first order of the base cells."""
        import scipy.sparse as sp
        w = {"B": 0, "C1": 1, "GK": 2, "SG1": 3, "GS1": 4}[which]
        nr, nc, nz = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
        check(lib.msp_export_amgs(self._ctx, w, ctypes.byref(nr), ctypes.byref(nc), ctypes.byref(nz), None, None,
                                  None))
        rp = np.zeros(nr.value + 1, np.int64)
        ci = np.zeros(nz.value, np.int32)
        v = np.zeros(nz.value)
        vp = lambda a: a.ctypes.data_as(ctypes.c_void_p)  # noqa: E731
        check(lib.msp_export_amgs(self._ctx, w, None, None, None, vp(rp), vp(ci), vp(v)))
        return sp.csr_matrix((v, ci, rp), shape=(nr.value, nc.value))

    def export_lrc(self):
        S = 1 << self.s
        k = self.opts.lrc_k
        kept = np.zeros(S, dtype=np.int32)
        ritz = np.zeros(S * max(k, 1))
        check(lib.msp_export_lrc(self._ctx, kept.ctypes.data_as(ctypes.c_void_p),
                                 ritz.ctypes.data_as(ctypes.c_void_p)))
        return kept, ritz.reshape(S, max(k, 1))[:, :k]

    # ------------------------------------------------------------------ timers
    KIND_NAMES = {0: "operator", 1: "dot", 2: "update", 3: "p_update", 4: "qs", 5: "cast", 6: "dense_coarse",
                  7: "fsai", 8: "lrc", 9: "amgs"}

    @staticmethod
    def kind_name(kind: int) -> str:
        if kind < 16:
            return Solver.KIND_NAMES.get(kind, f"kind{kind}")
        lev, op = divmod(kind - 16, 8)
        return f"L{lev}.{['A', 'M', 'GT', 'R', 'P', '?', '?', '?'][op]}"

    def set_timing(self, on: bool = True, kind: int = -1):
        check(lib.msp_set_timing(self._ctx, kind, 1 if on else 0))

    def reset_timing(self):
        check(lib.msp_reset_timing(self._ctx))

    def timing(self) -> dict:
        """{kind: (count, total_ms, total_bytes)} for kinds with launches."""
        out = {}
        for kind in range(16 + 8 * 20):
            cnt, ms, by = ctypes.c_int64(), ctypes.c_double(), ctypes.c_double()
            check(lib.msp_get_timing(self._ctx, kind, ctypes.byref(cnt), ctypes.byref(ms), ctypes.byref(by)))
            if cnt.value:
                out[kind] = (cnt.value, ms.value, by.value)
        return out

    def timing_kernels(self) -> dict:
        """{kind: kernel function name} for kinds with timed launches."""
        out = {}
        buf = ctypes.create_string_buffer(256)
        for kind in self.timing():
            check(lib.msp_get_timing_kernel(self._ctx, kind, buf, 256))
            out[kind] = buf.value.decode()
        return out

    def close(self):
        if getattr(self, "_ctx", None) and self._ctx.value:
            lib.msp_free(self._ctx)
            self._ctx = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class BatchSolver:
    """Many independent systems solved together: one launch of a captured
    HIP graph whose iterations are gated per system on the device.
    ``systems`` is a list of (A, img) pairs; options as for Solver (shared by
    all systems)."""

    def __init__(self, systems, **opts):
        self.n = []
        self._keep = []
        csrs = (_lib.msp_csr * len(systems))()
        maps = (_lib.msp_symmap * len(systems))()
        for i, (A, img) in enumerate(systems):
            img = np.ascontiguousarray(img, dtype=np.int64)
            n_b, S = img.shape
            s = S.bit_length() - 1
            indptr = np.ascontiguousarray(A.indptr, dtype=np.int64)
            indices = np.ascontiguousarray(A.indices, dtype=np.int32)
            data = np.ascontiguousarray(A.data, dtype=np.float64)
            self._keep.append((img, indptr, indices, data))
            n = indptr.size - 1
            self.n.append(n)
            csrs[i] = _lib.msp_csr(n, _ptr(indptr, ctypes.c_int64), _ptr(indices, ctypes.c_int32),
                                   _ptr(data, ctypes.c_double))
            maps[i] = _lib.msp_symmap(s, n_b, _ptr(img, ctypes.c_int64))
        self.opts = make_opts(**opts)
        self._h = ctypes.c_void_p()
        check(lib.msp_batch_setup(len(systems), csrs, maps, ctypes.byref(self.opts), ctypes.byref(self._h)))
        self._keep = None
        self.stats = (_lib.msp_stats * len(systems))()

    def set_chunk(self, iterations: int):
        """Iterations the next solve's graph holds (later solves size it from
        the iterations the previous one needed)."""
        check(lib.msp_batch_set_chunk(self._h, iterations))

    @property
    def last_launches(self) -> int:
        """Graph launches of the last solve (1 when one graph held them all)."""
        v = ctypes.c_int32()
        check(lib.msp_batch_last_launches(self._h, ctypes.byref(v)))
        return v.value

    def solve(self, bs, stream=None):
        """bs: list of float64 CUDA tensors (n_i,) or (n_i, m_i).  Returns the
        list of solutions with the same shapes."""
        import torch
        k = len(bs)
        ms = (ctypes.c_int32 * k)()
        pb = (ctypes.c_void_p * k)()
        px = (ctypes.c_void_p * k)()
        bts, xts, shapes = [], [], []
        for i, b in enumerate(bs):
            shapes.append(b.dim() == 1)
            B = b.reshape(self.n[i], -1)
            bt = B.t().contiguous()
            xt = torch.empty_like(bt)
            bts.append(bt)
            xts.append(xt)
            ms[i] = bt.shape[0]
            pb[i] = bt.data_ptr()
            px[i] = xt.data_ptr()
        st = stream if stream is not None else torch.cuda.current_stream(bs[0].device)
        self.status = check(lib.msp_batch_solve(self._h, ms, pb, px, ctypes.c_void_p(st.cuda_stream), self.stats))
        _warn_not_converged(self.status, "BatchSolver.solve")
        return [x.t().reshape(-1) if vec else x.t() for x, vec in zip(xts, shapes)]

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            lib.msp_batch_free(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
