"""Python binding of libfpde with the same names as the C ABI.

PyTorch is used only for device memory and streams: every step of the build
and of the apply runs in the library's HIP kernels.
"""
from __future__ import annotations

import ctypes as C

import numpy as np

from . import _abi
from ._abi import check, lib


def opts_struct(opts: dict | None = None, plan_only: bool = False) -> _abi.Opts:
    o = _abi.Opts()
    check(lib().fpde_opts_default(C.byref(o)), "fpde_opts_default")
    for key, val in (opts or {}).items():
        if key == "precision":
            o.precision = _abi.PREC_MIXED if val in ("mixed", _abi.PREC_MIXED) else _abi.PREC_FP64
        elif key == "jacobi":
            if val:
                o.flags |= _abi.FLAG_JACOBI
        elif hasattr(o, key):
            setattr(o, key, val)
    if plan_only:
        o.flags |= _abi.FLAG_PLAN_ONLY
    return o


def gauss_legendre(n: int):
    x = np.zeros(n)
    w = np.zeros(n)
    check(lib().fpde_gauss_legendre(n, x.ctypes.data_as(C.POINTER(C.c_double)),
                                    w.ctypes.data_as(C.POINTER(C.c_double))), "fpde_gauss_legendre")
    return x, w


def _stream_handle(stream):
    if stream is None:
        import torch
        return C.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, int):
        return C.c_void_p(stream)
    return C.c_void_p(stream.cuda_stream)


class Operator:
    """fpde_build / fpde_apply / fpde_solve / fpde_apply_adjoint / fpde_load_vector / fpde_export / fpde_stats."""

    def __init__(self, mesh, s, kappa, opts: dict | None = None, plan_only: bool = False):
        self._h = C.c_void_p()
        coords = np.ascontiguousarray(mesh.coords, dtype=np.float64)
        cells = np.ascontiguousarray(mesh.cells, dtype=np.int32)
        cint = np.ascontiguousarray(mesh.cell_interior, dtype=np.uint8)
        s = np.ascontiguousarray(np.atleast_2d(s), dtype=np.float64)
        kappa = np.ascontiguousarray(np.atleast_2d(kappa), dtype=np.float64)
        if s.shape != kappa.shape or s.shape[1] != coords.shape[1]:
            raise ValueError("s and kappa must be [F][n_nodes]")
        m = _abi.Mesh(mesh.dim, coords.shape[1], mesh.n_dofs, coords.ctypes.data_as(C.POINTER(C.c_double)),
                      cells.shape[1], cells.ctypes.data_as(C.POINTER(C.c_int32)),
                      cint.ctypes.data_as(C.POINTER(C.c_uint8)), float(mesh.exterior_radius))
        o = opts_struct(opts, plan_only)
        check(lib().fpde_build(C.byref(m), s.shape[0], s.ctypes.data_as(C.POINTER(C.c_double)),
                               kappa.ctypes.data_as(C.POINTER(C.c_double)), C.byref(o), C.byref(self._h)),
              "fpde_build")
        self.n_fields = s.shape[0]
        self.n_dofs = int(mesh.n_dofs)
        self.n_nodes = int(coords.shape[1])
        self.dim = int(mesh.dim)

    # ------------------------------------------------------------------ apply
    def apply(self, x, y=None, parts: int = _abi.PART_ALL, stream=None):
        """y = A x for device tensors x, y of shape [F, N, R] (float64 or float32)."""
        import torch
        if x.dim() == 2:
            x = x.unsqueeze(-1)
        if x.shape[0] != self.n_fields or x.shape[1] != self.n_dofs or not x.is_cuda:
            raise ValueError(f"x must be a device tensor [F={self.n_fields}, N={self.n_dofs}, R]")
        if not x.is_contiguous():
            x = x.contiguous()
        if y is None:
            y = torch.empty_like(x)
        elif y.dtype != x.dtype or y.shape != x.shape or not y.is_contiguous():
            raise ValueError("y must be a contiguous tensor with the shape and dtype of x")
        if x.dtype is torch.float64:
            dtype = _abi.F64
        elif x.dtype is torch.float32:
            dtype = _abi.F32
        else:
            raise ValueError("x must be float64 or float32")
        st = lib().fpde_apply_parts(self._h, parts, dtype, x.data_ptr(), y.data_ptr(), x.shape[2],
                                    torch.cuda.current_stream().cuda_stream if stream is None
                                    else (stream if isinstance(stream, int) else stream.cuda_stream))
        if st:
            check(st, "fpde_apply")
        return y

    def apply_noalloc(self, x, y, stream=None):
        """fpde_apply_noalloc: y = A x for caller-allocated device tensors x, y [F, N, 1] (float64 or
        float32) with the library's static scratch as workspace (no device allocation)."""
        import torch
        if x.dim() != 3 or tuple(x.shape) != (self.n_fields, self.n_dofs, 1) or not x.is_cuda:
            raise ValueError(f"x must be a device tensor [F={self.n_fields}, N={self.n_dofs}, 1]")
        if not (x.is_contiguous() and y.is_contiguous()) or y.shape != x.shape or y.dtype != x.dtype:
            raise ValueError("x and y must be contiguous tensors of the same shape and dtype")
        if x.dtype is torch.float64:
            dtype = _abi.F64
        elif x.dtype is torch.float32:
            dtype = _abi.F32
        else:
            raise ValueError("x must be float64 or float32")
        check(lib().fpde_apply_noalloc(self._h, dtype, C.c_void_p(x.data_ptr()), C.c_void_p(y.data_ptr()), 1,
                                       _stream_handle(stream)), "fpde_apply_noalloc")
        return y

    def load_vector(self, f_nodal, stream=None):
        import torch
        f = f_nodal.contiguous()
        out = torch.empty(self.n_dofs, dtype=torch.float64, device=f.device)
        check(lib().fpde_load_vector(self._h, C.c_void_p(f.data_ptr()), C.c_void_p(out.data_ptr()),
                                     _stream_handle(stream)), "fpde_load_vector")
        return out

    def solve(self, F, u=None, rtol: float = 1e-10, maxit: int = 10000, stream=None, raise_on_noconv=True):
        """Solve A u = F (device float64 [F, N, R] or [F, N]); u is the initial guess (zeros if None)."""
        import torch
        if F.dim() == 2:
            F = F.unsqueeze(-1)
        if tuple(F.shape[:2]) != (self.n_fields, self.n_dofs) or not F.is_cuda or F.dtype != torch.float64:
            raise ValueError(f"F must be a float64 device tensor [F={self.n_fields}, N={self.n_dofs}, R]")
        F = F.contiguous()
        if u is None:
            u = torch.zeros_like(F)
        elif u.shape != F.shape or u.dtype != torch.float64 or not u.is_contiguous():
            raise ValueError("u must be a contiguous float64 tensor shaped like F")
        info = _abi.SolveInfo()
        st = lib().fpde_solve(self._h, C.c_void_p(F.data_ptr()), C.c_void_p(u.data_ptr()), F.shape[2], rtol,
                              maxit, C.byref(info), _stream_handle(stream))
        out = {"iterations": info.iterations, "rel_residual": info.rel_residual,
               "converged": bool(info.converged), "refinements": info.refinements,
               "cond_estimate": info.cond_estimate}
        if st != _abi.FPDE_OK and (raise_on_noconv or st != _abi.FPDE_ENOCONV):
            check(st, "fpde_solve")
        return u, out

    def apply_adjoint(self, w, u, alpha: float = 1.0, stream=None):
        """alpha (grad_s, grad_kappa) [F, n_nodes] of sum_r w_r^T A(s, kappa) u_r for device float64 [F, N, R]."""
        import torch
        if w.dim() == 2:
            w = w.unsqueeze(-1)
        if u.dim() == 2:
            u = u.unsqueeze(-1)
        for v in (w, u):
            if tuple(v.shape[:2]) != (self.n_fields, self.n_dofs) or not v.is_cuda or v.dtype != torch.float64:
                raise ValueError(f"w, u must be float64 device tensors [F={self.n_fields}, N={self.n_dofs}, R]")
        if w.shape != u.shape:
            raise ValueError("w and u must have the same shape")
        w = w.contiguous()
        u = u.contiguous()
        gs = torch.empty((self.n_fields, self.n_nodes), dtype=torch.float64, device=w.device)
        gk = torch.empty_like(gs)
        check(lib().fpde_apply_adjoint(self._h, float(alpha), C.c_void_p(w.data_ptr()), C.c_void_p(u.data_ptr()),
                                       w.shape[2],
                                       C.c_void_p(gs.data_ptr()), C.c_void_p(gk.data_ptr()), _stream_handle(stream)),
              "fpde_apply_adjoint")
        return gs, gk

    # ------------------------------------------------------------------ inspection
    def export(self, what: str, field: int = 0) -> np.ndarray:
        code = _abi.EXPORT[what]
        n = C.c_int64(0)
        check(lib().fpde_export(self._h, code, field, None, C.byref(n)), "fpde_export")
        out = np.zeros(n.value, dtype=np.float64 if what in _abi.EXPORT_IS_FLOAT else np.int64)
        check(lib().fpde_export(self._h, code, field, C.c_void_p(out.ctypes.data), C.byref(n)), "fpde_export")
        return out

    def profile(self, enable: bool) -> dict:
        """Start (enable=True, resets) or stop (enable=False) device-event profiling of apply."""
        pr = _abi.Profile()
        check(lib().fpde_profile(self._h, 1 if enable else 0, C.byref(pr)), "fpde_profile")
        return {name: getattr(pr, name) for name, _ in pr._fields_}

    def stats(self) -> dict:
        s = _abi.Stats()
        check(lib().fpde_stats(self._h, C.byref(s)), "fpde_stats")
        return {name: getattr(s, name) for name, _ in s._fields_}

    def close(self):
        if self._h:
            lib().fpde_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
