"""MI355X (gfx950) implementation of the explicit RBF-FD Poisson iteration of
Vehovar, Rot and Kosec (arXiv 2502.12878).

This package is a thin Python binding over the C ABI in ``include/rbf.h``:
torch tensors provide device memory and the stream; every step of the method
(node building, neighbour search, weight solves, sweeps, adjoint) runs in the
library's HIP kernels.  ``Problem`` wraps one library handle.
"""
from __future__ import annotations

import ctypes as C

import numpy as np

from . import _abi
from ._abi import (RBF_EDIVERGED, RBF_EINVAL, RBF_ENOTCONVERGED, RBF_ESINGULAR, RBF_MODE_FP64, RBF_MODE_MIXED,
                   RBF_OK, LibraryMissing)

__all__ = ["Problem", "RbfError", "SolveK", "LibraryMissing", "RBF_MODE_FP64", "RBF_MODE_MIXED"]


class RbfError(RuntimeError):
    def __init__(self, status: int, message: str):
        self.status = status
        super().__init__(f"[{_abi.lib().rbf_status_string(status).decode()}] {message}")


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else None


class Problem:
    """One library handle on a GPU; buffers come from torch's caching allocator."""

    def __init__(self, device: int = 0, stream=None, use_torch_allocator: bool = True):
        import torch
        self.torch = torch
        self.device = torch.device("cuda", device)
        self._lib = _abi.lib()
        if stream is None:
            stream = torch.cuda.current_stream(self.device)
        self.stream = stream
        self._alloc = None
        if use_torch_allocator:
            dev = device

            def _alloc_cb(nbytes, ctx):
                try:
                    return torch.cuda.caching_allocator_alloc(int(nbytes), dev, self.stream)
                except Exception:
                    return None

            def _free_cb(p, ctx):
                torch.cuda.caching_allocator_delete(p)

            self._alloc_fn = _abi.ALLOC_FN(_alloc_cb)
            self._free_fn = _abi.FREE_FN(_free_cb)
            self._alloc = _abi.rbf_allocator(self._alloc_fn, self._free_fn, None)
        h = C.c_void_p()
        st = self._lib.rbf_create(C.byref(h), device, C.c_void_p(stream.cuda_stream),
                                  C.byref(self._alloc) if self._alloc is not None else None)
        if st != RBF_OK:
            raise RbfError(st, "rbf_create failed")
        self.h = h

    # ------------------------------------------------------------------ basics
    def close(self):
        if getattr(self, "h", None):
            self._lib.rbf_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, st, what):
        if st != RBF_OK:
            raise RbfError(st, f"{what}: {self._lib.rbf_last_error(self.h).decode()}")

    @property
    def sizes(self):
        d, N, Ni, nm = C.c_int(), C.c_int64(), C.c_int64(), C.c_int32()
        self._check(self._lib.rbf_get_sizes(self.h, C.byref(d), C.byref(N), C.byref(Ni), C.byref(nm)), "sizes")
        return {"dim": d.value, "N": N.value, "N_interior": Ni.value, "n_max": nm.value}

    def _cuda(self, t, dtype):
        torch = self.torch
        if not isinstance(t, torch.Tensor):
            t = torch.as_tensor(np.ascontiguousarray(t))
        return t.to(device=self.device, dtype=dtype).contiguous()

    # ------------------------------------------------------------------ nodes
    def build_nodes(self, dim: int, side: int, jitter: float, seed: int):
        torch = self.torch
        N = side ** dim
        xyz = torch.empty((dim, N), dtype=torch.float64, device=self.device)
        typ = torch.empty(N, dtype=torch.int8, device=self.device)
        self._check(self._lib.rbf_build_nodes(self.h, dim, side, jitter, seed & 0xFFFFFFFFFFFFFFFF, _ptr(xyz),
                                              _ptr(typ)), "build_nodes")
        return xyz, typ

    def set_nodes(self, xyz, typ):
        torch = self.torch
        xyz = self._cuda(xyz, torch.float64)
        typ = self._cuda(typ, torch.int8)
        dim, N = xyz.shape
        self._check(self._lib.rbf_set_nodes(self.h, dim, N, _ptr(xyz), _ptr(typ)), "set_nodes")

    def set_normals(self, normals):
        """Unit outward normals [dim, N] of the Neumann nodes (type 2)."""
        nv = self._cuda(normals, self.torch.float64)
        self._check(self._lib.rbf_set_normals(self.h, _ptr(nv)), "set_normals")

    # ------------------------------------------------------------------ stencils and weights
    def build_stencils(self, n=None, n_per_node=None):
        torch = self.torch
        if n_per_node is not None:
            npn = self._cuda(n_per_node, torch.int16)
            self._check(self._lib.rbf_build_stencils(self.h, 0, _ptr(npn)), "build_stencils")
        else:
            self._check(self._lib.rbf_build_stencils(self.h, int(n), None), "build_stencils")

    def compute_weights(self, m=None, m_per_node=None, keep_fp32: bool = False):
        torch = self.torch
        if m_per_node is not None:
            mpn = self._cuda(m_per_node, torch.int8)
            st = self._lib.rbf_compute_weights(self.h, -1, _ptr(mpn), int(keep_fp32))
        else:
            st = self._lib.rbf_compute_weights(self.h, int(m), None, int(keep_fp32))
        self._check(st, "compute_weights")

    def get_stencils(self) -> np.ndarray:
        s = self.sizes
        out = np.empty((s["N"], s["n_max"]), dtype=np.int32)
        self._check(self._lib.rbf_get_stencils(self.h, out.ctypes.data_as(C.c_void_p)), "get_stencils")
        return out

    def get_weights(self) -> np.ndarray:
        s = self.sizes
        out = np.empty((s["N"], s["n_max"]), dtype=np.float64)
        self._check(self._lib.rbf_get_weights(self.h, out.ctypes.data_as(C.c_void_p)), "get_weights")
        return out

    def set_stencils(self, idx: np.ndarray):
        idx = np.ascontiguousarray(idx, dtype=np.int32)
        self._check(self._lib.rbf_set_stencils(self.h, idx.ctypes.data_as(C.c_void_p), idx.shape[1]),
                    "set_stencils")

    def set_weights(self, w: np.ndarray, keep_fp32: bool = False):
        w = np.ascontiguousarray(w, dtype=np.float64)
        self._check(self._lib.rbf_set_weights(self.h, w.ctypes.data_as(C.c_void_p), int(keep_fp32)),
                    "set_weights")

    def autotune(self):
        self._check(self._lib.rbf_autotune(self.h), "autotune")

    def operator_info(self) -> dict:
        info = _abi.rbf_operator_info()
        self._check(self._lib.rbf_get_operator_info(self.h, C.byref(info)), "operator_info")
        return info.as_dict()

    def last_sweep_time(self):
        s, n = C.c_double(), C.c_int64()
        self._check(self._lib.rbf_last_sweep_time(self.h, C.byref(s), C.byref(n)), "last_sweep_time")
        return s.value, n.value

    # ------------------------------------------------------------------ operators
    def apply(self, u):
        u = self._cuda(u, self.torch.float64)
        out = self.torch.empty_like(u)
        self._check(self._lib.rbf_apply(self.h, _ptr(u), _ptr(out)), "apply")
        return out

    def apply_transpose(self, v):
        v = self._cuda(v, self.torch.float64)
        out = self.torch.empty_like(v)
        self._check(self._lib.rbf_apply_transpose(self.h, _ptr(v), _ptr(out)), "apply_transpose")
        return out

    def residual(self, f, u) -> float:
        f = self._cuda(f, self.torch.float64)
        u = self._cuda(u, self.torch.float64)
        r = C.c_double()
        self._check(self._lib.rbf_residual(self.h, _ptr(f), _ptr(u), C.byref(r)), "residual")
        return r.value

    def residual_noalloc(self, f, u, out=None):
        """max|L u - f| into the one-element device tensor ``out`` (created if
        None) by the no-allocation entry point: asynchronous on the handle's
        stream; at most 2^21 nodes; concurrent calls on one device race."""
        torch = self.torch
        f = self._cuda(f, torch.float64)
        u = self._cuda(u, torch.float64)
        if out is None:
            out = torch.empty(1, dtype=torch.float64, device=self.device)
        self._check(self._lib.rbf_residual_noalloc(self.h, _ptr(f), _ptr(u), _ptr(out)), "residual_noalloc")
        return out

    # ------------------------------------------------------------------ iteration
    def iterate(self, f, u, dt, max_steps, tol_rel=0.0, chunk=500, mode=RBF_MODE_FP64, inner_steps=500,
                stall_chunks=0, u_ref=None, err_target=0.0):
        """Run the explicit iteration in place on ``u`` (a float64 CUDA tensor).

        Returns (status, report).  Statuses EDIVERGED and ENOTCONVERGED are
        returned, not raised; any other failure raises RbfError.
        """
        torch = self.torch
        f = self._cuda(f, torch.float64)
        if not (isinstance(u, torch.Tensor) and u.is_cuda and u.dtype == torch.float64 and u.is_contiguous()):
            raise TypeError("u must be a contiguous float64 CUDA tensor (updated in place)")
        uref = None if u_ref is None else self._cuda(u_ref, torch.float64)
        p = _abi.rbf_iter_params(float(dt), int(max_steps), float(tol_rel), int(chunk), int(mode),
                                 int(inner_steps), int(stall_chunks),
                                 uref.data_ptr() if uref is not None else None, float(err_target))
        rep = _abi.rbf_iter_report()
        st = self._lib.rbf_iterate(self.h, _ptr(f), _ptr(u), C.byref(p), C.byref(rep))
        if st not in (RBF_OK, RBF_EDIVERGED, RBF_ENOTCONVERGED):
            self._check(st, "iterate")
        return st, rep.as_dict()

    def forward_ckpt(self, f, u0, K, every, dt, keep_checkpoints=True):
        torch = self.torch
        f = self._cuda(f, torch.float64)
        u0 = self._cuda(u0, torch.float64)
        N = u0.numel()
        ck = torch.empty((K // every + 1, N), dtype=torch.float64, device=self.device) if keep_checkpoints else None
        uK = torch.empty_like(u0)
        self._check(self._lib.rbf_forward_ckpt(self.h, _ptr(f), _ptr(u0), int(K), int(every), _ptr(ck), _ptr(uK),
                                               float(dt)), "forward_ckpt")
        return ck, uK

    def adjoint_f(self, gK, K, every, dt, ckpt=None):
        torch = self.torch
        gK = self._cuda(gK, torch.float64)
        grad = torch.empty_like(gK)
        self._check(self._lib.rbf_adjoint_f(self.h, _ptr(gK), int(K), int(every), _ptr(ckpt), _ptr(grad),
                                            float(dt)), "adjoint_f")
        return grad


def _solvek_cls():
    import torch

    class SolveK(torch.autograd.Function):
        """u_K(f): K explicit steps from u0 with source f (checkpointed);
        backward gives dJ/df by the library's transposed sweeps."""

        @staticmethod
        def forward(ctx, f, problem, u0, K, every, dt):
            ck, uK = problem.forward_ckpt(f.detach(), u0, K, every, dt)
            ctx.problem, ctx.K, ctx.every, ctx.dt = problem, K, every, dt
            ctx.save_for_backward(ck)
            return uK

        @staticmethod
        def backward(ctx, gK):
            (ck,) = ctx.saved_tensors
            g = ctx.problem.adjoint_f(gK.contiguous(), ctx.K, ctx.every, ctx.dt, ck)
            return g, None, None, None, None, None

    return SolveK


class _Lazy:
    _cls = None

    def __getattr__(self, name):
        if _Lazy._cls is None:
            _Lazy._cls = _solvek_cls()
        return getattr(_Lazy._cls, name)


SolveK = _Lazy()
