"""Binding of the total-variation regularisation kernel (include/fwi_tv.h;
Sec. 3.4, Algorithm 3 of arXiv 2506.20513)."""
from __future__ import annotations

import ctypes

import torch

from . import fwi

MAX_FIELDS = 4
EXPORTED = ("fwi_tv_workspace_bytes", "fwi_tv_gradient")
_ready = False


def lib() -> ctypes.CDLL:
    global _ready
    L = fwi.lib()
    if not _ready:
        i32, vp, sz, fp = ctypes.c_int32, ctypes.c_void_p, ctypes.c_size_t, ctypes.POINTER(ctypes.c_float)
        L.fwi_tv_workspace_bytes.argtypes = [i32, i32, i32]
        L.fwi_tv_workspace_bytes.restype = sz
        L.fwi_tv_gradient.argtypes = [vp, vp, i32, i32, i32, fp, fp, fp, i32, vp, sz, vp]
        L.fwi_tv_gradient.restype = ctypes.c_int
        _ready = True
    return L


def workspace_bytes(nfield: int, ny: int, nx: int) -> int:
    return int(lib().fwi_tv_workspace_bytes(nfield, ny, nx))


def _floats(vals, n):
    vals = list(vals) if hasattr(vals, "__len__") else [vals] * n
    if len(vals) != n:
        raise ValueError(f"expected {n} values, got {len(vals)}")
    return (ctypes.c_float * n)(*[float(v) for v in vals])


class TV:
    """Algorithm 3 for `nfield` fields of ny x nx cells with a workspace of
    its own.  __call__(X, grad) adds weight * (X - TVdenoise(X)) to grad
    (both [nfield][ny][nx] float32 on the GPU, contiguous)."""

    def __init__(self, nfield, ny, nx, mu, lam, weight, iters, device="cuda"):
        self.nfield, self.ny, self.nx, self.iters = int(nfield), int(ny), int(nx), int(iters)
        self.mu = _floats(mu, self.nfield)
        self.lam = _floats(lam, self.nfield)
        self.weight = _floats(weight, self.nfield)
        nb = workspace_bytes(self.nfield, self.ny, self.nx)
        if nb == 0:
            raise ValueError("fwi_tv_workspace_bytes: unsupported shape")
        self.ws = fwi.alloc_workspace(nb, device)
        self.ws_bytes = nb

    def __call__(self, X: torch.Tensor, grad: torch.Tensor, stream=None):
        shape = (self.nfield, self.ny, self.nx)
        for name, t in (("X", X), ("grad", grad)):
            if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != torch.float32:
                raise TypeError(f"{name}: expected a float32 GPU tensor")
            if tuple(t.shape) != shape or not t.is_contiguous():
                raise ValueError(f"{name}: expected a contiguous tensor of shape {shape}")
        st = lib().fwi_tv_gradient(X.data_ptr(), grad.data_ptr(), self.nfield, self.ny, self.nx,
                                   self.mu, self.lam, self.weight, self.iters,
                                   fwi._wsptr(self.ws), self.ws_bytes, fwi._stream(stream))
        if st != 0:
            raise fwi.FwiError(st, "fwi_tv_gradient")
        return grad
