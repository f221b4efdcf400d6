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


BYTES_PER_CELL_ITER = 28   # read U, Bx, By, X; write U, Bx, By (float32)


def main(argv=None):
    """Throughput of the Algorithm 3 kernel: eps_r and sigma fields of the
    given size, `iters` iterations per call."""
    import argparse
    import json
    import sys
    ap = argparse.ArgumentParser()
    ap.add_argument("--size", default="1064x2088", help="field rows x columns")
    ap.add_argument("--iters", type=int, default=50)
    ap.add_argument("--reps", type=int, default=5)
    args = ap.parse_args(argv)
    if not torch.cuda.is_available():
        print("tv: no GPU visible", file=sys.stderr)
        return 1
    ny, nx = (int(v) for v in args.size.split("x"))
    g = torch.Generator(device="cuda").manual_seed(0)
    X = torch.rand(2, ny, nx, generator=g, device="cuda") * torch.tensor([17.0, 0.05], device="cuda")[:, None, None] + torch.tensor([3.0, 0.001], device="cuda")[:, None, None]
    G = torch.zeros_like(X)
    op = TV(2, ny, nx, 8.0, 2.0, 1e-3, args.iters)
    op(X, G)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(args.reps):
        op(X, G)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / args.reps
    per_iter = ms / args.iters
    gbps = BYTES_PER_CELL_ITER * 2 * ny * nx / (per_iter * 1e-3) / 1e9
    print(json.dumps({"fields": 2, "shape": [ny, nx], "iters": args.iters, "ms_per_call": round(ms, 4),
                      "ms_per_iteration": round(per_iter, 5), "algorithmic_GBps": round(gbps, 1),
                      "frac_of_8TBps": round(gbps / 8000.0, 3)}), flush=True)
    return 0


if __name__ == "__main__":
    raise SystemExit(main())
