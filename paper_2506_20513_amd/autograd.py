"""PyTorch autograd around the C ABI.

Two functions, both differentiable in eps_r and sigma (arrays over the total
grid, CPML included, [NY][NX] float32 on the GPU):

  traces(problem, eps_r, sigma) -> [S][nt][R]
      fdtd_forward with checkpoints kept in the problem's workspace; the
      backward pass is fdtd_adjoint with the incoming trace gradient as the
      adjoint source (the exact transpose of the discrete forward map, Sec.
      2.1 Eqs. (8)-(13)), so any loss on the traces can be used.

  misfit(problem, eps_r, sigma, observed) -> J = 1/2 sum (traces - observed)^2
      (Eq. (6)); one fwi_gradient call computes J and its gradient together,
      the backward pass only scales the stored gradient.

The problem owns one workspace per mode and reuses it: a backward pass must
run before the next forward call on the same problem, which is how an
optimisation loop uses them; otherwise the backward pass raises.
"""
from __future__ import annotations

import numpy as np
import torch

from . import fwi


def _check_tensor(name, t, shape, dtype=torch.float32):
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name}: expected a torch tensor")
    if not t.is_cuda:
        raise ValueError(f"{name}: must be on the GPU")
    if t.dtype != dtype:
        raise TypeError(f"{name}: dtype {t.dtype}, expected {dtype}")
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name}: shape {tuple(t.shape)}, expected {tuple(shape)}")
    if not t.is_contiguous():
        raise ValueError(f"{name}: must be contiguous")


class Problem:
    """Grid, acquisition geometry and source wavelets of one inversion.

    grid: fwi.fwi_grid; src [S][2] and rec [S][R][2] int32 cell indices on the
    total grid; wavelet [S][nt] (array or tensor, line current in A, sampled
    at (n + 1/2) dt)."""

    def __init__(self, grid, src, rec, wavelet, device="cuda"):
        self.grid = grid
        self.device = torch.device(device)
        self.NX = grid.nx + 2 * grid.npml
        self.NY = grid.ny + 2 * grid.npml
        self.nt = grid.nt
        src = np.ascontiguousarray(src, np.int32).reshape(-1, 2)
        self.S = src.shape[0]
        rec = np.ascontiguousarray(rec, np.int32).reshape(self.S, -1, 2)
        self.R = rec.shape[1]
        self._src, self._rec = src, rec
        self._ws = {}
        self._generation = 0
        self.set_wavelet(wavelet)

    def set_wavelet(self, wavelet):
        w = torch.as_tensor(wavelet, dtype=torch.float32).to(self.device).contiguous()
        _check_tensor("wavelet", w, (self.S, self.nt))
        self.wavelet = w
        self.geom = fwi.Geometry(self._src, self._rec, w)
        self._generation += 1          # a changed source invalidates saved state

    @property
    def model_shape(self):
        return (self.NY, self.NX)

    @property
    def trace_shape(self):
        return (self.S, self.nt, self.R)

    def workspace(self, mode):
        """The workspace for `mode`.  The checkpointing modes need tens to
        hundreds of GB on large grids, so at most one of them is kept: taking
        one frees the other (and invalidates saved checkpoints)."""
        ws = self._ws.get(mode)
        if ws is None:
            if mode != fwi.FWI_SAVE_NONE:
                for m in [m for m in self._ws if m != fwi.FWI_SAVE_NONE]:
                    del self._ws[m]
                self._generation += 1
                torch.cuda.empty_cache()
            ws = fwi.alloc_workspace(fwi.workspace_bytes(self.grid, self.geom, mode), self.device)
            self._ws[mode] = ws
        return ws

    def release(self):
        """Free the workspaces (they are re-allocated on demand)."""
        self._ws.clear()
        self._generation += 1

    def _next(self):
        self._generation += 1
        return self._generation


class _Traces(torch.autograd.Function):
    @staticmethod
    def forward(ctx, eps_r, sigma, prob):
        _check_tensor("eps_r", eps_r, prob.model_shape)
        _check_tensor("sigma", sigma, prob.model_shape)
        # without a gradient to come, nothing needs saving for an adjoint
        mode = fwi.FWI_SAVE_CHECKPOINT if any(ctx.needs_input_grad[:2]) else fwi.FWI_SAVE_NONE
        ws = prob.workspace(mode)
        tr = torch.empty(prob.trace_shape, dtype=torch.float32, device=prob.device)
        fwi.fdtd_forward(prob.grid, prob.geom, eps_r, sigma, tr, mode, ws)
        ctx.prob = prob
        ctx.generation = prob._next()
        ctx.save_for_backward(eps_r, sigma)
        return tr

    @staticmethod
    def backward(ctx, grad_traces):
        prob = ctx.prob
        if prob._generation != ctx.generation:
            raise RuntimeError("traces: the problem ran another forward pass (or changed its "
                               "wavelet) before this backward pass; its checkpoints are gone")
        eps_r, sigma = ctx.saved_tensors
        g = grad_traces.to(torch.float32).contiguous()
        _check_tensor("grad_traces", g, prob.trace_shape)
        ge = torch.empty(prob.model_shape, dtype=torch.float32, device=prob.device)
        gs = torch.empty_like(ge)
        fwi.fdtd_adjoint(prob.grid, prob.geom, eps_r, sigma, g, ge, gs, None,
                         fwi.FWI_SAVE_CHECKPOINT, prob.workspace(fwi.FWI_SAVE_CHECKPOINT))
        return ge, gs, None


class _Misfit(torch.autograd.Function):
    @staticmethod
    def forward(ctx, eps_r, sigma, observed, prob):
        _check_tensor("eps_r", eps_r, prob.model_shape)
        _check_tensor("sigma", sigma, prob.model_shape)
        _check_tensor("observed", observed, prob.trace_shape)
        ws = prob.workspace(fwi.GRADIENT_WORKSPACE)
        mis = torch.empty(1, dtype=torch.float64, device=prob.device)
        ge = torch.empty(prob.model_shape, dtype=torch.float32, device=prob.device)
        gs = torch.empty_like(ge)
        fwi.fwi_gradient(prob.grid, prob.geom, eps_r, sigma, observed, mis, ge, gs, None, ws)
        prob._next()
        ctx.save_for_backward(ge, gs)
        return mis[0]

    @staticmethod
    def backward(ctx, grad_out):
        ge, gs = ctx.saved_tensors
        g = grad_out.to(torch.float32)
        return ge * g, gs * g, None, None


def traces(prob: Problem, eps_r, sigma):
    """Receiver traces [S][nt][R] of the model; differentiable."""
    return _Traces.apply(eps_r.contiguous(), sigma.contiguous(), prob)


def misfit(prob: Problem, eps_r, sigma, observed):
    """J = 1/2 sum (traces - observed)^2 as a float64 scalar (reduced in
    double on the GPU); its gradient comes from the same call."""
    return _Misfit.apply(eps_r.contiguous(), sigma.contiguous(), observed.contiguous(), prob)
