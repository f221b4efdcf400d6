"""Helpers for GPU tests: run the HIP library through its C ABI on torch
device memory and bring results back as numpy arrays."""
from __future__ import annotations

import numpy as np

from paper_2506_20513_amd import fwi


def rel_l2(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / nb) if nb > 0 else float(np.linalg.norm(a))


def mask_near(shape, src, rec, radius=3):
    """True away from sources and receivers (3-cell radius masked)."""
    NY, NX = shape
    jj, ii = np.mgrid[0:NY, 0:NX]
    m = np.ones(shape, dtype=bool)
    pts = np.concatenate([np.asarray(src).reshape(-1, 2), np.asarray(rec).reshape(-1, 2)])
    for i, j in np.unique(pts, axis=0):
        m &= (ii - i) ** 2 + (jj - j) ** 2 > radius * radius
    return m


class Run:
    """One problem on the device: grid, geometry, model, wavelet."""

    def __init__(self, grid, src, rec, wavelet, eps, sig, device="cuda"):
        import torch
        self.torch = torch
        self.grid = grid
        self.dev = device
        self.w = torch.from_numpy(np.ascontiguousarray(wavelet, np.float32)).to(device)
        self.geom = fwi.Geometry(src, rec, self.w)
        self.eps = torch.from_numpy(np.ascontiguousarray(eps, np.float32)).to(device)
        self.sig = torch.from_numpy(np.ascontiguousarray(sig, np.float32)).to(device)
        self.S, self.R, self.nt = self.geom.nshots, self.geom.nrec, grid.nt
        self.NX, self.NY = grid.nx + 2 * grid.npml, grid.ny + 2 * grid.npml

    def workspace(self, mode):
        return fwi.alloc_workspace(fwi.workspace_bytes(self.grid, self.geom, mode), self.dev)

    def forward(self, mode=fwi.FWI_SAVE_NONE, ws=None):
        torch = self.torch
        ws = self.workspace(mode) if ws is None else ws
        tr = torch.full((self.S, self.nt, self.R), float("nan"), device=self.dev)
        fwi.fdtd_forward(self.grid, self.geom, self.eps, self.sig, tr, mode, ws)
        torch.cuda.synchronize()
        return tr, ws

    def adjoint(self, residual, mode, ws, want_src_adjoint=False):
        torch = self.torch
        res = torch.from_numpy(np.ascontiguousarray(residual, np.float32)).to(self.dev) \
            if isinstance(residual, np.ndarray) else residual
        ge = torch.full((self.NY, self.NX), float("nan"), device=self.dev)
        gs = torch.full((self.NY, self.NX), float("nan"), device=self.dev)
        sa = torch.full((self.S, self.nt), float("nan"), device=self.dev) if want_src_adjoint else None
        fwi.fdtd_adjoint(self.grid, self.geom, self.eps, self.sig, res, ge, gs, sa, mode, ws)
        torch.cuda.synchronize()
        return ge, gs, sa

    def gradient(self, observed, want_traces=True, ws=None):
        torch = self.torch
        ob = torch.from_numpy(np.ascontiguousarray(observed, np.float32)).to(self.dev) \
            if isinstance(observed, np.ndarray) else observed
        ws = self.workspace(fwi.GRADIENT_WORKSPACE) if ws is None else ws
        mis = torch.full((1,), float("nan"), dtype=torch.float64, device=self.dev)
        ge = torch.full((self.NY, self.NX), float("nan"), device=self.dev)
        gs = torch.full((self.NY, self.NX), float("nan"), device=self.dev)
        tr = torch.full((self.S, self.nt, self.R), float("nan"), device=self.dev) if want_traces else None
        fwi.fwi_gradient(self.grid, self.geom, self.eps, self.sig, ob, mis, ge, gs, tr, ws)
        torch.cuda.synchronize()
        return mis, ge, gs, tr


def np_(t):
    return t.detach().cpu().numpy()


def gradient_regions(shape, npml, src, rec, radius=3):
    """Named boolean masks of the total grid for per-region gradient checks:
    each CPML strip (left, right, top, bottom; the PEC ring excluded), the
    deep half of the interior, and the interior with a `radius`-cell disc
    around every source and receiver removed."""
    NY, NX = shape
    jj, ii = np.mgrid[0:NY, 0:NX]
    upd = (ii >= 1) & (ii <= NX - 2) & (jj >= 1) & (jj <= NY - 2)
    interior = (ii >= npml) & (ii <= NX - 1 - npml) & (jj >= npml) & (jj <= NY - 1 - npml)
    out = {}
    if npml > 0:
        out["cpml_left"] = upd & (ii < npml)
        out["cpml_right"] = upd & (ii > NX - 1 - npml)
        out["cpml_top"] = upd & (jj < npml)
        out["cpml_bottom"] = upd & (jj > NY - 1 - npml)
    out["deep_half"] = interior & (jj >= npml + (NY - 2 * npml) // 2)
    out["interior_masked"] = interior & mask_near(shape, src, rec, radius)
    return out


def region_errors(g, og, regions, floor=1e-3):
    """Relative L2 error of g against og in every region.  A region that
    holds less than `floor` of og's whole norm (one the waves barely reach in
    the window) is measured against that floor instead of its own norm: FP32
    rounding leaves errors of about 1e-7 to 1e-6 of the whole norm anywhere
    the waves have been, which a nearly empty region cannot be held to
    relative to itself."""
    g = np.asarray(g, dtype=np.float64)
    og = np.asarray(og, dtype=np.float64)
    whole = np.linalg.norm(og)
    out = {}
    for k, m in regions.items():
        ref = max(np.linalg.norm(og[m]), floor * whole)
        out[k] = float(np.linalg.norm(g[m] - og[m]) / ref) if ref > 0 else 0.0
    return out


def late_window(tr, frac=1.0 / 3.0):
    """The last `frac` of the time samples of traces [S][nt][R]."""
    nt = tr.shape[1]
    return tr[:, nt - max(1, int(round(nt * frac))):, :]
