"""Thin ctypes binding of libfwi.so (C ABI in include/fwi.h).

Argument marshalling only: every step of the forward, adjoint and gradient
computation runs in the HIP library.  Device arrays are passed as torch CUDA
tensors (or raw integer device addresses); geometry is host int32 numpy
arrays.  The calls are asynchronous on the given stream (default: torch's
current stream).  A missing library raises at load time; there is no
fallback.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfwi.so")

FWI_OK = 0
FWI_EINVAL = -1
FWI_ECFL = -2
FWI_EGEOM = -3
FWI_ENOMEM = -4
FWI_EHIP = -5
FWI_ENONFINITE = -6
FWI_ESCRATCH = -7
STATIC_SCRATCH_BYTES = 64 << 20   # FWI_STATIC_SCRATCH_BYTES

FWI_SAVE_NONE = 0
FWI_SAVE_CHECKPOINT = 1
FWI_SAVE_HISTORY = 2
GRADIENT_WORKSPACE = -1   # fwi_workspace_bytes mode for fwi_gradient

EXPORTED = ("fwi_workspace_bytes", "fdtd_forward", "fdtd_adjoint", "fwi_gradient",
            "fwi_gradient_timed", "fwi_checkpoint_interval", "fwi_strerror",
            "fwi_batch_workspace_bytes", "fwi_batch_plan_create", "fwi_batch_plan_run",
            "fwi_batch_plan_info", "fwi_batch_plan_destroy", "fwi_gradient_static",
            "fwi_gradient_ex")


class FwiError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        super().__init__(f"{where}: status {status} ({strerror(status)})")


class fwi_grid(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
                ("npml", ctypes.c_int32), ("nt", ctypes.c_int32),
                ("dx", ctypes.c_double), ("dy", ctypes.c_double), ("dt", ctypes.c_double),
                ("cpml_order", ctypes.c_int32),
                ("cpml_sigma_scale", ctypes.c_double),
                ("cpml_kappa_max", ctypes.c_double),
                ("cpml_alpha_max", ctypes.c_double)]


TIMING_MAX_KINDS = 8


class fwi_kernel_time(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 32), ("launches", ctypes.c_int32),
                ("timed", ctypes.c_int32), ("avg_ms", ctypes.c_double),
                ("cell_updates", ctypes.c_double)]


class fwi_timing(ctypes.Structure):
    _fields_ = [("sample_every", ctypes.c_int32), ("nkinds", ctypes.c_int32),
                ("kind", fwi_kernel_time * TIMING_MAX_KINDS), ("shot_groups", ctypes.c_int32)]

    def as_dict(self):
        return {self.kind[k].name.decode(): dict(launches=self.kind[k].launches,
                                                 timed=self.kind[k].timed,
                                                 avg_ms=self.kind[k].avg_ms,
                                                 cell_updates=self.kind[k].cell_updates)
                for k in range(self.nkinds)}


class fwi_geom(ctypes.Structure):
    _fields_ = [("nshots", ctypes.c_int32), ("nrec", ctypes.c_int32),
                ("src_ij", ctypes.POINTER(ctypes.c_int32)),
                ("rec_ij", ctypes.POINTER(ctypes.c_int32)),
                ("wavelet", ctypes.c_void_p)]


_lib = None


class fwi_batch_problem(ctypes.Structure):
    _fields_ = [("grid", fwi_grid), ("geom", fwi_geom),
                ("eps_r", ctypes.c_void_p), ("sigma", ctypes.c_void_p),
                ("observed", ctypes.c_void_p), ("misfit", ctypes.c_void_p),
                ("grad_eps_r", ctypes.c_void_p), ("grad_sigma", ctypes.c_void_p)]


BATCH_MAX_TUNE = 16
FWI_TUNE_BANDS = 1
FWI_TUNE_DEPTH = 2
FWI_BATCH_DEPTH8 = 4


class fwi_batch_info(ctypes.Structure):
    _fields_ = [("nproblems", ctypes.c_int32), ("checkpoint_interval", ctypes.c_int32),
                ("band_rows", ctypes.c_int32), ("depth", ctypes.c_int32),
                ("steps", ctypes.c_int32), ("stencil_launches", ctypes.c_int32),
                ("graph", ctypes.c_int32), ("ntune", ctypes.c_int32),
                ("tune_depth", ctypes.c_int32 * BATCH_MAX_TUNE),
                ("tune_rows", ctypes.c_int32 * BATCH_MAX_TUNE),
                ("tune_ms", ctypes.c_double * BATCH_MAX_TUNE)]

    def as_dict(self):
        return {"nproblems": self.nproblems, "checkpoint_interval": self.checkpoint_interval,
                "band_rows": self.band_rows, "depth": self.depth, "steps": self.steps,
                "stencil_launches": self.stencil_launches, "graph": bool(self.graph),
                "tuning": [(self.tune_depth[k], self.tune_rows[k], self.tune_ms[k])
                           for k in range(self.ntune)]}


def lib() -> ctypes.CDLL:
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -m paper_2506_20513_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        G, Q = ctypes.POINTER(fwi_grid), ctypes.POINTER(fwi_geom)
        vp, sz = ctypes.c_void_p, ctypes.c_size_t
        L.fwi_workspace_bytes.argtypes = [G, Q, ctypes.c_int, ctypes.POINTER(sz)]
        L.fwi_checkpoint_interval.argtypes = [G, Q, ctypes.POINTER(ctypes.c_int32)]
        L.fdtd_forward.argtypes = [G, Q, vp, vp, vp, ctypes.c_int, vp, sz, vp]
        L.fdtd_adjoint.argtypes = [G, Q, vp, vp, vp, vp, vp, vp, ctypes.c_int, vp, sz, vp]
        L.fwi_gradient.argtypes = [G, Q, vp, vp, vp, vp, vp, vp, vp, vp, sz, vp]
        L.fwi_gradient_timed.argtypes = [G, Q, vp, vp, vp, vp, vp, vp, vp, vp, sz, vp,
                                         ctypes.POINTER(fwi_timing)]
        L.fwi_gradient_static.argtypes = [G, Q, vp, vp, vp, vp, vp, vp, vp, vp]
        L.fwi_gradient_ex.argtypes = [G, Q, vp, vp, vp, vp, vp, vp, vp, vp, sz, vp,
                                      ctypes.POINTER(fwi_timing), ctypes.c_int32]
        L.fwi_strerror.argtypes = [ctypes.c_int]
        L.fwi_strerror.restype = ctypes.c_char_p
        BP = ctypes.POINTER(fwi_batch_problem)
        L.fwi_batch_workspace_bytes.argtypes = [ctypes.c_int32, BP, ctypes.POINTER(sz)]
        L.fwi_batch_plan_create.argtypes = [ctypes.c_int32, BP, vp, sz, ctypes.c_int32, vp,
                                            ctypes.POINTER(vp)]
        L.fwi_batch_plan_run.argtypes = [vp, ctypes.c_int32, vp]
        L.fwi_batch_plan_info.argtypes = [vp, ctypes.POINTER(fwi_batch_info)]
        L.fwi_batch_plan_destroy.argtypes = [vp]
        L.fwi_batch_plan_destroy.restype = None
        for name in ("fwi_workspace_bytes", "fwi_checkpoint_interval", "fdtd_forward",
                     "fdtd_adjoint", "fwi_gradient", "fwi_gradient_timed", "fwi_gradient_static",
                     "fwi_gradient_ex",
                     "fwi_batch_workspace_bytes", "fwi_batch_plan_create", "fwi_batch_plan_run",
                     "fwi_batch_plan_info"):
            getattr(L, name).restype = ctypes.c_int
        _lib = L
    return _lib


def strerror(status: int) -> str:
    return lib().fwi_strerror(int(status)).decode()


# ---------------------------------------------------------------------------
def make_grid(nx, ny, npml, nt, dx, dy, dt, cpml_order=3, cpml_sigma_scale=1.0,
              cpml_kappa_max=1.0, cpml_alpha_max=0.0) -> fwi_grid:
    return fwi_grid(int(nx), int(ny), int(npml), int(nt), float(dx), float(dy),
                    float(dt), int(cpml_order), float(cpml_sigma_scale),
                    float(cpml_kappa_max), float(cpml_alpha_max))


def grid_from_config(cfg) -> fwi_grid:
    return make_grid(**cfg.grid_kwargs())


class Geometry:
    """Host geometry plus the device wavelet address, kept alive together."""

    def __init__(self, src_ij, rec_ij, wavelet=None):
        self.src = np.ascontiguousarray(src_ij, dtype=np.int32).reshape(-1, 2)
        S = self.src.shape[0]
        self.rec = np.ascontiguousarray(rec_ij, dtype=np.int32).reshape(S, -1, 2)
        self.wavelet = wavelet
        self.c = fwi_geom(S, self.rec.shape[1],
                          self.src.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                          self.rec.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                          _ptr(wavelet) or 0)

    @property
    def nshots(self):
        return self.src.shape[0]

    @property
    def nrec(self):
        return self.rec.shape[1]


def _ptr(x):
    """Device address of a tensor / int / None (NULL)."""
    if x is None:
        return None
    if isinstance(x, int):
        return x
    return x.data_ptr()


def _stream(stream):
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


def _nbytes(ws):
    if ws is None:
        return 0
    if isinstance(ws, int):
        raise TypeError("pass the workspace as a tensor, or as (address, nbytes)")
    if isinstance(ws, tuple):
        return ws[1]
    return ws.numel() * ws.element_size()


def _wsptr(ws):
    if isinstance(ws, tuple):
        return ws[0]
    return _ptr(ws)


def _check(status, where):
    if status != FWI_OK:
        raise FwiError(status, where)


# ---------------------------------------------------------------------------
def workspace_bytes(grid: fwi_grid, geom: Geometry, save_mode: int) -> int:
    out = ctypes.c_size_t(0)
    _check(lib().fwi_workspace_bytes(ctypes.byref(grid), ctypes.byref(geom.c),
                                     int(save_mode), ctypes.byref(out)),
           "fwi_workspace_bytes")
    return int(out.value)


def checkpoint_interval(grid: fwi_grid, geom: Geometry) -> int:
    out = ctypes.c_int32(0)
    _check(lib().fwi_checkpoint_interval(ctypes.byref(grid), ctypes.byref(geom.c),
                                         ctypes.byref(out)), "fwi_checkpoint_interval")
    return int(out.value)


def fdtd_forward(grid, geom, eps_r, sigma, traces, save_mode, ws, stream=None,
                 raise_on_error=True) -> int:
    st = lib().fdtd_forward(ctypes.byref(grid), ctypes.byref(geom.c), _ptr(eps_r),
                            _ptr(sigma), _ptr(traces), int(save_mode), _wsptr(ws),
                            _nbytes(ws), _stream(stream))
    if raise_on_error:
        _check(st, "fdtd_forward")
    return st


def fdtd_adjoint(grid, geom, eps_r, sigma, residual, grad_eps_r, grad_sigma,
                 src_adjoint, save_mode, ws, stream=None, raise_on_error=True) -> int:
    st = lib().fdtd_adjoint(ctypes.byref(grid), ctypes.byref(geom.c), _ptr(eps_r),
                            _ptr(sigma), _ptr(residual), _ptr(grad_eps_r),
                            _ptr(grad_sigma), _ptr(src_adjoint), int(save_mode),
                            _wsptr(ws), _nbytes(ws), _stream(stream))
    if raise_on_error:
        _check(st, "fdtd_adjoint")
    return st


def fwi_gradient(grid, geom, eps_r, sigma, observed, misfit, grad_eps_r, grad_sigma,
                 traces_out, ws, stream=None, raise_on_error=True) -> int:
    st = lib().fwi_gradient(ctypes.byref(grid), ctypes.byref(geom.c), _ptr(eps_r),
                            _ptr(sigma), _ptr(observed), _ptr(misfit),
                            _ptr(grad_eps_r), _ptr(grad_sigma), _ptr(traces_out),
                            _wsptr(ws), _nbytes(ws), _stream(stream))
    if raise_on_error:
        _check(st, "fwi_gradient")
    return st


def fwi_gradient_timed(grid, geom, eps_r, sigma, observed, misfit, grad_eps_r, grad_sigma,
                       traces_out, ws, timing: fwi_timing, stream=None,
                       raise_on_error=True) -> int:
    st = lib().fwi_gradient_timed(ctypes.byref(grid), ctypes.byref(geom.c), _ptr(eps_r),
                                  _ptr(sigma), _ptr(observed), _ptr(misfit),
                                  _ptr(grad_eps_r), _ptr(grad_sigma), _ptr(traces_out),
                                  _wsptr(ws), _nbytes(ws), _stream(stream),
                                  ctypes.byref(timing) if timing is not None else None)
    if raise_on_error:
        _check(st, "fwi_gradient_timed")
    return st


def fwi_gradient_ex(grid, geom, eps_r, sigma, observed, misfit, grad_eps_r, grad_sigma,
                    traces_out, ws, timing: fwi_timing | None = None, shot_groups: int = 0,
                    stream=None, raise_on_error=True) -> int:
    """fwi_gradient(_timed) with the shots in `shot_groups` concurrent groups
    (0 = the library's choice); results identical for every group count."""
    st = lib().fwi_gradient_ex(ctypes.byref(grid), ctypes.byref(geom.c), _ptr(eps_r),
                               _ptr(sigma), _ptr(observed), _ptr(misfit),
                               _ptr(grad_eps_r), _ptr(grad_sigma), _ptr(traces_out),
                               _wsptr(ws), _nbytes(ws), _stream(stream),
                               ctypes.byref(timing) if timing is not None else None,
                               int(shot_groups))
    if raise_on_error:
        _check(st, "fwi_gradient_ex")
    return st


def fwi_gradient_static(grid, geom, eps_r, sigma, observed, misfit, grad_eps_r, grad_sigma,
                        traces_out, stream=None, raise_on_error=True) -> int:
    """fwi_gradient with the library's static device scratch as workspace
    (no allocation; problems up to STATIC_SCRATCH_BYTES of workspace)."""
    st = lib().fwi_gradient_static(ctypes.byref(grid), ctypes.byref(geom.c), _ptr(eps_r),
                                   _ptr(sigma), _ptr(observed), _ptr(misfit),
                                   _ptr(grad_eps_r), _ptr(grad_sigma), _ptr(traces_out),
                                   _stream(stream))
    if raise_on_error:
        _check(st, "fwi_gradient_static")
    return st


def alloc_workspace(nbytes: int, device="cuda"):
    """A 256-byte aligned device byte buffer from torch's allocator."""
    import torch
    t = torch.empty(max(int(nbytes), 1) + 256, dtype=torch.uint8, device=device)
    off = (-t.data_ptr()) % 256
    v = t[off:off + int(nbytes)]
    assert v.data_ptr() % 256 == 0
    return v


# ---- batched gradients of independent problems -------------------------------
class BatchProblem:
    """One problem of a batch: grid, Geometry, and device arrays (kept alive
    here).  eps_r, sigma [NY][NX]; observed [S][nt][R]; misfit a float64
    device scalar; grad_eps_r, grad_sigma [NY][NX]."""

    def __init__(self, grid, geom, eps_r, sigma, observed, misfit, grad_eps_r, grad_sigma):
        self.grid, self.geom = grid, geom
        self.arrays = (eps_r, sigma, observed, misfit, grad_eps_r, grad_sigma)
        self.c = fwi_batch_problem(grid, geom.c, _ptr(eps_r), _ptr(sigma), _ptr(observed),
                                   _ptr(misfit), _ptr(grad_eps_r), _ptr(grad_sigma))


def _batch_array(problems):
    arr = (fwi_batch_problem * len(problems))()
    for k, p in enumerate(problems):
        arr[k] = p.c
    return arr


def batch_workspace_bytes(problems) -> int:
    out = ctypes.c_size_t()
    _check(lib().fwi_batch_workspace_bytes(len(problems), _batch_array(problems),
                                           ctypes.byref(out)), "fwi_batch_workspace_bytes")
    return out.value


class BatchPlan:
    """A plan over `problems` (a list of BatchProblem) in workspace `ws`.
    run() evaluates every problem's misfit and gradient (asynchronous on the
    stream); close() releases the plan."""

    def __init__(self, problems, ws, autotune=True, stream=None):
        """autotune: True (time temporal depths and band heights), False
        (depth 4, default bands) or FWI_TUNE_* / FWI_BATCH_DEPTH8 flags."""
        if autotune is True:
            flags = FWI_TUNE_BANDS | FWI_TUNE_DEPTH
        elif autotune is False or autotune is None:
            flags = 0
        else:
            flags = int(autotune)
        self.problems = list(problems)
        self.ws = ws
        self._arr = _batch_array(self.problems)
        h = ctypes.c_void_p()
        _check(lib().fwi_batch_plan_create(len(self.problems), self._arr, _wsptr(ws),
                                           _nbytes(ws), flags, _stream(stream),
                                           ctypes.byref(h)), "fwi_batch_plan_create")
        self._h = h

    def run(self, use_graph=True, stream=None):
        if not self._h:
            raise RuntimeError("plan is closed")
        _check(lib().fwi_batch_plan_run(self._h, int(bool(use_graph)), _stream(stream)),
               "fwi_batch_plan_run")

    def info(self) -> dict:
        i = fwi_batch_info()
        _check(lib().fwi_batch_plan_info(self._h, ctypes.byref(i)), "fwi_batch_plan_info")
        return i.as_dict()

    def close(self):
        if self._h:
            lib().fwi_batch_plan_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
