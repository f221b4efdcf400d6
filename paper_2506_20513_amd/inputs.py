"""Seeded synthetic inputs: run configurations, models, acquisition
geometry and source wavelets.

This module holds none of the method's arithmetic (no field update, no
coefficient, no CPML profile, no adjoint).  It is shared by the tests, the
benchmark and the CPU oracle's callers so that both sides see identical
inputs.

The paper's own models exist only as figures and its field data is not
available, so the generators below produce seeded stand-ins with the shapes
and value ranges of the paper's experiments (Sec. 4) and of the workloads
this library is measured on.

Conventions: total grid [NY][NX] = interior [ny][nx] padded by npml cells on
every side by edge replication; x (index i) is horizontal and contiguous, y
(index j) is depth.  Geometry is given as (i, j) cell indices on the total
grid.  The wavelet is sampled at t = (n + 1/2) dt, the time at which the
E update that consumes it is centred.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, replace

import numpy as np

C0 = 299792458.0
MU0 = 4.0e-7 * math.pi
EPS0 = 1.0 / (MU0 * C0 * C0)


@dataclass(frozen=True)
class RunConfig:
    name: str
    nx: int
    ny: int
    npml: int
    nt: int
    dx: float
    dy: float
    f0: float              # Ricker centre frequency (Hz)
    nshots: int
    nrec: int
    cfl_fraction: float = 0.9
    cpml_order: int = 3
    cpml_sigma_scale: float = 1.0
    cpml_kappa_max: float = 1.0
    dt_override: float | None = None

    @property
    def NX(self) -> int:
        return self.nx + 2 * self.npml

    @property
    def NY(self) -> int:
        return self.ny + 2 * self.npml

    @property
    def dt(self) -> float:
        """A fraction of the vacuum stability bound (Eq. (11) with c = c0)."""
        if self.dt_override is not None:
            return self.dt_override
        return self.cfl_fraction / (C0 * math.sqrt(1.0 / self.dx ** 2 + 1.0 / self.dy ** 2))

    @property
    def cpml_alpha_max(self) -> float:
        return math.pi * self.f0 * EPS0

    def grid_kwargs(self) -> dict:
        return dict(nx=self.nx, ny=self.ny, npml=self.npml, nt=self.nt,
                    dx=self.dx, dy=self.dy, dt=self.dt,
                    cpml_order=self.cpml_order,
                    cpml_sigma_scale=self.cpml_sigma_scale,
                    cpml_kappa_max=self.cpml_kappa_max,
                    cpml_alpha_max=self.cpml_alpha_max)

    def with_(self, **kw) -> "RunConfig":
        return replace(self, **kw)


# ---------------------------------------------------------------------------
# Workload configurations
# ---------------------------------------------------------------------------
def config_tiny() -> RunConfig:
    """128x128 interior, dx = dy = 0.02 m, 800 steps, 200 MHz, 10-cell CPML,
    one source and 32 surface receivers every 4 cells."""
    return RunConfig("tiny-128x128", 128, 128, 10, 800, 0.02, 0.02, 200e6, 1, 32)


def config_survey() -> RunConfig:
    """512x256 interior, dx = 0.01 m, 3000 steps, 400 MHz, 20-cell CPML,
    24 shots x 128 receivers."""
    return RunConfig("survey-512x256", 512, 256, 20, 3000, 0.01, 0.01, 400e6, 24, 128)


def config_large() -> RunConfig:
    """2048x1024 interior, dx = 0.005 m, 6000 steps, 400 MHz (top band),
    20-cell CPML, 64 shots x 256 receivers."""
    return RunConfig("large-2048x1024", 2048, 1024, 20, 6000, 0.005, 0.005, 400e6, 64, 256)


def config_uneven(n_models: int = 96, seed: int = 5) -> list[RunConfig]:
    """Independent problems of uneven size for the batched gradient: interior
    nx uniform in [200, 640] and ny in [100, 320] cells, dx = dy = 0.01 m,
    nt uniform in [1500, 4000], 20-cell CPML, 8 shots x 64 surface
    receivers, Ricker 200 MHz; models as in the 128x128 workload (seeded per
    problem)."""
    rng = np.random.default_rng(seed)
    out = []
    for m in range(n_models):
        nx = int(rng.integers(200, 641))
        ny = int(rng.integers(100, 321))
        nt = int(rng.integers(1500, 4001))
        out.append(RunConfig(f"uneven-{m}-{nx}x{ny}", nx, ny, 20, nt, 0.01, 0.01, 200e6, 8, 64))
    return out


def config_paper_shapes() -> list[RunConfig]:
    """Grid shapes of the paper's three experiments (Tables 2-4), none a
    multiple of 64, used as odd-shape cases.  Step counts shortened."""
    return [
        RunConfig("crosshole-220x120", 220, 120, 10, 300, 0.05, 0.05, 100e6, 2, 40),
        RunConfig("overthrust-120x220", 120, 220, 10, 300, 0.02, 0.02, 400e6, 2, 1),
        RunConfig("sandpit-80x374", 80, 374, 10, 300, 0.025, 0.025, 500e6, 1, 3),
    ]


# ---------------------------------------------------------------------------
# Wavelet
# ---------------------------------------------------------------------------
def ricker(nt: int, dt: float, f0: float, amp: float = 1.0, t0: float | None = None,
           dtype=np.float32) -> np.ndarray:
    """Ricker wavelet (the paper's 'ricker' source amplitude, Tables 2-4)
    sampled at t = (n + 1/2) dt; delay t0 = sqrt(2)/f0 by default."""
    if t0 is None:
        t0 = math.sqrt(2.0) / f0
    t = (np.arange(nt, dtype=np.float64) + 0.5) * dt - t0
    a = (math.pi * f0 * t) ** 2
    return (amp * (1.0 - 2.0 * a) * np.exp(-a)).astype(dtype)


def wavelets(cfg: RunConfig, dtype=np.float32) -> np.ndarray:
    w = ricker(cfg.nt, cfg.dt, cfg.f0, dtype=dtype)
    return np.ascontiguousarray(np.broadcast_to(w, (cfg.nshots, cfg.nt)), dtype=dtype)


# ---------------------------------------------------------------------------
# Geometry
# ---------------------------------------------------------------------------
def _spread(first: int, span: int, count: int) -> np.ndarray:
    if count == 1:
        return np.array([first])
    return np.array([first + int(round(k * span / (count - 1))) for k in range(count)])


def geometry(cfg: RunConfig) -> tuple[np.ndarray, np.ndarray]:
    """Surface acquisition: sources one cell below the top of the interior,
    receivers three cells below it.  Returns int32 src [S][2], rec [S][R][2]."""
    p = cfg.npml
    S, R = cfg.nshots, cfg.nrec
    if cfg.name.startswith("tiny"):
        src_i = np.array([p + 64])
        rec_i = p + 2 + 4 * np.arange(R)
    elif cfg.name.startswith("survey"):
        src_i = p + 10 + np.array([int(round(k * 491 / 23)) for k in range(S)])
        rec_i = p + 2 + 4 * np.arange(R)
    elif cfg.name.startswith("large"):
        src_i = p + 16 + np.array([int(round(k * 2015 / 63)) for k in range(S)])
        rec_i = p + 4 + 8 * np.arange(R)
    else:
        margin = 2
        src_i = _spread(p + margin, cfg.nx - 1 - 2 * margin, S)
        rec_i = _spread(p + margin + 1, cfg.nx - 3 - 2 * margin, R)
    src = np.stack([src_i, np.full(S, p + 1)], axis=1).astype(np.int32)
    rec1 = np.stack([rec_i, np.full(R, p + 3)], axis=1).astype(np.int32)
    rec = np.ascontiguousarray(np.broadcast_to(rec1, (S, R, 2)), dtype=np.int32)
    return np.ascontiguousarray(src), rec


# ---------------------------------------------------------------------------
# Models
# ---------------------------------------------------------------------------
def pad_edge(a: np.ndarray, npml: int) -> np.ndarray:
    return np.pad(a, npml, mode="edge")


def _gauss(a: np.ndarray, sigma_cells: float) -> np.ndarray:
    from scipy.ndimage import gaussian_filter
    return gaussian_filter(a, sigma_cells, mode="nearest")


def model_tiny(cfg: RunConfig, seed: int = 1) -> tuple[np.ndarray, np.ndarray]:
    """Three horizontal layers (eps_r 4 / 9 / 16, interfaces at 1/3 and 2/3 of
    the interior depth) plus two discs (radius 6-16 cells, eps_r 1-25);
    sigma in 16x16-cell blocks, each uniform in [0, 0.02] S/m."""
    rng = np.random.default_rng(seed)
    nx, ny = cfg.nx, cfg.ny
    eps = np.empty((ny, nx))
    eps[: ny // 3] = 4.0
    eps[ny // 3: 2 * ny // 3] = 9.0
    eps[2 * ny // 3:] = 16.0
    jj, ii = np.mgrid[0:ny, 0:nx]
    for _ in range(2):
        r = rng.uniform(6, 16)
        m = r + 4
        ci = rng.uniform(m, nx - 1 - m)
        cj = rng.uniform(m, ny - 1 - m)
        eps[(ii - ci) ** 2 + (jj - cj) ** 2 <= r * r] = rng.uniform(1, 25)
    nb_y, nb_x = -(-ny // 16), -(-nx // 16)
    blocks = rng.uniform(0.0, 0.02, size=(nb_y, nb_x))
    sig = np.kron(blocks, np.ones((16, 16)))[:ny, :nx]
    return (pad_edge(eps, cfg.npml).astype(np.float32),
            pad_edge(sig, cfg.npml).astype(np.float32))


def _layered(rng, nx, ny, nlayers, lo, hi):
    x = np.arange(nx) / nx
    base = np.sort(rng.uniform(0.08, 0.95, size=nlayers - 1)) * ny
    vals = rng.uniform(lo, hi, size=nlayers)
    out = np.full((ny, nx), vals[0])
    jj = np.arange(ny)[:, None]
    for k, b in enumerate(base):
        amp = rng.uniform(0.01, 0.05) * ny
        ph = rng.uniform(0, 2 * math.pi, size=2)
        depth = b + amp * np.sin(2 * math.pi * x + ph[0]) + 0.5 * amp * np.sin(4 * math.pi * x + ph[1])
        out = np.where(jj >= depth[None, :], vals[k + 1], out)
    return out


def _inclusions(rng, nx, ny, count, sigma_g, scale):
    inc = np.zeros((ny, nx))
    jj, ii = np.mgrid[0:ny, 0:nx]
    for _ in range(count):
        r = rng.uniform(2.0, 5.0) * sigma_g
        ci = rng.uniform(0, nx)
        cj = rng.uniform(0.1 * ny, ny)
        inc[(ii - ci) ** 2 + (jj - cj) ** 2 <= r * r] += rng.uniform(-1, 1) * scale
    return _gauss(inc, sigma_g)


def model_layered(cfg: RunConfig, seed: int) -> tuple[np.ndarray, np.ndarray]:
    """6-8 layers with sinusoidally perturbed interfaces, eps_r per layer in
    [3, 20] plus 3-6 Gaussian-smoothed inclusions, clipped to [3, 20]; sigma
    from an independent layering in [0.001, 0.05] S/m, smoothed the same
    way.  Inclusion smoothing length 4 cells per 512 interior columns."""
    rng = np.random.default_rng(seed)
    nx, ny = cfg.nx, cfg.ny
    sigma_g = 4.0 * nx / 512.0
    eps = _layered(rng, nx, ny, int(rng.integers(6, 9)), 3.0, 20.0)
    eps = eps + _inclusions(rng, nx, ny, int(rng.integers(3, 7)), sigma_g, 8.0)
    eps = np.clip(eps, 3.0, 20.0)
    sig = _layered(rng, nx, ny, int(rng.integers(6, 9)), 0.001, 0.05)
    sig = _gauss(sig, sigma_g) + _inclusions(rng, nx, ny, int(rng.integers(3, 7)), sigma_g, 0.02)
    sig = np.clip(sig, 0.001, 0.05)
    return (pad_edge(eps, cfg.npml).astype(np.float32),
            pad_edge(sig, cfg.npml).astype(np.float32))


def smooth_model(eps: np.ndarray, sig: np.ndarray, npml: int, sigma_cells: float):
    """Initial model for a gradient: the true interior Gaussian-smoothed and
    re-padded by edge replication."""
    ei = eps[npml:eps.shape[0] - npml, npml:eps.shape[1] - npml].astype(np.float64)
    si = sig[npml:sig.shape[0] - npml, npml:sig.shape[1] - npml].astype(np.float64)
    return (pad_edge(_gauss(ei, sigma_cells), npml).astype(np.float32),
            pad_edge(_gauss(si, sigma_cells), npml).astype(np.float32))


def model_for(cfg: RunConfig, seed: int | None = None):
    """(true eps_r, true sigma, initial eps_r, initial sigma) for a config."""
    if cfg.name.startswith("tiny"):
        e, s = model_tiny(cfg, 1 if seed is None else seed)
        e0, s0 = smooth_model(e, s, cfg.npml, 6.0)
        return e, s, e0, s0
    if cfg.name.startswith("uneven"):
        k = int(cfg.name.split("-")[1])
        e, s = model_tiny(cfg, 1000 + k if seed is None else seed)
        e0, s0 = smooth_model(e, s, cfg.npml, 6.0)
        return e, s, e0, s0
    if cfg.name.startswith("survey"):
        seed = 2 if seed is None else seed
    elif cfg.name.startswith("large"):
        seed = 4 if seed is None else seed
    else:
        seed = 7 if seed is None else seed
    e, s = model_layered(cfg, seed)
    e0, s0 = smooth_model(e, s, cfg.npml, 10.0 * cfg.nx / 512.0)
    return e, s, e0, s0


def random_fields(shape, seed, lo=-1.0, hi=1.0, dtype=np.float32):
    return np.random.default_rng(seed).uniform(lo, hi, size=shape).astype(dtype)
