"""Learned gradient preconditioner for the dual-parameter FWI of arXiv
2506.20513 (the inversion loop of Sec. 3.1: eps_r and sigma from the trace
misfit Eq. (6) with the adjoint gradients Eqs. (12)-(13) of Sec. 2.1).

The paper has no learned component; this module adds one on top of its
inversion.

1. Plain L-BFGS FWI runs on seeded 128x128 models, and on seeded 512x256
   layered models with the survey acquisition, generate pairs.  Each pair
   maps the state at iterate k (grad_eps, grad_sigma, eps_r, sigma) to the
   update the run makes from there to its final iterate K.
2. The encoder-decoder CNN of `nn` (BF16 MFMA kernels, FP32 accumulation)
   is trained on both sets of pairs with Adam.  On a model whose cells are
   finer per wavelength than the training models', it is applied to the
   gradient pooled to the training resolution and its output upsampled.
3. Inside an inversion, the network proposes a step at every iterate.  The
   objective decrease judges the proposal: it needs a descent direction and
   at least a tenth of the decrease its slope predicts, within two trial
   lengths (the first one carried over from the previous proposal's
   quadratic fit, so an accepted proposal usually costs one evaluation).
   Otherwise the plain L-BFGS step is taken.  Both kinds of steps feed the
   same L-BFGS curvature memory.  A proposal whose first trial length fails,
   or whose decrease falls short of what the L-BFGS step's quadratic model
   predicts for itself, is a strike; after two strikes in a row the run
   continues as plain L-BFGS.

Network input at iterate k: the two gradient planes divided by the rms of
the run's first gradient (so the input shows how far the gradient has
shrunk), and the two model planes u, v.

Units: the optimiser works on the interior models normalised as in fwi_loop
(u = eps_r / eps_scale, v = sigma / sig_scale), on x = [u; v] flattened.
The rows just below the surface stay fixed, and every iterate is projected
onto eps_r >= eps_min, sigma >= sig_min.

    python -m paper_2506_20513_amd.precond --runs 667 --survey-runs 96 --epochs 30 --survey --large
"""
from __future__ import annotations

import argparse
import json
import math
import sys
import time
from dataclasses import dataclass, field

import numpy as np
import torch

from . import autograd as AG
from . import fwi_loop as FL
from . import nn


# ---------------------------------------------------------------------------
# Objective on normalised interior models
# ---------------------------------------------------------------------------
class Objective:
    """f(x) = J(m(x)) / J0 + tv_weight (TV(u) + TV(v)) and its gradient.

    J is the trace misfit of Eq. (6) and J0 its value at the initial model.
    x is flat [u; v] over the interior (ny * nx each).  The gradient is zero
    on the fixed surface rows."""

    def __init__(self, prob: AG.Problem, observed: torch.Tensor, eps0: torch.Tensor,
                 sig0: torch.Tensor, st: FL.Settings):
        self.prob, self.obs, self.st = prob, observed.contiguous(), st
        self.npml = prob.grid.npml
        NY, NX = prob.model_shape
        self.ny, self.nx = NY - 2 * self.npml, NX - 2 * self.npml
        sl = (slice(self.npml, NY - self.npml), slice(self.npml, NX - self.npml))
        self.x0 = torch.cat([(eps0[sl] / st.eps_scale).reshape(-1),
                             (sig0[sl] / st.sig_scale).reshape(-1)]).contiguous()
        self.free = torch.ones(self.ny, self.nx, dtype=torch.bool, device=eps0.device)
        self.free[: st.mask_rows] = False
        self.free = torch.cat([self.free.reshape(-1), self.free.reshape(-1)])
        n = self.ny * self.nx
        self.lo = torch.cat([torch.full((n,), st.eps_min / st.eps_scale, device=eps0.device),
                             torch.full((n,), st.sig_min / st.sig_scale, device=eps0.device)])
        self.J0 = None
        self.evals = 0
        self.last_J = None

    def project(self, x):
        x = torch.where(self.free, x, self.x0)
        return torch.maximum(x, self.lo)

    def planes(self, x):
        n = self.ny * self.nx
        return x[:n].view(self.ny, self.nx), x[n:].view(self.ny, self.nx)

    def models(self, x):
        u, v = self.planes(x)
        return (FL.pad_interior(u * self.st.eps_scale, self.npml).contiguous(),
                FL.pad_interior(v * self.st.sig_scale, self.npml).contiguous())

    def __call__(self, x):
        xx = x.detach().clone().requires_grad_(True)
        e, s = self.models(xx)
        J = AG.misfit(self.prob, e, s, self.obs)
        if self.J0 is None:
            self.J0 = float(J.detach())
        u, v = self.planes(xx)
        loss = J / self.J0 + self.st.tv_weight * (FL.total_variation(u) + FL.total_variation(v))
        loss.backward()
        self.evals += 1
        self.last_J = float(J.detach())
        g = torch.where(self.free, xx.grad, torch.zeros_like(xx.grad))
        return float(loss.detach()), g


# ---------------------------------------------------------------------------
# L-BFGS (two-loop recursion, Nocedal and Wright Alg. 7.4) with a projected
# Armijo backtracking line search
# ---------------------------------------------------------------------------
class LBFGS:
    def __init__(self, history: int = 10):
        self.history = history
        self.S, self.Y = [], []

    def reset(self):
        self.S, self.Y = [], []

    def update(self, s, y):
        """Store the pair if its curvature s.y is positive (keeps H positive
        definite without a Wolfe curvature condition)."""
        sy = float(torch.dot(s, y))
        if sy > 1e-12 * float(torch.dot(y, y)) and sy > 0:
            self.S.append(s)
            self.Y.append(y)
            if len(self.S) > self.history:
                self.S.pop(0)
                self.Y.pop(0)

    def direction(self, g):
        """-H g with the limited-memory inverse Hessian H (initial scaling
        s.y / y.y of the newest pair); None without stored pairs."""
        if not self.S:
            return None
        q = g.clone()
        alpha = []
        for s, y in zip(reversed(self.S), reversed(self.Y)):
            a = float(torch.dot(s, q)) / float(torch.dot(y, s))
            q -= a * y
            alpha.append(a)
        s, y = self.S[-1], self.Y[-1]
        r = q * (float(torch.dot(s, y)) / float(torch.dot(y, y)))
        for (s, y), a in zip(zip(self.S, self.Y), reversed(alpha)):
            b = float(torch.dot(y, r)) / float(torch.dot(y, s))
            r += (a - b) * s
        return -r


def line_search(obj, x, f, g, d, t0=1.0, trials=8, c1=1e-4, shrink=0.25):
    """Projected backtracking: accept t if f(P(x + t d)) <= f + c1 g.(P(x + t d) - x).
    Returns (x_new, f_new, g_new, t) or None."""
    t = t0
    for _ in range(trials):
        xn = obj.project(x + t * d)
        step = xn - x
        dec = float(torch.dot(g, step))
        if dec >= 0:          # the projection removed every descent component
            return None
        fn, gn = obj(xn)
        if fn <= f + c1 * dec:
            return xn, fn, gn, t
        t *= shrink
    return None


def proposal_search(obj, x, f, g, d, t0=1.0, c1=0.1):
    """At most two trial lengths along a proposed direction d.  The first is
    t0; a length is accepted if it achieves at least the fraction c1 of the
    decrease the slope g.d predicts (stricter than the Armijo test of the
    L-BFGS steps).  If t0 fails, the second trial is the minimiser of the
    quadratic through f(x), the slope and the first trial (within [0.05 t0,
    0.5 t0]).  Returns (result or None, suggested t0 for the next proposal):
    the quadratic's minimiser from the last trial, within [0.1, 4]."""
    # cleared before any early return, so that a rejected proposal never
    # reads as passed from an earlier call
    obj.first_trial_passed = False
    gd = float(torch.dot(g, d))
    if gd >= 0:
        return None, t0
    t = t0
    for trial in range(2):
        xn = obj.project(x + t * d)
        dec = float(torch.dot(g, xn - x))
        if dec >= 0:
            return None, t0
        fn, gn = obj(xn)
        curv = (fn - f - t * gd) / (t * t)     # f(x + s d) ~ f + s gd + s^2 curv
        ts = -gd / (2.0 * curv) if curv > 0 else 2.0 * t
        nxt = min(4.0, max(0.1, ts))
        if fn <= f + c1 * dec:
            obj.first_trial_passed = trial == 0
            return (xn, fn, gn, t), nxt
        t = min(0.5 * t, max(0.05 * t, ts))
    return None, nxt


@dataclass
class Iterate:
    k: int
    f: float
    J: float
    evals: int
    seconds: float
    source: str          # "start", "lbfgs", "steepest" or "net"


@dataclass
class Run:
    xs: list = field(default_factory=list)      # iterates (flat, on the GPU)
    gs: list = field(default_factory=list)      # gradients at the iterates
    log: list = field(default_factory=list)     # Iterate records
    seconds: float = 0.0

    @property
    def final_f(self):
        return self.log[-1].f


def minimise(obj: Objective, iters: int, history: int = 10, first_step: float = 0.05,
             proposer=None, target_f: float | None = None, keep: bool = False,
             max_strikes: int = 2, log=None) -> Run:
    """L-BFGS on obj from obj.x0 for `iters` iterations (or until f <=
    target_f).  proposer(x, g) -> direction or None is tried first at every
    iterate (proposal_search: at most two evaluations, starting from the
    length the previous proposal's quadratic fit suggested); the decrease it
    achieves decides, otherwise the L-BFGS step is taken.  A proposal is a
    strike when its first trial length does not pass (even if the second
    one does), or when it decreases the objective by less than the L-BFGS
    step's own quadratic model predicts (-g.d_L / 2, once L-BFGS holds
    curvature pairs); after max_strikes strikes in a row the proposer is no
    longer asked and the run continues as plain L-BFGS.  keep: retain
    iterates and gradients (for training pairs)."""
    torch.cuda.synchronize() if obj.x0.is_cuda else None
    t0 = time.perf_counter()
    mem = LBFGS(history)
    x = obj.project(obj.x0)
    f, g = obj(x)
    run = Run()

    def note(k, src):
        if obj.x0.is_cuda:
            torch.cuda.synchronize()
        run.log.append(Iterate(k, f, obj.last_J, obj.evals, time.perf_counter() - t0, src))
        if log:
            it = run.log[-1]
            log(f"  iterate {it.k}: f {it.f:.6g}, {it.evals} evaluations, {it.seconds:.2f} s, {src}")
        if keep:
            run.xs.append(x.clone())
            run.gs.append(g.clone())

    note(0, "start")
    strikes = 0
    t_net = 1.0
    for k in range(1, iters + 1):
        if target_f is not None and f <= target_f:
            break
        res, src = None, None
        if proposer is not None and strikes < max_strikes:
            d = proposer(x, g)
            passed = False
            if d is not None:
                res, t_net = proposal_search(obj, x, f, g, d, t0=t_net)
                passed = res is not None and getattr(obj, "first_trial_passed", False)
                dl = mem.direction(g)
                if res is not None and passed and dl is not None:
                    # the L-BFGS step's own quadratic model predicts a decrease
                    # of -g.d/2; a proposal that does worse is kept (it is paid
                    # for) but does not earn another try
                    passed = f - res[1] >= -0.5 * float(torch.dot(g, dl))
            src = "net"
            # a proposal that needed its second trial length, failed, or fell
            # short of the L-BFGS prediction is a strike
            strikes = 0 if passed else strikes + 1
        if res is None:
            d = mem.direction(g)
            src = "lbfgs"
            if d is None or float(torch.dot(g, d)) >= 0:
                mem.reset()
                gmax = float(g.abs().max())
                if gmax == 0:
                    break
                d = -g * (first_step / gmax)
                src = "steepest"
            res = line_search(obj, x, f, g, d, t0=1.0)
            if res is None and src == "lbfgs":
                mem.reset()
                d = -g * (first_step / float(g.abs().max()))
                src = "steepest"
                res = line_search(obj, x, f, g, d, t0=1.0)
            if res is None:
                break
        xn, fn, gn, _ = res
        mem.update(xn - x, gn - g)
        x, f, g = xn, fn, gn
        note(k, src)
    run.seconds = run.log[-1].seconds
    run.x = x
    return run


# ---------------------------------------------------------------------------
# Features and targets
# ---------------------------------------------------------------------------
def gradient_scales(obj: Objective, g0):
    """1 / rms of the eps_r and sigma parts of the run's first gradient."""
    n = obj.ny * obj.nx
    out = []
    for part in (g0[:n], g0[n:]):
        r = float(torch.sqrt(torch.mean(part.double() ** 2)))
        out.append(1.0 / r if r > 0 else 0.0)
    return out


def feature_planes(obj: Objective, x, g, gscale):
    """[4][ny][nx] float32 (g_u, g_v, u, v) and their scales [4] (gscale
    for the gradient planes, 1 for the models)."""
    n = obj.ny * obj.nx
    planes = torch.stack([g[:n], g[n:], x[:n], x[n:]]).view(4, obj.ny, obj.nx).float()
    sc = torch.tensor([gscale[0], gscale[1], 1.0, 1.0], dtype=torch.float32, device=x.device)
    return planes.contiguous(), sc


# The grid spacing and centre frequency of the training models: the network
# has learnt features of a given size in wavelengths per cell.
TRAIN_DX = 0.02
TRAIN_F0 = 200e6


def wavelength_factor(dx: float, f0: float) -> int:
    """Power-of-two resampling factor that brings a model sampled at dx with
    a source of centre frequency f0 to the training models' cells per
    wavelength (the wavelength in cells scales as 1 / (f0 dx))."""
    r = (TRAIN_F0 * TRAIN_DX) / (f0 * dx)
    f = 1
    while f * 2 <= r * 1.4142135623730951:
        f *= 2
    return f


class Preconditioner:
    """The trained network applied to one iterate: x, g -> proposed step
    (flat like x, zero on the fixed rows).

    factor > 1 applies the network at the training models' cells per
    wavelength: the packed input is average-pooled `factor` times smaller
    (pooling kernel), the network runs on it, and its output is brought
    back by nearest upsampling (upsampling kernel)."""

    def __init__(self, net: nn.Net, factor: int = 1):
        if factor < 1 or factor & (factor - 1):
            raise ValueError("factor must be a power of two")
        self.net = net
        self.factor = factor
        self.calls = 0
        self.seconds = 0.0
        self.gscale = None

    def __call__(self, obj: Objective, x, g):
        """The first call of a run must be at its starting iterate: its
        gradient sets the normalisation of the gradient planes."""
        t = time.perf_counter()
        if self.gscale is None:
            self.gscale = gradient_scales(obj, g)
        planes, sc = feature_planes(obj, x, g, self.gscale)
        H, W = obj.ny, obj.nx
        if H % (8 * self.factor) or W % (8 * self.factor):
            raise ValueError(f"interior {H}x{W} is not a multiple of {8 * self.factor}")
        xin = torch.empty(H * W * nn.CPAD, dtype=torch.bfloat16, device=x.device)
        nn.pack4(planes, sc, xin, 1, H, W)
        h, w = H, W
        while h > H // self.factor:
            xd = torch.empty((h // 2) * (w // 2) * nn.CPAD, dtype=torch.bfloat16, device=x.device)
            nn.pool2(xin, xd, 1, h, w, nn.CPAD)
            xin, h, w = xd, h // 2, w // 2
        y = self.net.forward(xin, 1, h, w)
        while h < H:
            yu = torch.empty((2 * h) * (2 * w) * nn.CPAD, dtype=torch.bfloat16, device=x.device)
            nn.up2_add(y, None, yu, 1, 2 * h, 2 * w, nn.CPAD)
            y, h, w = yu, 2 * h, 2 * w
        out = torch.empty(2 * H * W, dtype=torch.float32, device=x.device)
        nn.unpack2(y, torch.ones(2, device=x.device), out, 1, H, W, nn.CPAD)
        d = torch.where(obj.free, out.to(x.dtype), torch.zeros_like(x))
        self.calls += 1
        self.seconds += time.perf_counter() - t
        return d


# ---------------------------------------------------------------------------
# Dataset from plain runs
# ---------------------------------------------------------------------------
@dataclass
class Dataset:
    planes: torch.Tensor     # [M][4][H][W] float32
    scales: torch.Tensor     # [M][4] float32
    targets: torch.Tensor    # [M][H][W][2] float32 (normalised units)

    def __len__(self):
        return self.planes.shape[0]


def tiny_problem(seed: int, smoothing: float, device="cuda"):
    """A seeded 128x128 problem (the small survey-shaped configuration): true
    model, smoothed start, observed traces, and the autograd problem."""
    from . import fwi
    from . import inputs as I
    cfg = I.config_tiny()
    e, s = I.model_tiny(cfg, seed)
    e0, s0 = I.smooth_model(e, s, cfg.npml, smoothing)
    src, rec = I.geometry(cfg)
    w = torch.from_numpy(I.wavelets(cfg).copy()).to(device)
    prob = AG.Problem(fwi.grid_from_config(cfg), src, rec, w, device=device)
    T = lambda a: torch.from_numpy(a).to(device)
    with torch.no_grad():
        obs = AG.traces(prob, T(e), T(s))
    return cfg, prob, obs, T(e), T(s), T(e0), T(s0)


def survey_problem(seed: int, smoothing: float, device="cuda"):
    """A seeded 512x256 layered model with the survey acquisition (24 shots x
    128 receivers, 400 MHz, dx = 0.01 m): true model, start smoothed with a
    Gaussian of `smoothing` cells, observed traces, and the autograd
    problem."""
    from . import fwi
    from . import inputs as I
    cfg = I.config_survey()
    e, s = I.model_layered(cfg, seed)
    e0, s0 = I.smooth_model(e, s, cfg.npml, smoothing)
    src, rec = I.geometry(cfg)
    w = torch.from_numpy(I.wavelets(cfg).copy()).to(device)
    prob = AG.Problem(fwi.grid_from_config(cfg), src, rec, w, device=device)
    T = lambda a: torch.from_numpy(a).to(device)
    with torch.no_grad():
        obs = AG.traces(prob, T(e), T(s))
    return cfg, prob, obs, T(e), T(s), T(e0), T(s0)


def _one_run(r: int, seed0: int, iters: int, st: FL.Settings, smoothing: float, device,
             kind: str = "tiny"):
    """Pairs of plain run r: features at every iterate but the last, and the
    update from there to the last iterate."""
    if kind == "tiny":
        cfg, prob, obs, e, s, e0, s0 = tiny_problem(seed0 + r, smoothing, device)
    else:
        cfg, prob, obs, e, s, e0, s0 = survey_problem(seed0 + r, 2.0 * smoothing, device)
    obj = Objective(prob, obs, e0, s0, st)
    run = minimise(obj, iters, keep=True)
    xK = run.xs[-1]
    n = obj.ny * obj.nx
    gsc = gradient_scales(obj, run.gs[0])
    planes, scales, targets = [], [], []
    for xk, gk in zip(run.xs[:-1], run.gs[:-1]):
        p, sc = feature_planes(obj, xk, gk, gsc)
        planes.append(p)
        scales.append(sc)
        dx = (xK - xk).float()
        targets.append(torch.stack([dx[:n], dx[n:]], dim=-1).view(obj.ny, obj.nx, 2))
    return planes, scales, targets, obj.evals, run.log[-1].J / obj.J0


def generate(nruns: int, iters: int, seed0: int, st: FL.Settings, log=print,
             device="cuda", workers: int = 1, kind: str = "tiny") -> tuple[Dataset, dict]:
    """Pairs from nruns plain L-BFGS runs on seeded 128x128 models (seeds
    seed0 .. seed0 + nruns - 1, start models smoothed with a Gaussian of
    4 to 10 cells).  Pair k of a run: features at iterate k, target x_K - x_k
    with K the run's last iterate.

    workers > 1 runs that many runs at a time, each host thread on its own
    stream (default priority): a 128x128 gradient leaves the GPU mostly idle
    between its launches.  Runs are independent and deterministic, and the
    pairs are gathered in run order, so the dataset does not depend on
    `workers`.  kind = "survey" takes seeded 512x256 layered models with the
    survey acquisition instead, starts smoothed over 8 to 20 cells (the
    survey workload's start is smoothed over 10 cells; the 2048x1024 model's
    over 40, i.e. 20 once resampled by 2 to the survey's cell size)."""
    from . import fwi
    fwi.lib()
    nn.lib()
    rng = np.random.default_rng(seed0)
    smooth = [float(rng.uniform(4.0, 10.0)) for _ in range(nruns)]
    results = [None] * nruns
    t0 = time.perf_counter()
    done = [0]

    def note():
        done[0] += 1
        if log and done[0] % max(1, nruns // 10) == 0:
            log(f"generate: {done[0]}/{nruns} runs, {time.perf_counter() - t0:.1f} s")

    if workers <= 1:
        for r in range(nruns):
            results[r] = _one_run(r, seed0, iters, st, smooth[r], device, kind)
            note()
    else:
        import threading
        lock = threading.Lock()
        errors = []

        def worker(w):
            stream = torch.cuda.Stream(device=device)
            try:
                with torch.cuda.stream(stream):
                    for r in range(w, nruns, workers):
                        out = _one_run(r, seed0, iters, st, smooth[r], device, kind)
                        stream.synchronize()
                        results[r] = out
                        with lock:
                            note()
            except Exception as ex:       # reported after the join
                errors.append(ex)

        threads = [threading.Thread(target=worker, args=(w,)) for w in range(workers)]
        for th in threads:
            th.start()
        for th in threads:
            th.join()
        if errors:
            raise errors[0]
        torch.cuda.synchronize()
    planes, scales, targets = [], [], []
    evals, final = 0, []
    for p, sc, tg, ne, fr in results:
        planes += p
        scales += sc
        targets += tg
        evals += ne
        final.append(fr)
    stats = {"runs": nruns, "evaluations": evals, "seconds": time.perf_counter() - t0,
             "final_rel_misfit": float(np.mean(final)), "workers": workers}
    return Dataset(torch.stack(planes), torch.stack(scales), torch.stack(targets)), stats


def _batch_loss(net: nn.Net, ds: Dataset, idx, xin, dy):
    b = idx.numel()
    H, W = ds.planes.shape[2], ds.planes.shape[3]
    nn.pack4(ds.planes[idx].contiguous(), ds.scales[idx].contiguous(), xin, b, H, W)
    y = net.forward(xin, b, H, W)
    return net.loss_and_grad(y, ds.targets[idx].contiguous(), dy, b, H, W)


def mean_loss(net: nn.Net, ds: Dataset, ids, batch: int = 32) -> float:
    """Mean squared error of the network over the pairs `ids`."""
    H, W = ds.planes.shape[2], ds.planes.shape[3]
    xin = torch.empty(batch * H * W * nn.CPAD, dtype=torch.bfloat16, device=ds.planes.device)
    tot = 0.0
    for i in range(0, ids.numel(), batch):
        idx = ids[i:i + batch]
        tot += float(_batch_loss(net, ds, idx, xin, None)) * idx.numel()
    return tot / max(ids.numel(), 1)


def train(ds, epochs: int, batch: int = 32, lr: float = 1e-3, seed: int = 0,
          val_frac: float = 0.05, warmup: int = 100, log=print, device="cuda") -> tuple[nn.Net, dict]:
    """Adam on the mean squared error between network output and target:
    linear warm-up over `warmup` steps, then cosine decay to zero.  A
    fraction val_frac of the pairs is held out for validation.

    ds: one Dataset or a list of them (images of different sizes).  Each
    dataset is cut into batches of about `batch` x 128 x 128 pixels, and
    every epoch visits all batches of all datasets in a seeded random
    order."""
    sets = ds if isinstance(ds, (list, tuple)) else [ds]
    g = torch.Generator().manual_seed(seed)
    net = nn.Net(seed=seed, device=device)
    parts = []
    for d in sets:
        M = len(d)
        perm = torch.randperm(M, generator=g)
        nval = int(M * val_frac)
        H, W = d.planes.shape[2], d.planes.shape[3]
        b = max(1, round(batch * 128 * 128 / (H * W)))
        parts.append({"ds": d, "val": perm[:nval].to(device), "tr": perm[nval:].to(device),
                      "batch": b, "H": H, "W": W,
                      "xin": torch.empty(b * H * W * nn.CPAD, dtype=torch.bfloat16, device=device),
                      "dy": torch.empty(b * H * W * nn.CPAD, dtype=torch.bfloat16, device=device)})
    hist = {"epochs": [], "zero_predictor_val": None,
            "train_ids": parts[0]["tr"], "val_ids": parts[0]["val"]}
    nval_all = sum(p["val"].numel() for p in parts)
    if nval_all:
        hist["zero_predictor_val"] = float(sum(float((p["ds"].targets[p["val"]].double() ** 2).sum())
                                               for p in parts if p["val"].numel())
                                           / sum(p["val"].numel() * p["H"] * p["W"] * 2
                                                 for p in parts))
    t0 = time.perf_counter()
    steps = 0
    per_epoch = sum(p["tr"].numel() // p["batch"] for p in parts)
    total = max(1, epochs * per_epoch)
    warmup = min(warmup, max(1, total // 10))
    for ep in range(epochs):
        plan = []
        for k, p in enumerate(parts):
            order = p["tr"][torch.randperm(p["tr"].numel(), generator=g).to(device)]
            nb = p["tr"].numel() // p["batch"]
            plan += [(k, order[i * p["batch"]:(i + 1) * p["batch"]]) for i in range(nb)]
        shuffle = torch.randperm(len(plan), generator=g).tolist()
        losses = torch.zeros(max(len(plan), 1), dtype=torch.float64, device=device)
        for i, j in enumerate(shuffle):
            k, idx = plan[j]
            p = parts[k]
            losses[i] = _batch_loss(net, p["ds"], idx, p["xin"], p["dy"])[0]
            net.backward(p["dy"])
            f = min(1.0, (steps + 1) / warmup) * 0.5 * (1.0 + math.cos(math.pi * steps / total))
            net.adam_step(lr * f)
            steps += 1
        vl = float("nan")
        if nval_all:
            vl = sum(mean_loss(net, p["ds"], p["val"], p["batch"]) * p["val"].numel()
                     for p in parts if p["val"].numel()) / nval_all
        torch.cuda.synchronize()
        rec = {"epoch": ep + 1, "train_loss": float(losses.mean()), "val_loss": vl,
               "seconds": time.perf_counter() - t0}
        hist["epochs"].append(rec)
        if log:
            log(f"train: {rec}")
    hist["steps"] = steps
    hist["seconds"] = time.perf_counter() - t0
    return net, hist


def minimise_wolfe(obj: Objective, iters: int, history: int = 10, log=None) -> Run:
    """The inversion driver's plain method on the same objective: torch's
    L-BFGS with a strong-Wolfe line search (as fwi_loop.invert runs it),
    `iters` iterations, on the projected point (surface rows fixed, bounds
    clamped).  The final objective is evaluated once more at the projected
    last iterate, outside the timed region."""
    sync = (lambda: torch.cuda.synchronize()) if obj.x0.is_cuda else (lambda: None)
    sync()
    t0 = time.perf_counter()
    x = obj.project(obj.x0).clone().requires_grad_(True)
    opt = torch.optim.LBFGS([x], lr=1.0, max_iter=iters, history_size=history,
                            line_search_fn="strong_wolfe", tolerance_grad=1e-12,
                            tolerance_change=1e-12)
    run = Run()

    def closure():
        opt.zero_grad()
        f, g = obj(obj.project(x.detach()))
        x.grad = g.clone()
        if log:
            log(f"  wolfe evaluation {obj.evals}: f {f:.6g}, {time.perf_counter() - t0:.2f} s")
        return torch.tensor(f, dtype=x.dtype, device=x.device)

    opt.step(closure)
    sync()
    seconds = time.perf_counter() - t0
    evals = obj.evals
    xf = obj.project(x.detach())
    f, _ = obj(xf)
    obj.evals = evals
    run.log.append(Iterate(iters, f, obj.last_J, evals, seconds, "lbfgs-wolfe"))
    run.seconds = seconds
    run.x = xf
    return run


def compare(net: nn.Net, problems, iters: int, st: FL.Settings, log=print,
            verbose: bool = False, plain_method: str = "armijo") -> list:
    """Plain L-BFGS for `iters` iterations, then the learned variant until it
    reaches the plain run's final objective (at most 2 iters iterations).
    plain_method: "armijo" (this module's projected L-BFGS, the learned
    run's own fallback) or "wolfe" (the inversion driver's strong-Wolfe
    L-BFGS).  Returns one record per problem with both wall-clock times.
    verbose: log every iterate."""
    out = []
    for item in problems:
        name, prob, obs, e0, s0 = item[:5]
        factor = item[5] if len(item) > 5 else 1
        obj = Objective(prob, obs, e0, s0, st)
        if verbose and log:
            log(f"{name}: plain L-BFGS ({plain_method})")
        if plain_method == "wolfe":
            plain = minimise_wolfe(obj, iters, log=log if verbose else None)
        else:
            plain = minimise(obj, iters, log=log if verbose else None)
        target = plain.final_f
        objn = Objective(prob, obs, e0, s0, st)
        pc = Preconditioner(net, factor)
        if verbose and log:
            log(f"{name}: learned, until f <= {target:.6g}")
        learned = minimise(objn, 2 * iters, proposer=lambda x, g: pc(objn, x, g),
                           target_f=target, log=log if verbose else None)
        reached = learned.final_f <= target
        rec = {"problem": name, "plain_method": plain_method,
               "plain_seconds": round(plain.seconds, 3),
               "plain_evaluations": obj.evals, "plain_final_f": target,
               "plain_final_rel_misfit": plain.log[-1].J / obj.J0,
               "learned_seconds": round(learned.seconds, 3),
               "learned_evaluations": objn.evals, "learned_final_f": learned.final_f,
               "learned_reached_plain_final": bool(reached),
               "learned_iterations": learned.log[-1].k,
               "net_steps_accepted": sum(1 for it in learned.log if it.source == "net"),
               "resampling_factor": factor,
               "net_seconds": round(pc.seconds, 3)}
        if log:
            log(f"compare: {rec}")
        out.append(rec)
    return out


def _survey_problem(cfg, factor=None):
    from . import fwi
    from . import inputs as I
    e, s, e0, s0 = I.model_for(cfg)
    src, rec = I.geometry(cfg)
    w = torch.from_numpy(I.wavelets(cfg).copy()).cuda()
    prob = AG.Problem(fwi.grid_from_config(cfg), src, rec, w)
    with torch.no_grad():
        obs = AG.traces(prob, torch.from_numpy(e).cuda(), torch.from_numpy(s).cuda())
    f = wavelength_factor(cfg.dx, cfg.f0) if not factor else factor
    return (cfg.name, prob, obs, torch.from_numpy(e0).cuda(), torch.from_numpy(s0).cuda(), f)


def _summary(res):
    return {"plain_seconds": round(sum(r["plain_seconds"] for r in res), 3),
            "learned_seconds": round(sum(r["learned_seconds"] for r in res), 3),
            "plain_evaluations": sum(r["plain_evaluations"] for r in res),
            "learned_evaluations": sum(r["learned_evaluations"] for r in res),
            "reached": sum(r["learned_reached_plain_final"] for r in res), "problems": len(res)}


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--runs", type=int, default=667)
    ap.add_argument("--workers", type=int, default=8,
                    help="runs generated at a time, one host thread and stream each")
    ap.add_argument("--iters", type=int, default=30)
    ap.add_argument("--epochs", type=int, default=30)
    ap.add_argument("--batch", type=int, default=32)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--eval", type=int, default=8, help="held-out 128x128 problems")
    ap.add_argument("--survey", action="store_true", help="also compare on the 512x256 survey")
    ap.add_argument("--survey-iters", type=int, default=10)
    ap.add_argument("--large", action="store_true", help="also compare on the 2048x1024 model")
    ap.add_argument("--large-iters", type=int, default=5)
    ap.add_argument("--save", default=None, help="write the trained parameters (.npy)")
    ap.add_argument("--factor", type=int, default=0,
                    help="resampling factor of the network on the survey and large models; 0 = "
                         "matched to the training models' cells per wavelength (1 on the survey, "
                         "2 on the large model)")
    ap.add_argument("--survey-runs", type=int, default=96,
                    help="also train on pairs from this many plain runs on seeded 512x256 "
                         "layered models (seeds 20000 on; the survey comparison uses seed 2)")
    ap.add_argument("--survey-pair-iters", type=int, default=10)
    ap.add_argument("--load", default=None,
                    help="trained parameters (.npy) to use instead of generating and training")
    ap.add_argument("--plain", default="armijo", choices=["armijo", "wolfe"],
                    help="plain method the learned run must match: this module's projected "
                         "L-BFGS (armijo) or the inversion driver's strong-Wolfe L-BFGS (wolfe)")
    args = ap.parse_args(argv)
    if not torch.cuda.is_available():
        print("precond: no GPU visible", file=sys.stderr)
        return 1
    err = lambda m: print(m, file=sys.stderr, flush=True)
    st = FL.Settings(tv_weight=1e-3)
    out = {}
    if args.load:
        net = nn.Net(np.load(args.load, allow_pickle=False))
        out["params"] = args.load
    else:
        ds, gstats = generate(args.runs, args.iters, 10000, st, log=err, workers=args.workers)
        err(f"generate: {gstats}")
        sets = [ds]
        if args.survey_runs:
            ds2, gs2 = generate(args.survey_runs, args.survey_pair_iters, 20000, st, log=err,
                                workers=min(args.workers, 4), kind="survey")
            err(f"generate survey: {gs2}")
            out["generate_survey"] = gs2
            sets.append(ds2)
        net, thist = train(sets, args.epochs, args.batch, args.lr, log=err)
        if args.save:
            np.save(args.save, net.state_dict()["params"])
        out.update({"pairs": gstats["runs"] * args.iters, "generate": gstats,
                    "train": {k: thist[k] for k in ("steps", "seconds", "zero_predictor_val")},
                    "train_last": thist["epochs"][-1] if thist["epochs"] else None})
        del ds, sets
        torch.cuda.empty_cache()
    problems = []
    for k in range(args.eval):
        cfg, prob, obs, e, s, e0, s0 = tiny_problem(50000 + k, 6.0)
        problems.append((f"tiny-128x128-seed{50000 + k}", prob, obs, e0, s0))
    if problems:
        res = compare(net, problems, args.iters, st, log=err, plain_method=args.plain)
        out["compare"] = res
        out["summary"] = _summary(res)
    del problems
    from . import inputs as I
    if args.survey:
        r = compare(net, [_survey_problem(I.config_survey(), args.factor)], args.survey_iters, st,
                    log=err, verbose=True, plain_method=args.plain)
        out["compare_survey"] = r
    if args.large:
        torch.cuda.empty_cache()
        err("large: building the problem (observed traces)")
        r = compare(net, [_survey_problem(I.config_large(), args.factor)], args.large_iters, st,
                    log=err, verbose=True, plain_method=args.plain)
        out["compare_large"] = r
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
