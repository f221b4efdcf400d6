"""Host checks of the optimiser under the learned preconditioner (no GPU):
the L-BFGS two-loop recursion satisfies the secant equation, the projected
L-BFGS run minimises a convex quadratic, an exact proposal is accepted in
one step, and a bad proposal is always rejected in favour of the plain
step (the misfit decrease is the judge)."""
import numpy as np
import pytest
import torch

from paper_2506_20513_amd import precond as PC


class Quadratic:
    """f(x) = 1/2 (x - x*)^T A (x - x*) with the Objective interface."""

    def __init__(self, n=40, cond=100.0, seed=0, lo=None):
        g = torch.Generator().manual_seed(seed)
        Q, _ = torch.linalg.qr(torch.randn(n, n, generator=g, dtype=torch.float64))
        ev = torch.logspace(0, np.log10(cond), n, dtype=torch.float64)
        self.A = Q @ torch.diag(ev) @ Q.T
        self.xs = torch.randn(n, generator=g, dtype=torch.float64)
        self.x0 = torch.zeros(n, dtype=torch.float64)
        self.free = torch.ones(n, dtype=torch.bool)
        self.free[:3] = False
        self.lo = torch.full((n,), -1e30, dtype=torch.float64) if lo is None else lo
        self.evals = 0
        self.last_J = None
        self.J0 = None
        self.ny, self.nx = 1, n // 2

    def project(self, x):
        return torch.maximum(torch.where(self.free, x, self.x0), self.lo)

    def __call__(self, x):
        r = x - self.xs
        f = 0.5 * float(r @ self.A @ r)
        self.evals += 1
        self.last_J = f
        if self.J0 is None:
            self.J0 = f
        g = torch.where(self.free, self.A @ r, torch.zeros_like(r))
        return f, g

    def constrained_min(self):
        # minimiser over the free coordinates with the fixed ones at x0
        F = self.free
        x = self.x0.clone()
        Aff = self.A[F][:, F]
        Afx = self.A[F][:, ~F]
        x[F] = self.xs[F] - torch.linalg.solve(Aff, Afx @ (x[~F] - self.xs[~F]))
        return x


def test_two_loop_satisfies_the_secant_equation():
    q = Quadratic()
    mem = PC.LBFGS(history=5)
    g = torch.Generator().manual_seed(1)
    for _ in range(4):
        s = torch.randn(40, generator=g, dtype=torch.float64)
        mem.update(s, q.A @ s)
    s, y = mem.S[-1], mem.Y[-1]
    assert torch.allclose(mem.direction(y), -s, rtol=1e-10, atol=1e-12)
    # pairs without positive curvature are not stored
    n = len(mem.S)
    mem.update(torch.ones(40, dtype=torch.float64), -torch.ones(40, dtype=torch.float64))
    assert len(mem.S) == n
    assert PC.LBFGS().direction(y) is None


def test_history_is_bounded():
    mem = PC.LBFGS(history=3)
    for k in range(6):
        s = torch.zeros(5, dtype=torch.float64)
        s[k % 5] = 1.0
        mem.update(s, 2 * s)
    assert len(mem.S) == 3 and torch.equal(mem.S[-1], mem.Y[-1] / 2)


def test_minimise_converges_on_a_quadratic_with_fixed_coordinates():
    q = Quadratic()
    run = PC.minimise(q, 200, first_step=0.5)
    xm = q.constrained_min()
    r = xm - q.xs
    fmin = 0.5 * float(r @ q.A @ r)
    print("f", run.final_f, "min", fmin, "evals", q.evals)
    assert run.final_f - fmin <= 1e-10 * q.J0
    assert torch.equal(run.x[:3], q.x0[:3])
    fs = [it.f for it in run.log]
    assert all(b <= a for a, b in zip(fs, fs[1:]))       # Armijo: monotone


def test_minimise_respects_the_lower_bounds():
    lo = torch.full((40,), -1e30, dtype=torch.float64)
    lo[10:20] = 0.5
    q = Quadratic(lo=lo)
    run = PC.minimise(q, 100, first_step=0.5)
    assert float(run.x[10:20].min()) >= 0.5
    assert run.final_f < q.J0


def test_exact_proposal_is_accepted_and_bad_one_falls_back():
    q = Quadratic(seed=3)
    xm = q.constrained_min()
    run = PC.minimise(q, 5, proposer=lambda x, g: xm - x)
    assert run.log[1].source == "net" and run.final_f <= 1e-12 * q.J0 + 0.5 * float(
        (xm - q.xs) @ q.A @ (xm - q.xs))
    plain = PC.minimise(Quadratic(seed=4), 15)
    bad = PC.minimise(Quadratic(seed=4), 15, proposer=lambda x, g: g.clone())
    assert [it.f for it in bad.log] == [it.f for it in plain.log]
    assert all(it.source != "net" for it in bad.log)


def test_ascent_proposals_after_a_good_one_are_struck():
    """A proposer that is right once and then proposes ascent directions is
    dropped after max_strikes proposals: the ascent proposals count as
    strikes even though the good proposal before them passed."""
    q = Quadratic(seed=6)
    xm = q.constrained_min()
    calls = []

    def proposer(x, g):
        calls.append(len(calls))
        if len(calls) == 1:
            return 0.5 * (xm - x)          # a good step, first trial passes
        return g.clone()                    # ascent from then on

    run = PC.minimise(q, 12, proposer=proposer, max_strikes=2)
    assert run.log[1].source == "net"
    assert len(calls) == 3, calls           # one good proposal, then two strikes
    assert all(it.source != "net" for it in run.log[2:])


def test_strong_wolfe_plain_run_minimises_and_keeps_fixed_coordinates():
    """The driver's strong-Wolfe L-BFGS on the same objective interface
    (the plain method of the comparison) converges on the quadratic, keeps
    the fixed coordinates and reports its final objective."""
    q = Quadratic(seed=7)
    run = PC.minimise_wolfe(q, 60)
    xm = q.constrained_min()
    r = xm - q.xs
    fmin = 0.5 * float(r @ q.A @ r)
    assert run.final_f - fmin <= 1e-8 * q.J0
    assert torch.equal(run.x[:3], q.x0[:3])
    assert run.log[-1].evals == q.evals and run.log[-1].evals >= 60


def test_target_stops_the_run():
    q = Quadratic(seed=5)
    full = PC.minimise(q, 50)
    tgt = full.log[10].f
    part = PC.minimise(Quadratic(seed=5), 50, target_f=tgt)
    assert part.final_f <= tgt and part.log[-1].k == 10


def test_wavelength_factor():
    """Models with more cells per wavelength than the training ones are
    resampled by the nearest power of two (cells per wavelength ~ 1/(f0 dx))."""
    assert PC.wavelength_factor(0.02, 200e6) == 1          # the training models
    assert PC.wavelength_factor(0.01, 400e6) == 1          # same cells per wavelength
    assert PC.wavelength_factor(0.005, 400e6) == 2         # twice as many
    assert PC.wavelength_factor(0.005, 200e6) == 4
    assert PC.wavelength_factor(0.04, 200e6) == 1          # coarser: never upsampled
