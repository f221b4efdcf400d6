"""Pins of the TV-regularisation oracle (oracle/tv_oracle.py, Algorithm 3
of arXiv 2506.20513 read as split-Bregman TV denoising), each fixed by
something other than the oracle itself:

- a constant model is a fixed point (the TV term of a flat model is zero);
- a two-level step profile (rows identical, circular) converges to the
  closed-form ROF solution u1 = a + 2 s / (mu L1), u2 = b - 2 s / (mu L2);
- a random model converges to the ROF minimiser computed by Chambolle's
  dual projection algorithm (2004), written here independently;
- the isotropic soft threshold matches its closed form element by element;
- planted mistakes in a copy of the oracle fail at least one pin.
"""
import importlib.util
import math
import os
import sys

import numpy as np
import pytest

import oracle.tv_oracle as T

SRC = T.__file__


def _chambolle(f, theta, iters=60000, tau=0.124):
    """argmin_u 1/(2 theta) ||u - f||^2 + sum sqrt(ux^2 + uy^2), circular
    forward differences; Chambolle, J. Math. Imaging Vis. 20 (2004),
    projection algorithm, u = f - theta div p."""
    ny, nx = f.shape
    px = np.zeros_like(f)
    py = np.zeros_like(f)
    ip = [(i + 1) % nx for i in range(nx)]
    im = [(i - 1) % nx for i in range(nx)]
    jp = [(j + 1) % ny for j in range(ny)]
    jm = [(j - 1) % ny for j in range(ny)]
    for _ in range(iters):
        div = (px - px[:, im]) + (py - py[jm, :])
        w = div - f / theta
        gx = w[:, ip] - w
        gy = w[jp, :] - w
        den = 1.0 + tau * np.sqrt(gx * gx + gy * gy)
        px = (px + tau * gx) / den
        py = (py + tau * gy) / den
    div = (px - px[:, im]) + (py - py[jm, :])
    return f - theta * div


def _rof_energy(U, Xn, mu):
    ux = np.roll(U, -1, 1) - U
    uy = np.roll(U, -1, 0) - U
    return 0.5 * mu * float(np.sum((U - Xn) ** 2)) + float(np.sum(np.sqrt(ux ** 2 + uy ** 2)))


# ---------------------------------------------------------------------------
def pin_constant(mod=T):
    X = np.full((5, 7), 3.25)
    return float(np.max(np.abs(mod.tv_gradient(X, 8.0, 2.0, 25, 1.0))))


def pin_step(mod=T):
    a, b, L1, L2, mu = 1.5, 4.0, 5, 7, 6.0
    X = np.tile(np.r_[np.full(L1, a), np.full(L2, b)], (4, 1))
    s = 4.0
    want = np.tile(np.r_[np.full(L1, a + 2 * s / (mu * L1)), np.full(L2, b - 2 * s / (mu * L2))], (4, 1))
    U = mod.tv_denoise(X, mu, 4.0, 3000)
    return float(np.max(np.abs(U - want)))


def pin_chambolle(mod=T):
    rng = np.random.default_rng(3)
    X = rng.uniform(0.5, 2.0, size=(6, 7))
    X[2:5, 1:4] += 1.5
    mu = 5.0
    s = float(np.max(np.abs(X)))
    Uc = s * _chambolle(X / s, 1.0 / mu)
    Ua = mod.tv_denoise(X, mu, 3.0, 6000)
    return float(np.max(np.abs(Ua - Uc))) / s


def pin_shrink(mod=T):
    rng = np.random.default_rng(4)
    wx, wy = rng.normal(size=(2, 9, 11))
    t = 0.8
    zx, zy = mod.shrink(wx, wy, t)
    worst = 0.0
    for j in range(9):
        for i in range(11):
            m = math.hypot(wx[j, i], wy[j, i])
            k = max(m - t, 0.0) / m if m > 0 else 0.0
            worst = max(worst, abs(zx[j, i] - k * wx[j, i]), abs(zy[j, i] - k * wy[j, i]))
    return worst


def test_constant_model_is_a_fixed_point():
    assert pin_constant() <= 1e-13


def test_step_profile_matches_closed_form_rof_solution():
    e = pin_step()
    print("step profile error", e)
    assert e <= 1e-8


def test_converges_to_the_chambolle_rof_minimiser():
    e = pin_chambolle()
    print("relative distance to the Chambolle solution", e)
    assert e <= 1e-5


def test_shrink_matches_closed_form():
    assert pin_shrink() <= 1e-15


def test_zero_model_and_energy_decrease():
    assert np.all(T.tv_denoise(np.zeros((3, 4)), 2.0, 1.0, 5) == 0)
    rng = np.random.default_rng(5)
    X = rng.uniform(1, 3, size=(8, 9))
    s = float(np.max(np.abs(X)))
    U = T.tv_denoise(X, 4.0, 2.0, 400) / s
    assert _rof_energy(U, X / s, 4.0) < _rof_energy(X / s, X / s, 4.0)


# ---------------------------------------------------------------------------
MUTATIONS = [
    ("adjoint-sign", "DtZB = -(bwd_x(Zx - Bx) + bwd_y(Zy - By))",
     "DtZB = (bwd_x(Zx - Bx) + bwd_y(Zy - By))", ["chambolle", "step"]),
    ("forward-as-backward", "DxU, DyU = fwd_x(U), fwd_y(U)",
     "DxU, DyU = bwd_x(U), bwd_y(U)", ["chambolle", "step"]),
    ("plain-jacobi", "(R + lam * (4.0 * U + neighbour_sum(U))) / (mu + 8.0 * lam)",
     "(R + lam * neighbour_sum(U)) / (mu + 4.0 * lam)", ["chambolle"]),
    ("centre-weight", "(mu + 8.0 * lam)", "(mu + 4.0 * lam)", ["constant"]),
    ("multiplier-sign", "Bx = Bx + DxU - Zx", "Bx = Bx - DxU + Zx", ["chambolle", "step"]),
    ("threshold", "shrink(DxU + Bx, DyU + By, 1.0 / lam)", "shrink(DxU + Bx, DyU + By, lam)",
     ["chambolle", "step"]),
    ("transposed-axis", "return np.roll(U, -1, axis=1) - U", "return np.roll(U, -1, axis=0) - U",
     ["chambolle", "step"]),
    ("anisotropic-shrink", "mag = np.sqrt(wx * wx + wy * wy)", "mag = np.abs(wx) + np.abs(wy)",
     ["shrink", "chambolle"]),
    ("no-rescale", "return s * U  ", "return U  ", ["constant", "step"]),
]

PINS = {
    "constant": (pin_constant, 1e-13),
    "step": (pin_step, 1e-8),
    "chambolle": (pin_chambolle, 1e-5),
    "shrink": (pin_shrink, 1e-15),
}


@pytest.mark.parametrize("name,old,new,catchers", MUTATIONS, ids=[m[0] for m in MUTATIONS])
def test_tv_pins_catch_planted_mistake(tmp_path, name, old, new, catchers):
    src = open(SRC).read()
    assert src.count(old) == 1, f"mutation anchor not unique/present: {old!r}"
    p = tmp_path / "tv_mutant.py"
    p.write_text(src.replace(old, new))
    spec = importlib.util.spec_from_file_location("tv_mutant_" + name.replace("-", "_"), p)
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    caught = []
    for pin in catchers:
        fn, tol = PINS[pin]
        with np.errstate(all="ignore"):
            v = fn(mod)
        if not (v <= tol):
            caught.append(pin)
    assert caught, f"mutation {name} not caught by {catchers}"
