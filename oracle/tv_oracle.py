"""FP64 CPU oracle of the total-variation regularisation step (arXiv
2506.20513, Sec. 3.4 "Optimization strategy", Algorithm 3 and the TV
definition that follows it).

TEST INFRASTRUCTURE ONLY: only the tests, the smoke check and the
benchmark's CPU-baseline leg may use it.  The product library shares no
code with it.

Reading of Algorithm 3.  The paper names the steps but not the equations,
so this is a split-Bregman (ADMM) iteration for the TV-denoising
(Rudin-Osher-Fatemi) problem

    U* = argmin_U  mu/2 ||U - Xn||^2 + TV(U),
    TV(U) = sum_ij sqrt((Dx U)^2 + (Dy U)^2),

where Dx, Dy are circular forward differences and Xn = X / s is the model
divided by its largest magnitude s (the "initialize" and "restore scale"
steps).  Auxiliaries Z = (Zx, Zy) stand for (Dx U, Dy U); B = (Bx, By) are
the scaled multipliers.  Start: U = Xn, Z = B = 0.  One iteration:

  2. backward differences (circular) of Zx - Bx and Zy - By, which give the
     adjoint D^T (Z - B) = -(bwd_x(Zx - Bx) + bwd_y(Zy - By));
  3. right-hand side  R = mu Xn + lam D^T (Z - B);
  4. a linearised solve of (mu + lam D^T D) U = R, D^T D being the 5-point
     negative Laplacian (eigenvalues in [0, 8]): U <- (R + lam (4 U + sum
     of the 4 neighbours of U)) / (mu + 8 lam), i.e. the neighbour average
     is the convolution of U with [[0,1,0],[1,4,1],[0,1,0]] / 8.  This is
     the proximal (linearised) ADMM step with metric lam (8 I - D^T D),
     which is positive semidefinite, so the iteration converges to the ROF
     minimiser for every mu, lam > 0.  A plain Jacobi sweep, U <- (R + lam
     * neighbour sum) / (mu + 4 lam), corresponds to an indefinite metric
     and stalls at wrong points once lam exceeds about mu / 5;
  5. forward differences (circular) of the new U;
  6. Z <- shrink(D U + B, 1/lam), the isotropic soft threshold
     shrink(w, t) = w max(|w| - t, 0) / |w|, |w| = sqrt(wx^2 + wy^2);
  7. B <- B + D U - Z.

  8. The result is s U.  The term added to the model gradient is
     weight * (X - s U): the gradient of the Moreau envelope of the TV term
     (zero on a constant model, pulling each cell towards its TV-denoised
     value otherwise).

Pins (tests/test_tv_oracle.py): a constant model is a fixed point; the
iteration converges to the ROF minimiser computed by Chambolle's dual
projection algorithm (an independent method); a two-level step profile
has the closed-form ROF solution; the shrink function matches its closed
form; planted mistakes fail at least one pin.
"""
from __future__ import annotations

import numpy as np


def fwd_x(U):
    """(Dx U)[j, i] = U[j, i+1] - U[j, i], circular in i (axis 1)."""
    return np.roll(U, -1, axis=1) - U


def fwd_y(U):
    """(Dy U)[j, i] = U[j+1, i] - U[j, i], circular in j (axis 0)."""
    return np.roll(U, -1, axis=0) - U


def bwd_x(V):
    """V[j, i] - V[j, i-1], circular."""
    return V - np.roll(V, 1, axis=1)


def bwd_y(V):
    """V[j, i] - V[j-1, i], circular."""
    return V - np.roll(V, 1, axis=0)


def neighbour_sum(U):
    """Sum of the four edge neighbours (circular), the 5-point stencil
    without its centre."""
    return (np.roll(U, 1, axis=0) + np.roll(U, -1, axis=0)
            + np.roll(U, 1, axis=1) + np.roll(U, -1, axis=1))


def shrink(wx, wy, t):
    """Isotropic soft threshold of the vector field (wx, wy) at t."""
    mag = np.sqrt(wx * wx + wy * wy)
    f = np.where(mag > t, (mag - t) / np.where(mag > 0, mag, 1.0), 0.0)
    return wx * f, wy * f


def tv(U):
    """Isotropic TV with circular forward differences."""
    return float(np.sum(np.sqrt(fwd_x(U) ** 2 + fwd_y(U) ** 2)))


def tv_denoise(X, mu: float, lam: float, iters: int):
    """Algorithm 3 steps 1-8 on one 2D model X [ny][nx]; returns s U."""
    X = np.asarray(X, dtype=np.float64)
    s = float(np.max(np.abs(X)))
    if s == 0.0:
        return np.zeros_like(X)
    Xn = X / s                                            # 1. initialise
    U = Xn.copy()
    Zx = np.zeros_like(Xn)
    Zy = np.zeros_like(Xn)
    Bx = np.zeros_like(Xn)
    By = np.zeros_like(Xn)
    for _ in range(iters):
        DtZB = -(bwd_x(Zx - Bx) + bwd_y(Zy - By))        # 2. backward differences
        R = mu * Xn + lam * DtZB                          # 3. right-hand side
        U = (R + lam * (4.0 * U + neighbour_sum(U))) / (mu + 8.0 * lam)   # 4. neighbour average
        DxU, DyU = fwd_x(U), fwd_y(U)                     # 5. forward differences
        Zx, Zy = shrink(DxU + Bx, DyU + By, 1.0 / lam)    # 6. soft threshold
        Bx = Bx + DxU - Zx                                # 7. multipliers
        By = By + DyU - Zy
    return s * U                                          # 8. restore scale


def tv_gradient(X, mu: float, lam: float, iters: int, weight: float):
    """The term Algorithm 3 adds to a model gradient: weight (X - TVdenoise(X))."""
    X = np.asarray(X, dtype=np.float64)
    return weight * (X - tv_denoise(X, mu, lam, iters))
