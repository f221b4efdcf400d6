"""Parity of the TV-regularisation kernel (include/fwi_tv.h, Algorithm 3)
with the FP64 oracle (oracle/tv_oracle.py) on the same seeded models.

The kernel iterates in float32.  The iteration is a contraction towards the
TV-denoised model, so rounding errors do not grow; the comparison is on the
added gradient term weight * (X - s U), a difference of nearly equal
values, in relative L2 against the gradient tolerance 1e-3 (measured
values are printed)."""
import numpy as np
import pytest

import oracle.tv_oracle as T
from paper_2506_20513_amd import tv

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU visible")
    tv.lib()


def _models(nf, ny, nx, seed):
    rng = np.random.default_rng(seed)
    X = np.empty((nf, ny, nx))
    for f in range(nf):
        base = rng.uniform(3, 20) if f == 0 else rng.uniform(0.001, 0.05)
        X[f] = base * (1 + 0.2 * rng.standard_normal((ny, nx)))
        X[f, ny // 3: ny // 2, nx // 4: nx // 2] *= 1.5
    return X.astype(np.float32)


@pytest.mark.parametrize("nf,ny,nx,iters", [(2, 37, 70, 1), (2, 37, 70, 2), (2, 64, 130, 30),
                                            (1, 5, 3, 12), (2, 256, 512, 20)])
def test_tv_gradient_matches_oracle(nf, ny, nx, iters):
    import torch
    X = _models(nf, ny, nx, 11 + ny)
    mu, lam, w = [6.0, 4.0][:nf], [2.0, 3.0][:nf], [0.5, 2.0][:nf]
    g0 = np.random.default_rng(1).standard_normal((nf, ny, nx)).astype(np.float32)
    op = tv.TV(nf, ny, nx, mu, lam, w, iters)
    Xd = torch.from_numpy(X).cuda()
    gd = torch.from_numpy(g0).cuda()
    op(Xd, gd)
    torch.cuda.synchronize()
    got = gd.cpu().numpy().astype(np.float64) - g0
    for f in range(nf):
        ref = T.tv_gradient(X[f].astype(np.float64), mu[f], lam[f], iters, w[f])
        e = np.linalg.norm(got[f] - ref) / np.linalg.norm(ref)
        print(f"field {f} {ny}x{nx} iters {iters}: rel L2 {e:.2e}", flush=True)
        assert e <= 1e-3


def test_tv_constant_and_zero_fields_add_nothing():
    import torch
    X = np.zeros((2, 9, 66), np.float32)
    X[0] = 7.5
    op = tv.TV(2, 9, 66, 5.0, 2.0, 1.0, 10)
    g = torch.full((2, 9, 66), 0.25, device="cuda")
    op(torch.from_numpy(X).cuda(), g)
    torch.cuda.synchronize()
    assert float((g - 0.25).abs().max()) <= 1e-6


def test_tv_repeated_calls_are_identical():
    import torch
    X = torch.from_numpy(_models(2, 40, 96, 3)).cuda()
    op = tv.TV(2, 40, 96, 5.0, 2.0, 1.0, 15)
    a = torch.zeros(2, 40, 96, device="cuda")
    b = torch.zeros(2, 40, 96, device="cuda")
    op(X, a)
    op(X, b)
    torch.cuda.synchronize()
    assert torch.equal(a, b)
