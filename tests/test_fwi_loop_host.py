"""Host-side pieces of the FWI driver: the multiscale low-pass, the TV term
and the CPML padding of the interior model (plain torch on the CPU)."""
import numpy as np
import pytest
import torch

from paper_2506_20513_amd import fwi_loop as L


def _gauss_pulse(n, dt, f, t0, tau):
    """cos(2 pi f (t - t0)) under a Gaussian envelope of width tau: its
    spectrum is a line at f widened by about 1/(pi tau)."""
    t = np.arange(n) * dt
    return np.exp(-((t - t0) / tau) ** 2) * np.cos(2 * np.pi * f * (t - t0))


def test_lowpass_passes_low_and_stops_high_frequencies():
    n, dt, fc = 20000, 1e-11, 2e8
    lo = torch.tensor(_gauss_pulse(n, dt, 2e7, 1e-7, 2e-8))    # content below 60 MHz
    hi = torch.tensor(_gauss_pulse(n, dt, 2e9, 1e-7, 2e-9))    # 2 GHz +- 0.16 GHz
    ylo = L.lowpass(lo, dt, fc)
    yhi = L.lowpass(hi, dt, fc)
    # |H| = 1/sqrt(1 + (f/fc)^12): 1 - 3e-7 at 0.3 fc, below 2e-6 from 9 fc on;
    # the causal filter delays the pulse, so compare energies
    assert abs(float(torch.linalg.norm(ylo) / torch.linalg.norm(lo)) - 1) < 1e-5
    assert float(torch.linalg.norm(yhi) / torch.linalg.norm(hi)) < 1e-5


def test_lowpass_commutes_with_a_linear_filter():
    """Wavelet and traces filtered alike stay consistent: for a trace that is
    the wavelet convolved with a causal response h, filtering the wavelet
    first gives the filtered trace."""
    rng = np.random.default_rng(0)
    n, dt, fc = 4096, 1e-11, 3e8
    w = _gauss_pulse(n, dt, 4e8, 1e-8, 1.5e-9)
    h = np.zeros(400)
    h[rng.integers(0, 400, 12)] = rng.standard_normal(12)
    tr = np.convolve(w, h)[:n]
    a = L.lowpass(torch.tensor(tr), dt, fc).numpy()
    b = np.convolve(L.lowpass(torch.tensor(w), dt, fc).numpy(), h)[:n]
    assert np.linalg.norm(a - b) / np.linalg.norm(a) < 1e-12


def test_lowpass_along_time_axis_of_traces():
    x = torch.randn(3, 500, 7, dtype=torch.float64)
    y = L.lowpass(x, 1e-10, 1e9, dim=1)
    for r in range(7):
        assert torch.allclose(y[:, :, r], L.lowpass(x[:, :, r], 1e-10, 1e9, dim=-1))


def test_total_variation_of_a_step_and_of_a_ramp():
    n, d = 32, 1e-3
    step = torch.zeros(n, n, dtype=torch.float64)
    step[:, n // 2:] = 1.0
    tv = float(L.total_variation(step, delta=d))
    expect = (n * np.sqrt(1 + d * d) + (n * n - n) * d) / (n * n)
    assert abs(tv - expect) < 1e-12
    ramp = torch.arange(n, dtype=torch.float64)[None, :].repeat(n, 1) * 0.5
    # |Dx| = 0.5 except the last column (0); Dy = 0
    expect = ((n - 1) * n * np.sqrt(0.25 + d * d) + n * d) / (n * n)
    assert abs(float(L.total_variation(ramp, delta=d)) - expect) < 1e-12


def test_pad_interior_replicates_edges_and_sums_gradients():
    x = torch.arange(12, dtype=torch.float64).reshape(3, 4).requires_grad_(True)
    p = L.pad_interior(x, 2)
    assert p.shape == (7, 8)
    assert torch.equal(p[2:5, 2:6], x.detach())
    assert torch.equal(p[0, :], torch.tensor([0., 0, 0, 1, 2, 3, 3, 3], dtype=torch.float64))
    assert torch.equal(p[:, -1], torch.tensor([3., 3, 3, 7, 11, 11, 11], dtype=torch.float64))
    p.sum().backward()
    g = x.grad
    assert g[0, 0] == 9 and g[1, 1] == 1 and g[0, 1] == 3 and g[1, 0] == 3
    assert float(g.sum()) == 7 * 8


def test_problem_rejects_host_tensors():
    from paper_2506_20513_amd import autograd as AG, fwi
    grid = fwi.make_grid(10, 10, 2, 20, 0.01, 0.01, 1e-11)
    with pytest.raises(ValueError):
        AG.Problem(grid, np.array([[5, 5]]), np.array([[[6, 6]]]), np.zeros((1, 20)), device="cpu")


def test_pad_interior_gradient_equals_replicate_pad_adjoint():
    """The explicit adjoint of the edge replication equals autograd through
    torch's replicate padding (float64, CPU), including the corners."""
    import torch
    import torch.nn.functional as F
    from paper_2506_20513_amd import fwi_loop as L
    g = torch.Generator().manual_seed(3)
    x = torch.randn(7, 9, generator=g, dtype=torch.float64, requires_grad=True)
    w = torch.randn(7 + 6, 9 + 6, generator=g, dtype=torch.float64)
    (L.pad_interior(x, 3) * w).sum().backward()
    ours = x.grad.clone()
    x.grad = None
    (F.pad(x[None, None], (3, 3, 3, 3), mode="replicate")[0, 0] * w).sum().backward()
    assert torch.allclose(ours, x.grad, rtol=1e-13, atol=1e-13)
    assert torch.equal(L.pad_interior(x, 3).detach(),
                       F.pad(x[None, None], (3, 3, 3, 3), mode="replicate")[0, 0].detach())
