"""The allocation-free gradient entry point (fwi_gradient_static) against
fwi_gradient with a caller workspace, through the C ABI: two calls in a
row on one device, the second on a smaller problem, so the static scratch
holds the first call's state when the second starts.  The reference calls
run on a workspace filled with NaN bytes, so any read of a workspace byte
the call did not write first would show in its results."""
import numpy as np
import pytest

from paper_2506_20513_amd import fwi
from paper_2506_20513_amd import inputs as I

pytestmark = pytest.mark.gpu


def _problem(cfg, src, rec, seed):
    import torch
    e, s, e0, s0 = I.model_for(cfg)
    rng = np.random.default_rng(seed)
    w = torch.from_numpy(I.wavelets(cfg)[:len(src)].copy()).cuda()
    obs = torch.from_numpy(
        (1e-3 * rng.standard_normal((len(src), cfg.nt, rec.shape[1]))).astype(np.float32)).cuda()
    return dict(grid=fwi.grid_from_config(cfg), geom=fwi.Geometry(src, rec, w), w=w,
                e0=torch.from_numpy(e0).cuda(), s0=torch.from_numpy(s0).cuda(), obs=obs,
                shape=(cfg.NY, cfg.NX), tshape=(len(src), cfg.nt, rec.shape[1]))


def _outputs(p):
    import torch
    return (torch.full((1,), float("nan"), dtype=torch.float64, device="cuda"),
            torch.full(p["shape"], float("nan"), device="cuda"),
            torch.full(p["shape"], float("nan"), device="cuda"),
            torch.full(p["tshape"], float("nan"), device="cuda"))


def _reference(p):
    import torch
    nb = fwi.workspace_bytes(p["grid"], p["geom"], fwi.GRADIENT_WORKSPACE)
    ws = fwi.alloc_workspace(nb)
    ws.fill_(255)                      # every float in the workspace is NaN
    out = _outputs(p)
    fwi.fwi_gradient(p["grid"], p["geom"], p["e0"], p["s0"], p["obs"], *out, ws)
    torch.cuda.synchronize()
    return [o.cpu() for o in out]


def _static(p):
    import torch
    out = _outputs(p)
    fwi.fwi_gradient_static(p["grid"], p["geom"], p["e0"], p["s0"], p["obs"], *out)
    torch.cuda.synchronize()
    return [o.cpu() for o in out]


def test_static_gradient_matches_workspace_gradient_twice():
    import torch
    big = I.config_tiny().with_(nt=400)
    src, rec = I.geometry(big)
    A = _problem(big, src, rec, 1)
    small = I.RunConfig("small-60x44", 60, 44, 6, 250, 0.02, 0.02, 300e6, 2, 7)
    src_b = np.array([[20, 8], [45, 30]], np.int32)
    rec_b = np.array([[[8 + 6 * r, 10] for r in range(7)],
                      [[10 + 5 * r, 40] for r in range(7)]], np.int32)
    B = _problem(small, src_b, rec_b, 2)
    nA = fwi.workspace_bytes(A["grid"], A["geom"], fwi.GRADIENT_WORKSPACE)
    nB = fwi.workspace_bytes(B["grid"], B["geom"], fwi.GRADIENT_WORKSPACE)
    assert nB < nA <= fwi.STATIC_SCRATCH_BYTES
    print(f"static scratch: problem A {nA / 2**20:.1f} MiB, problem B {nB / 2**20:.1f} MiB",
          flush=True)

    refA, refB = _reference(A), _reference(B)
    for name, p, ref in (("A", A, refA), ("B", B, refB)):
        got = _static(p)
        for k, (g, r) in enumerate(zip(got, ref)):
            assert torch.isfinite(r).all(), (name, k)
            assert torch.equal(g, r), (name, k, float((g - r).abs().max()))
