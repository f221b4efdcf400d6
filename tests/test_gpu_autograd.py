"""The autograd layer and the FWI driver on the GPU.

- traces() with a loss of 1/2 sum (traces - observed)^2 back-propagates to
  the same gradient the fused fwi_gradient call returns;
- traces() under another loss back-propagates to the oracle's adjoint
  gradient of that loss;
- misfit() scales its stored gradient by the incoming gradient;
- a backward pass after the problem ran another forward raises;
- a short multiscale L-BFGS inversion on the 128x128 workload lowers the
  misfit of every band and moves eps_r towards the true model.
"""
import numpy as np
import pytest

from paper_2506_20513_amd import fwi
from paper_2506_20513_amd import inputs as I

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU visible")
    fwi.lib()


@pytest.fixture(scope="module")
def case():
    import torch
    from paper_2506_20513_amd import autograd as AG
    cfg = I.config_tiny().with_(nt=600)
    e, s, e0, s0 = I.model_for(cfg)
    src, rec = I.geometry(cfg)
    w = torch.from_numpy(I.wavelets(cfg)).cuda()
    prob = AG.Problem(fwi.grid_from_config(cfg), src, rec, w)
    T = lambda a: torch.from_numpy(a).cuda()
    with torch.no_grad():
        obs = AG.traces(prob, T(e), T(s))
    return dict(cfg=cfg, prob=prob, e=T(e), s=T(s), e0=T(e0), s0=T(s0), w=w, obs=obs)


def test_traces_backward_matches_fused_gradient(case):
    import torch
    from paper_2506_20513_amd import autograd as AG
    prob = case["prob"]
    e = case["e0"].clone().requires_grad_(True)
    s = case["s0"].clone().requires_grad_(True)
    tr = AG.traces(prob, e, s)
    loss = 0.5 * ((tr - case["obs"]) ** 2).sum()
    loss.backward()
    ws = fwi.alloc_workspace(fwi.workspace_bytes(prob.grid, prob.geom, fwi.GRADIENT_WORKSPACE))
    mis = torch.empty(1, dtype=torch.float64, device="cuda")
    ge = torch.empty_like(e)
    gs = torch.empty_like(s)
    fwi.fwi_gradient(prob.grid, prob.geom, case["e0"], case["s0"], case["obs"], mis, ge, gs,
                     None, ws)
    torch.cuda.synchronize()
    for a, b in ((e.grad, ge), (s.grad, gs)):
        err = float(torch.linalg.norm(a - b) / torch.linalg.norm(b))
        print("traces-backward vs fused gradient", err, flush=True)
        assert err <= 1e-6
    assert abs(float(loss) - float(mis)) <= 1e-5 * float(mis)


def test_traces_backward_matches_oracle_adjoint():
    """traces() under a loss that is not the misfit: L = sum q * traces +
    1/2 sum (traces - observed)^2 with fixed random weights q.  Its backward
    feeds dL/dtraces to the HIP adjoint; the oracle runs its own adjoint
    (Algorithm 2) with the same adjoint source evaluated at its own traces.
    Gradients within 1e-3, the loss within 1e-4 (relative)."""
    import torch

    import oracle
    from paper_2506_20513_amd import autograd as AG
    from tests.gpu_util import rel_l2
    cfg = I.config_tiny().with_(nt=600)
    e, s, e0, s0 = I.model_for(cfg)
    src, rec = I.geometry(cfg)
    wn = I.wavelets(cfg)
    kw = dict(cpml_order=cfg.cpml_order, cpml_sigma_scale=cfg.cpml_sigma_scale,
              cpml_kappa_max=cfg.cpml_kappa_max, cpml_alpha_max=cfg.cpml_alpha_max)
    obs, _ = oracle.Problem(e, s, cfg.npml, cfg.dx, cfg.dy, cfg.dt, **kw).forward(
        src, rec, wn, cfg.nt)
    obs = obs.astype(np.float32)
    rng = np.random.default_rng(12)
    q = (float(np.abs(obs).max()) * rng.standard_normal(obs.shape)).astype(np.float32)

    P = oracle.Problem(e0, s0, cfg.npml, cfg.dx, cfg.dy, cfg.dt, **kw)
    otr, hists = P.forward(src, rec, wn, cfg.nt, keep_history=True)
    oL = float(np.sum(q.astype(np.float64) * otr) + 0.5 * np.sum((otr - obs) ** 2))
    oge, ogs, _ = P.adjoint(src, rec, q + (otr - obs), hists, cfg.nt)
    del hists

    w = torch.from_numpy(wn).cuda()
    prob = AG.Problem(fwi.grid_from_config(cfg), src, rec, w)
    et = torch.from_numpy(e0).cuda().requires_grad_(True)
    st = torch.from_numpy(s0).cuda().requires_grad_(True)
    tr = AG.traces(prob, et, st)
    qt, ot = torch.from_numpy(q).cuda(), torch.from_numpy(obs).cuda()
    loss = (qt.double() * tr.double()).sum() + 0.5 * ((tr.double() - ot.double()) ** 2).sum()
    loss.backward()
    errs = {"loss": abs(float(loss.detach()) - oL) / abs(oL),
            "eps": rel_l2(et.grad.cpu().numpy(), oge), "sig": rel_l2(st.grad.cpu().numpy(), ogs)}
    print("autograd vs oracle", errs, flush=True)
    assert errs["loss"] <= 1e-4
    assert errs["eps"] <= 1e-3 and errs["sig"] <= 1e-3


def test_misfit_backward_scales_with_the_incoming_gradient(case):
    from paper_2506_20513_amd import autograd as AG
    prob = case["prob"]
    e = case["e0"].clone().requires_grad_(True)
    s = case["s0"].clone().requires_grad_(True)
    J = AG.misfit(prob, e, s, case["obs"])
    (3.0 * J).backward()
    g3e, g3s = e.grad.clone(), s.grad.clone()
    e.grad = None
    s.grad = None
    AG.misfit(prob, e, s, case["obs"]).backward()
    assert J.dtype.is_floating_point and float(J) > 0
    assert np.allclose(g3e.cpu().numpy(), 3.0 * e.grad.cpu().numpy(), rtol=1e-6, atol=0)
    assert np.allclose(g3s.cpu().numpy(), 3.0 * s.grad.cpu().numpy(), rtol=1e-6, atol=0)


def test_backward_after_another_forward_raises(case):
    import torch
    from paper_2506_20513_amd import autograd as AG
    prob = case["prob"]
    e = case["e0"].clone().requires_grad_(True)
    tr1 = AG.traces(prob, e, case["s0"])
    tr2 = AG.traces(prob, e, case["s0"])
    with pytest.raises(RuntimeError):
        tr1.sum().backward()
    tr2.sum().backward()            # the latest one is still valid
    torch.cuda.synchronize()
    assert torch.isfinite(e.grad).all()


def test_wrong_shapes_are_rejected_before_launch(case):
    import torch
    from paper_2506_20513_amd import autograd as AG
    prob = case["prob"]
    with pytest.raises(ValueError):
        AG.traces(prob, case["e0"][:-1], case["s0"][:-1])
    with pytest.raises(ValueError):
        AG.misfit(prob, case["e0"], case["s0"], case["obs"][:, :-1])
    with pytest.raises(TypeError):
        AG.traces(prob, case["e0"].double(), case["s0"])


def test_short_multiscale_inversion_reduces_misfit(case):
    import torch
    from paper_2506_20513_amd import fwi_loop as L
    cfg, prob = case["cfg"], case["prob"]
    st = L.Settings(bands=(100e6, None), iters=8, optimizer="lbfgs", tv_weight=1e-3)
    r = L.invert(prob, case["w"], case["obs"], case["e0"], case["s0"], st, cfg.dt,
                 log=lambda m: print(m, flush=True))
    sl = (slice(cfg.npml, cfg.NY - cfg.npml), slice(cfg.npml, cfg.NX - cfg.npml))

    def rel(a, b):
        return float(torch.linalg.norm(a[sl] - b[sl]) / torch.linalg.norm(b[sl]))

    for band in (100e6, 0.0):
        h = [x for x in r.history if x.band == band]
        print("band", band, "relative misfit", h[0].rel_misfit, "->", h[-1].rel_misfit, flush=True)
        assert h[-1].rel_misfit < 0.7
    e_before, e_after = rel(case["e0"], case["e"]), rel(r.eps_r, case["e"])
    print("eps_r model error", e_before, "->", e_after, flush=True)
    assert e_after < e_before
    assert float(r.eps_r.min()) >= 1.0 and float(r.sigma.min()) >= 0.0


def test_paper_recipe_adam_with_algorithm3_tv(case):
    """The paper's schedule (Adam, eps_r alone first, then both, Algorithm 3
    TV through the HIP kernel) lowers the misfit and keeps sigma fixed
    during the eps_r-only stage."""
    import torch
    from paper_2506_20513_amd import fwi_loop as L
    cfg, prob = case["cfg"], case["prob"]
    st = L.paper_recipe(iters=12, stage1=4)
    seen = []
    r = L.invert(prob, case["w"], case["obs"], case["e0"], case["s0"], st, cfg.dt,
                 log=lambda m: print(m, flush=True))
    h = r.history
    print("paper recipe relative misfit", h[0].rel_misfit, "->", h[-1].rel_misfit, flush=True)
    assert h[-1].rel_misfit < 0.9 * h[0].rel_misfit
    assert float(r.eps_r.min()) >= 1.0 and float(r.sigma.min()) >= 0.0
    st1 = L.paper_recipe(iters=3, stage1=5)       # eps_r-only for every iteration
    r1 = L.invert(prob, case["w"], case["obs"], case["e0"], case["s0"], st1, cfg.dt, log=seen.append)
    # sigma untouched (up to the float32 round trip through normalised units)
    assert torch.allclose(r1.sigma, case["s0"], rtol=1e-6, atol=0)
    with pytest.raises(ValueError):
        L.invert(prob, case["w"], case["obs"], case["e0"], case["s0"],
                 L.Settings(bands=(None,), iters=1, tv_mode="admm"), cfg.dt, log=seen.append)


def test_driver_snapshot_and_resume(tmp_path, capsys):
    """The driver writes the models after every band and a second run
    resumes from that snapshot (its starting model error is the first run's
    final one)."""
    import json
    from paper_2506_20513_amd import fwi_loop as L
    snap = str(tmp_path / "snap.npz")
    assert L.main(["--workload", "tiny", "--bands", "100e6", "--iters", "3",
                   "--snapshot", snap]) == 0
    first = json.loads(capsys.readouterr().out.strip().splitlines()[-1])
    assert first["bands"][0]["evaluations"] >= 1
    assert L.main(["--workload", "tiny", "--bands", "full", "--iters", "2",
                   "--init-model", snap]) == 0
    second = json.loads(capsys.readouterr().out.strip().splitlines()[-1])
    assert abs(second["eps_model_error_start"] - first["eps_model_error_final"]) <= 1e-6
    assert second["init_model"] == snap
