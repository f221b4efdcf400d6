"""Batched gradients of independent problems of uneven size on the GPU.

Every problem of a batch gets exactly what fwi_gradient gives it alone (bit
for bit: same per-cell arithmetic, and checkpoint re-forward equals stored
history for any interval); the captured graph replays the same results run
after run, with eager work in between; the result does not depend on the
autotuned band height; models updated in place are picked up by the next
run.  At temporal depth 8 (forced, or chosen by the autotuner over depth
and band height) the results agree within FP32 rounding.  Problems are also
checked against the FP64 oracle, with the oracle's own observed data.
"""
import numpy as np
import pytest

import oracle
from paper_2506_20513_amd import fwi
from paper_2506_20513_amd import inputs as I
from tests.gpu_util import np_, rel_l2

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU visible")
    fwi.lib()


def small_uneven(n=5, seed=9):
    rng = np.random.default_rng(seed)
    cfgs = []
    for m in range(n):
        nx, ny = int(rng.integers(60, 160)), int(rng.integers(40, 120))
        nt = int(rng.integers(150, 420))
        S, R = int(rng.integers(1, 4)), int(rng.integers(5, 21))
        cfgs.append(I.RunConfig(f"uneven-{m}-{nx}x{ny}", nx, ny, int(rng.integers(4, 12)), nt,
                                0.02, 0.02, 200e6, S, R))
    return cfgs


class Case:
    def __init__(self, cfg):
        import torch
        self.cfg = cfg
        e, s, e0, s0 = I.model_for(cfg)
        self.src, self.rec = I.geometry(cfg)
        self.w = torch.from_numpy(I.wavelets(cfg)).cuda()
        self.grid = fwi.grid_from_config(cfg)
        self.geom = fwi.Geometry(self.src, self.rec, self.w)
        T = lambda a: torch.from_numpy(a).cuda()
        self.e, self.s, self.e0, self.s0 = T(e), T(s), T(e0), T(s0)
        ws = fwi.alloc_workspace(fwi.workspace_bytes(self.grid, self.geom, fwi.FWI_SAVE_NONE))
        self.obs = torch.empty((cfg.nshots, cfg.nt, cfg.nrec), device="cuda")
        fwi.fdtd_forward(self.grid, self.geom, self.e, self.s, self.obs, fwi.FWI_SAVE_NONE, ws)
        self.mis = torch.full((1,), float("nan"), dtype=torch.float64, device="cuda")
        self.ge = torch.full((cfg.NY, cfg.NX), float("nan"), device="cuda")
        self.gs = torch.full((cfg.NY, cfg.NX), float("nan"), device="cuda")

    def problem(self):
        return fwi.BatchProblem(self.grid, self.geom, self.e0, self.s0, self.obs, self.mis,
                                self.ge, self.gs)

    def single(self):
        import torch
        ws = fwi.alloc_workspace(fwi.workspace_bytes(self.grid, self.geom, fwi.GRADIENT_WORKSPACE))
        mis = torch.empty(1, dtype=torch.float64, device="cuda")
        ge = torch.empty_like(self.ge)
        gs = torch.empty_like(self.gs)
        fwi.fwi_gradient(self.grid, self.geom, self.e0, self.s0, self.obs, mis, ge, gs, None, ws)
        torch.cuda.synchronize()
        return float(mis.item()), np_(ge), np_(gs)

    def result(self):
        return float(self.mis.item()), np_(self.ge), np_(self.gs)


def make_plan(cases, autotune=fwi.FWI_TUNE_BANDS):
    probs = [c.problem() for c in cases]
    ws = fwi.alloc_workspace(fwi.batch_workspace_bytes(probs))
    return fwi.BatchPlan(probs, ws, autotune=autotune)


@pytest.fixture(scope="module")
def batch():
    import torch
    cases = [Case(c) for c in small_uneven()]
    torch.cuda.synchronize()
    for c in cases:
        print("problem", c.cfg.name, "nt", c.cfg.nt, "shots", c.cfg.nshots, flush=True)
    plan = make_plan(cases)
    print("plan", plan.info(), flush=True)
    refs = [c.single() for c in cases]
    return dict(cases=cases, plan=plan, refs=refs)


def same(a, b):
    return a[0] == b[0] and np.array_equal(a[1], b[1]) and np.array_equal(a[2], b[2])


def test_batched_equals_single_problem_gradients(batch):
    import torch
    info = batch["plan"].info()
    assert info["graph"] and info["nproblems"] == len(batch["cases"])
    batch["plan"].run()
    torch.cuda.synchronize()
    for c, ref in zip(batch["cases"], batch["refs"]):
        got = c.result()
        print(c.cfg.name, "misfit", got[0], ref[0], flush=True)
        assert same(got, ref), c.cfg.name


def test_graph_replays_match_eager_runs(batch):
    import torch
    plan, cases, refs = batch["plan"], batch["cases"], batch["refs"]
    for rep in range(3):
        for c in cases:                       # clobber the outputs first
            c.ge.fill_(float("nan"))
            c.mis.fill_(float("nan"))
        plan.run(use_graph=(rep != 1))
        torch.cuda.synchronize()
        x = torch.randn(1000, 1000, device="cuda") @ torch.randn(1000, 1000, device="cuda")
        torch.cuda.synchronize()
        del x
        for c, ref in zip(cases, refs):
            assert same(c.result(), ref), (rep, c.cfg.name)


def test_autotune_does_not_change_results(batch):
    import torch
    plan = make_plan(batch["cases"], autotune=False)
    assert plan.info()["band_rows"] == 0
    plan.run()
    torch.cuda.synchronize()
    for c, ref in zip(batch["cases"], batch["refs"]):
        assert same(c.result(), ref), c.cfg.name
    plan.close()


def test_updated_model_is_used_by_the_next_run(batch):
    import torch
    plan, cases = batch["plan"], batch["cases"]
    c0 = cases[0]
    saved = c0.e0.clone()
    c0.e0.mul_(1.05)
    try:
        ref = c0.single()
        plan.run()
        torch.cuda.synchronize()
        assert same(c0.result(), ref)
    finally:
        c0.e0.copy_(saved)


def _oracle_problem(c, eps, sig):
    cfg = c.cfg
    return oracle.Problem(eps, sig, cfg.npml, cfg.dx, cfg.dy, cfg.dt, cpml_order=cfg.cpml_order,
                          cpml_sigma_scale=cfg.cpml_sigma_scale,
                          cpml_kappa_max=cfg.cpml_kappa_max, cpml_alpha_max=cfg.cpml_alpha_max)


def _against_oracle(plan, c):
    """Run `plan` with case c's observed data replaced by the oracle's
    forward of its true model (restored afterwards), and compare c's misfit
    and gradients with the oracle's gradient for the same data."""
    import torch
    cfg = c.cfg
    w = np_(c.w)
    obs_o, _ = _oracle_problem(c, np_(c.e), np_(c.s)).forward(c.src, c.rec, w, cfg.nt)
    obs_o = obs_o.astype(np.float32)
    J, oge, ogs, _ = _oracle_problem(c, np_(c.e0), np_(c.s0)).gradient(c.src, c.rec, w, obs_o,
                                                                      cfg.nt)
    saved = c.obs.clone()
    try:
        c.obs.copy_(torch.from_numpy(obs_o))
        plan.run()
        torch.cuda.synchronize()
        mis, ge, gs = c.result()
    finally:
        c.obs.copy_(saved)
    errs = (abs(mis - J) / J, rel_l2(ge, oge), rel_l2(gs, ogs))
    print(c.cfg.name, "against the oracle: misfit, grad eps, grad sigma", errs, flush=True)
    assert errs[0] <= 1e-4 and errs[1] <= 1e-3 and errs[2] <= 1e-3


def test_one_batched_problem_against_the_oracle(batch):
    _against_oracle(batch["plan"], batch["cases"][1])


def test_depth8_batch(batch):
    """The same batch at temporal depth 8 (FWI_BATCH_DEPTH8): within FP32
    rounding of the depth-4 single-problem gradients (the imaging sums group
    by 8 steps instead of 4), and one problem against the oracle."""
    import torch
    plan = make_plan(batch["cases"], autotune=fwi.FWI_BATCH_DEPTH8)
    info = plan.info()
    assert info["depth"] == 8 and info["graph"], info
    plan.run()
    torch.cuda.synchronize()
    for c, ref in zip(batch["cases"], batch["refs"]):
        mis, ge, gs = c.result()
        errs = (abs(mis - ref[0]) / ref[0], rel_l2(ge, ref[1]), rel_l2(gs, ref[2]))
        print(c.cfg.name, "depth 8 vs depth 4", errs, flush=True)
        assert errs[0] <= 1e-6 and errs[1] <= 1e-5 and errs[2] <= 1e-5, errs
    _against_oracle(plan, batch["cases"][3])
    plan.close()


def test_autotuner_over_depth_and_bands(batch):
    """The full autotuner times both depths with every band height and runs
    the cheapest; bit for bit the single-problem results at depth 4, within
    rounding at depth 8."""
    import torch
    plan = make_plan(batch["cases"], autotune=True)
    info = plan.info()
    print("autotuned plan", info, flush=True)
    depths = sorted({d for d, _, _ in info["tuning"]})
    assert depths == [4, 8] and len(info["tuning"]) == 14
    best = min(info["tuning"], key=lambda t: t[2])
    assert (info["depth"], info["band_rows"]) == (best[0], best[1])
    plan.run()
    torch.cuda.synchronize()
    for c, ref in zip(batch["cases"], batch["refs"]):
        got = c.result()
        if info["depth"] == 4:
            assert same(got, ref), c.cfg.name
        else:
            assert rel_l2(got[1], ref[1]) <= 1e-5 and rel_l2(got[2], ref[2]) <= 1e-5
    plan.close()
