"""A gradient whose shots run in concurrent groups (fwi_gradient_ex): every
shot's arithmetic, the misfit over all shots and the shot-ordered gradient
sum are those of one group, so the results must agree bit for bit for every
group count, through the automatic choice as well, and the timing must count
the same cell-updates.  The oracle comparisons of the large workload
(test_gpu_fullwindow, test_gpu_parity) run through the automatic two-group
path."""
import numpy as np
import pytest

from paper_2506_20513_amd import fwi
from paper_2506_20513_amd import inputs as I

pytestmark = pytest.mark.gpu


def _problem(cfg):
    import torch
    e, s, e0, s0 = I.model_for(cfg)
    src, rec = I.geometry(cfg)
    w = torch.from_numpy(I.wavelets(cfg)).cuda()
    geom = fwi.Geometry(src, rec, w)
    grid = fwi.grid_from_config(cfg)
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()  # noqa: E731
    obs = torch.empty((cfg.nshots, cfg.nt, cfg.nrec), device="cuda")
    ws = fwi.alloc_workspace(fwi.workspace_bytes(grid, geom, fwi.FWI_SAVE_NONE))
    fwi.fdtd_forward(grid, geom, dev(e), dev(s), obs, fwi.FWI_SAVE_NONE, ws)
    torch.cuda.synchronize()
    return grid, geom, dev(e0), dev(s0), obs


def _run(cfg, grid, geom, e0, s0, obs, ws, groups, timing=None):
    import torch
    mis = torch.empty(1, dtype=torch.float64, device="cuda")
    ge = torch.empty((cfg.NY, cfg.NX), device="cuda")
    gs = torch.empty_like(ge)
    tr = torch.empty((cfg.nshots, cfg.nt, cfg.nrec), device="cuda")
    fwi.fwi_gradient_ex(grid, geom, e0, s0, obs, mis, ge, gs, tr, ws, timing=timing,
                        shot_groups=groups)
    torch.cuda.synchronize()
    return [t.cpu() for t in (mis, ge, gs, tr)]


def _same(a, b):
    import torch
    return all(torch.equal(x, y) for x, y in zip(a, b))


def test_survey_grid_every_group_count_bitwise():
    cfg = I.config_survey().with_(nt=300)
    grid, geom, e0, s0, obs = _problem(cfg)
    ws = fwi.alloc_workspace(fwi.workspace_bytes(grid, geom, fwi.GRADIENT_WORKSPACE))
    ref = _run(cfg, grid, geom, e0, s0, obs, ws, 1)
    assert float(ref[0]) > 0 and float(ref[1].abs().max()) > 0
    for g in (2, 3, 4, 0):
        got = _run(cfg, grid, geom, e0, s0, obs, ws, g)
        print(f"groups {g}: bitwise equal {_same(got, ref)}", flush=True)
        assert _same(got, ref), g
    # the static entry (one group) agrees too
    import torch
    mis = torch.empty(1, dtype=torch.float64, device="cuda")
    ge = torch.empty((cfg.NY, cfg.NX), device="cuda")
    gs = torch.empty_like(ge)
    nb = fwi.workspace_bytes(grid, geom, fwi.GRADIENT_WORKSPACE)
    if nb <= fwi.STATIC_SCRATCH_BYTES:
        fwi.fwi_gradient_static(grid, geom, e0, s0, obs, mis, ge, gs, None)
        torch.cuda.synchronize()
        assert torch.equal(ge.cpu(), ref[1]) and torch.equal(mis.cpu(), ref[0])


def test_large_grid_automatic_groups_bitwise_and_timing():
    """2088 x 1064 cells, 64 shots, a short window: the automatic choice is
    four groups; results as with one group, and the timing of both counts
    the same cell-updates (the four-group call makes four times the
    launches, each over a quarter of the shots)."""
    cfg = I.config_large().with_(nt=48)
    grid, geom, e0, s0, obs = _problem(cfg)
    ws = fwi.alloc_workspace(fwi.workspace_bytes(grid, geom, fwi.GRADIENT_WORKSPACE))
    t1, t0 = fwi.fwi_timing(sample_every=1), fwi.fwi_timing(sample_every=1)
    ref = _run(cfg, grid, geom, e0, s0, obs, ws, 1, t1)
    got = _run(cfg, grid, geom, e0, s0, obs, ws, 0, t0)
    assert _same(got, ref)
    d1, d0 = t1.as_dict(), t0.as_dict()
    assert t1.shot_groups == 1 and t0.shot_groups == 4
    for k in ("k_fwd_sweep", "k_fwd_reforward", "k_adj"):
        assert d0[k]["launches"] == 4 * d1[k]["launches"], (k, d0[k], d1[k])
        assert d0[k]["cell_updates"] == d1[k]["cell_updates"], k
        assert d0[k]["timed"] == d0[k]["launches"] and d0[k]["avg_ms"] > 0, k
    ws2 = fwi.alloc_workspace(fwi.workspace_bytes(grid, geom, fwi.GRADIENT_WORKSPACE))
    assert _same(_run(cfg, grid, geom, e0, s0, obs, ws2, 3), ref)


def test_groups_on_a_side_stream_without_traces_out():
    """The grouped call on a non-default caller stream, with the traces kept
    in the workspace, twice in a row on the same workspace: the same
    results as one group on the default stream."""
    import torch
    cfg = I.config_survey().with_(nt=160)
    grid, geom, e0, s0, obs = _problem(cfg)
    ws = fwi.alloc_workspace(fwi.workspace_bytes(grid, geom, fwi.GRADIENT_WORKSPACE))
    ref = _run(cfg, grid, geom, e0, s0, obs, ws, 1)
    side = torch.cuda.Stream()
    for _ in range(2):
        mis = torch.full((1,), float("nan"), dtype=torch.float64, device="cuda")
        ge = torch.full((cfg.NY, cfg.NX), float("nan"), device="cuda")
        gs = torch.full_like(ge, float("nan"))
        torch.cuda.synchronize()
        with torch.cuda.stream(side):
            fwi.fwi_gradient_ex(grid, geom, e0, s0, obs, mis, ge, gs, None, ws, shot_groups=3,
                                stream=side)
        side.synchronize()
        assert torch.equal(mis.cpu(), ref[0])
        assert torch.equal(ge.cpu(), ref[1]) and torch.equal(gs.cpu(), ref[2])


def test_group_count_checks():
    import torch
    cfg = I.config_tiny().with_(nt=20)
    grid, geom, e0, s0, obs = _problem(cfg)
    ws = fwi.alloc_workspace(fwi.workspace_bytes(grid, geom, fwi.GRADIENT_WORKSPACE))
    mis = torch.empty(1, dtype=torch.float64, device="cuda")
    ge = torch.empty((cfg.NY, cfg.NX), device="cuda")
    gs = torch.empty_like(ge)
    for bad in (-1, 5):
        st = fwi.fwi_gradient_ex(grid, geom, e0, s0, obs, mis, ge, gs, None, ws,
                                 shot_groups=bad, raise_on_error=False)
        assert st == fwi.FWI_EINVAL
    # more groups than shots: as many groups as shots (here one)
    assert fwi.fwi_gradient_ex(grid, geom, e0, s0, obs, mis, ge, gs, None, ws,
                               shot_groups=4, raise_on_error=False) == fwi.FWI_OK
