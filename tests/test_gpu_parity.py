"""GPU (HIP, gfx950) against the FP64 oracle, element by element, through
the C ABI.  Tolerances: relative L2 1e-4 on receiver traces and 1e-3 on the
eps_r / sigma gradients (also with a 3-cell radius around sources and
receivers masked, where near-field cells dominate the norm).  The oracle
consumes the same FP32-rounded model, wavelet and observed data, promoted to
double, so input rounding is not counted as error."""
import numpy as np
import pytest

import oracle
from paper_2506_20513_amd import fwi
from paper_2506_20513_amd import inputs as I
from tests.gpu_util import (Run, gradient_regions, late_window, mask_near, np_,
                            region_errors, rel_l2)

pytestmark = pytest.mark.gpu

TR_TOL = 1e-4
GR_TOL = 1e-3


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU visible")
    fwi.lib()   # raises if the HIP library is missing: no fallback


def oracle_problem(cfg, eps, sig):
    return oracle.Problem(eps, sig, cfg.npml, cfg.dx, cfg.dy, cfg.dt,
                          cpml_order=cfg.cpml_order, cpml_sigma_scale=cfg.cpml_sigma_scale,
                          cpml_kappa_max=cfg.cpml_kappa_max, cpml_alpha_max=cfg.cpml_alpha_max)


def make_case(cfg, seed=None):
    e, s, e0, s0 = I.model_for(cfg, seed)
    src, rec = I.geometry(cfg)
    w = I.wavelets(cfg)
    obs, _ = oracle_problem(cfg, e, s).forward(src, rec, w, cfg.nt)
    return dict(cfg=cfg, e=e, s=s, e0=e0, s0=s0, src=src, rec=rec, w=w,
                obs=obs.astype(np.float32))


@pytest.fixture(scope="module")
def tiny():
    c = make_case(I.config_tiny())
    P = oracle_problem(c["cfg"], c["e0"], c["s0"])
    J, ge, gs, tr = P.gradient(c["src"], c["rec"], c["w"], c["obs"], c["cfg"].nt)
    c.update(J=J, ge=ge, gs=gs, tr=tr)
    return c


def run_of(c, model="init"):
    cfg = c["cfg"]
    e, s = (c["e0"], c["s0"]) if model == "init" else (c["e"], c["s"])
    return Run(fwi.grid_from_config(cfg), c["src"], c["rec"], c["w"], e, s)


def check_gradients(ge, gs, oge, ogs, src, rec):
    m = mask_near(oge.shape, src, rec)
    errs = dict(eps=rel_l2(ge, oge), sig=rel_l2(gs, ogs),
                eps_masked=rel_l2(ge[m], oge[m]), sig_masked=rel_l2(gs[m], ogs[m]))
    print("gradient rel L2:", errs, flush=True)
    for k, v in errs.items():
        assert v <= GR_TOL, (k, v)


def test_tiny_forward_traces(tiny):
    r = run_of(tiny, "true")
    tr, _ = r.forward()
    err = rel_l2(np_(tr), tiny["obs"])
    print("traces rel L2", err, flush=True)
    assert err <= TR_TOL


def test_tiny_gradient(tiny):
    r = run_of(tiny)
    mis, ge, gs, tr = r.gradient(tiny["obs"])
    assert rel_l2(np_(tr), tiny["tr"]) <= TR_TOL
    assert abs(float(mis.item()) - tiny["J"]) <= 1e-4 * tiny["J"]
    check_gradients(np_(ge), np_(gs), tiny["ge"], tiny["gs"], tiny["src"], tiny["rec"])


def test_checkpoint_and_history_agree_bitwise(tiny):
    """Re-forward from checkpoints reproduces the stored history exactly."""
    r = run_of(tiny)
    out = {}
    for mode in (fwi.FWI_SAVE_HISTORY, fwi.FWI_SAVE_CHECKPOINT):
        tr, ws = r.forward(mode)
        res = tr - r.torch.from_numpy(tiny["obs"]).to(r.dev)
        ge, gs, sa = r.adjoint(res, mode, ws, want_src_adjoint=True)
        out[mode] = (np_(tr), np_(ge), np_(gs), np_(sa))
    for a, b in zip(out[fwi.FWI_SAVE_HISTORY], out[fwi.FWI_SAVE_CHECKPOINT]):
        assert np.array_equal(a, b)


@pytest.mark.parametrize("nt", [403, 258])
def test_checkpoint_and_history_agree_bitwise_ragged_nt(nt):
    """nt not a multiple of the streaming depth: every adjoint pass starts at
    a multiple of the depth whatever the checkpoint interval, so the imaging
    sums group the same way and the results still agree bit for bit."""
    c = make_case(I.config_tiny().with_(nt=nt))
    r = run_of(c)
    out = {}
    for mode in (fwi.FWI_SAVE_HISTORY, fwi.FWI_SAVE_CHECKPOINT):
        tr, ws = r.forward(mode)
        res = tr - r.torch.from_numpy(c["obs"]).to(r.dev)
        ge, gs, sa = r.adjoint(res, mode, ws, want_src_adjoint=True)
        out[mode] = (np_(tr), np_(ge), np_(gs), np_(sa))
    print("checkpoint interval", fwi.checkpoint_interval(r.grid, r.geom), flush=True)
    for a, b in zip(out[fwi.FWI_SAVE_HISTORY], out[fwi.FWI_SAVE_CHECKPOINT]):
        assert np.array_equal(a, b)


def test_checkpoint_and_history_agree_bitwise_depth8():
    """The same on a grid of 2^20 cells (1024 x 1024 total), which runs its
    streaming passes at temporal depth 8; nt = 203 is ragged against both
    the depth and the checkpoint interval."""
    c = make_case(I.config_tiny().with_(nx=1004, ny=1004, nt=203))
    r = run_of(c)
    k = fwi.checkpoint_interval(r.grid, r.geom)
    print("checkpoint interval", k, flush=True)
    assert k % 8 == 0
    out = {}
    for mode in (fwi.FWI_SAVE_HISTORY, fwi.FWI_SAVE_CHECKPOINT):
        tr, ws = r.forward(mode)
        res = tr - r.torch.from_numpy(c["obs"]).to(r.dev)
        ge, gs, sa = r.adjoint(res, mode, ws, want_src_adjoint=True)
        out[mode] = (np_(tr), np_(ge), np_(gs), np_(sa))
        del ws
    for a, b in zip(out[fwi.FWI_SAVE_HISTORY], out[fwi.FWI_SAVE_CHECKPOINT]):
        assert np.array_equal(a, b)
    # and the traces against the oracle at this size
    rt = run_of(c, "true")
    tr, _ = rt.forward()
    err = rel_l2(np_(tr), c["obs"])
    print("depth-8 traces rel L2", err, flush=True)
    assert err <= TR_TOL


def test_gradient_entry_point_matches_forward_adjoint(tiny):
    r = run_of(tiny)
    mis, ge, gs, tr = r.gradient(tiny["obs"])
    tr2, ws = r.forward(fwi.FWI_SAVE_CHECKPOINT)
    res = tr2 - r.torch.from_numpy(tiny["obs"]).to(r.dev)
    ge2, gs2, _ = r.adjoint(res, fwi.FWI_SAVE_CHECKPOINT, ws)
    assert np.array_equal(np_(tr), np_(tr2))
    assert np.array_equal(np_(ge), np_(ge2)) and np.array_equal(np_(gs), np_(gs2))


def test_deterministic_run_to_run(tiny):
    r = run_of(tiny)
    a = [np_(x) for x in r.gradient(tiny["obs"])]
    b = [np_(x) for x in r.gradient(tiny["obs"])]
    for x, y in zip(a, b):
        assert np.array_equal(x, y)


def test_dot_product_fp32():
    """<A w, r> = <w, A^T r> for the wavelet-to-trace map on the GPU."""
    cfg = I.config_tiny().with_(nt=400, nshots=2)
    e, s, _, _ = I.model_for(cfg)
    src, rec = I.geometry(cfg.with_(nshots=1))
    src = np.concatenate([src, src + np.array([[30, 10]], np.int32)])
    rec = np.concatenate([rec, rec[:, ::-1]])
    rng = np.random.default_rng(3)
    w = rng.standard_normal((2, cfg.nt)).astype(np.float32)
    r = rng.standard_normal((2, cfg.nt, cfg.nrec)).astype(np.float32)
    run = Run(fwi.grid_from_config(cfg), src, rec, w, e, s)
    tr, ws = run.forward(fwi.FWI_SAVE_HISTORY)
    _, _, sa = run.adjoint(r, fwi.FWI_SAVE_HISTORY, ws, want_src_adjoint=True)
    lhs = float(np.sum(np_(tr).astype(np.float64) * r))
    rhs = float(np.sum(w.astype(np.float64) * np_(sa)))
    print("dot product", lhs, rhs, flush=True)
    assert abs(lhs - rhs) <= 1e-5 * abs(lhs)


@pytest.mark.parametrize("cfg", I.config_paper_shapes(), ids=lambda c: c.name)
def test_paper_shapes(cfg):
    """Grid shapes of the paper's experiments (none a multiple of 64)."""
    c = make_case(cfg)
    P = oracle_problem(cfg, c["e0"], c["s0"])
    J, oge, ogs, otr = P.gradient(c["src"], c["rec"], c["w"], c["obs"], cfg.nt)
    mis, ge, gs, tr = run_of(c).gradient(c["obs"])
    assert rel_l2(np_(tr), otr) <= TR_TOL
    check_gradients(np_(ge), np_(gs), oge, ogs, c["src"], c["rec"])


def test_pec_box_duplicate_receivers_and_source_at_receiver():
    """npml = 0 (pure PEC box), receivers sharing cells, a receiver on the
    source cell, ragged tiles (NX = 37, NY = 23)."""
    cfg = I.RunConfig("edge-35x21", 35, 21, 0, 120, 0.01, 0.01, 1e9, 2, 5)
    rng = np.random.default_rng(8)
    e = (1 + 9 * rng.random((cfg.NY, cfg.NX))).astype(np.float32)
    s = (0.03 * rng.random((cfg.NY, cfg.NX))).astype(np.float32)
    e_t = (e * (1 + 0.1 * rng.random(e.shape))).astype(np.float32)
    src = np.array([[5, 4], [30, 17]], np.int32)
    rec = np.array([[[5, 4], [10, 10], [10, 10], [33, 1], [1, 19]],
                    [[10, 10], [10, 10], [10, 10], [30, 17], [2, 2]]], np.int32)
    w = I.wavelets(cfg)
    obs, _ = oracle_problem(cfg, e_t, s).forward(src, rec, w, cfg.nt)
    obs = obs.astype(np.float32)
    J, oge, ogs, otr = oracle_problem(cfg, e, s).gradient(src, rec, w, obs, cfg.nt)
    mis, ge, gs, tr = Run(fwi.grid_from_config(cfg), src, rec, w, e, s).gradient(obs)
    assert rel_l2(np_(tr), otr) <= TR_TOL
    assert rel_l2(np_(ge), oge) <= GR_TOL and rel_l2(np_(gs), ogs) <= GR_TOL


@pytest.mark.parametrize("nt", [1, 2, 5])
def test_few_steps(nt):
    """nt = 1: traces are all zero (Ez^0 = 0) and so is the gradient."""
    cfg = I.config_tiny().with_(nt=nt)
    c = make_case(cfg)
    c["obs"] = c["obs"] + np.float32(1.0)
    J, oge, ogs, otr = oracle_problem(cfg, c["e0"], c["s0"]).gradient(
        c["src"], c["rec"], c["w"], c["obs"], nt)
    mis, ge, gs, tr = run_of(c).gradient(c["obs"])
    assert np.allclose(np_(tr), otr, rtol=1e-4, atol=1e-6 * (np.abs(otr).max() + 1e-30))
    if nt == 1:
        assert np.all(np_(ge) == 0) and np.all(np_(gs) == 0)
    else:
        assert rel_l2(np_(ge), oge) <= GR_TOL and rel_l2(np_(gs), ogs) <= GR_TOL
    assert abs(float(mis.item()) - J) <= 1e-5 * J


def test_survey_sampled_shots():
    """512x256 / 24 shots / 3000 steps, all shots batched in one sweep on the
    GPU; the oracle recomputes shots 0 and 23 one by one for the traces, and
    the gradient of shot 0 alone (observed data: the oracle's shot-0 traces)."""
    cfg = I.config_survey()
    e, s, e0, s0 = I.model_for(cfg)
    src, rec = I.geometry(cfg)
    w = I.wavelets(cfg)
    run = Run(fwi.grid_from_config(cfg), src, rec, w, e, s)
    tr, _ = run.forward()
    tr = np_(tr)
    P = oracle_problem(cfg, e, s)
    otr0 = None
    for k in (0, cfg.nshots - 1):
        otr, _ = P.forward(src[k:k + 1], rec[k:k + 1], w[k:k + 1], cfg.nt)
        err = rel_l2(tr[k], otr[0])
        print("shot", k, "traces rel L2", err, flush=True)
        assert err <= TR_TOL
        if k == 0:
            otr0 = otr
    # gradient of shot 0 on the smoothed model, against the oracle's own
    # traces of the true model as observed data
    obs0 = otr0.astype(np.float32)
    P0 = oracle_problem(cfg, e0, s0)
    J, oge, ogs, _ = P0.gradient(src[:1], rec[:1], w[:1], obs0, cfg.nt)
    mis, ge, gs, _ = Run(fwi.grid_from_config(cfg), src[:1], rec[:1], w[:1], e0, s0).gradient(obs0)
    check_gradients(np_(ge), np_(gs), oge, ogs, src[:1], rec[:1])


def _conductor_case(nx, ny, npml, nt, dx, dy, f0, seed, span=None):
    """Anisotropic cells (dy != dx), a lossy layered model, and perfect
    conductors (sigma = 1e3 S/m > 100, Sec. 3.2): a hollow ring and a solid
    disc.  Two shots at different depths, receivers on a surface line and a
    vertical line (so traces see both axes).  Everything sits in the
    top-left span x span cells of the interior (the whole interior by
    default), so that a short window still reaches it on a large grid."""
    cfg = I.RunConfig(f"aniso-{nx}x{ny}", nx, ny, npml, nt, dx, dy, f0, 2, 24)
    _, _, e0, s0 = I.model_for(cfg, seed)
    NY, NX = cfg.NY, cfg.NX
    sx, sy = (nx, ny) if span is None else (min(span, nx), min(span, ny))
    jj, ii = np.mgrid[0:NY, 0:NX]
    # the true model: the smooth start plus two anomalies inside the span,
    # and a shallow layer 10% faster, so that the residual is a sizeable part
    # of the traces from the direct wave on (a residual that is a tiny
    # difference of two nearly equal FP32 traces would be known to the GPU
    # only to its rounding)
    e, s = e0.copy(), s0.copy()
    e[:npml + max(4, sy // 12)] *= np.float32(1.0 / 1.1)
    for fi, fj, rad, de, ds in ((0.45, 0.5, 0.12, 0.35, 0.01), (0.8, 0.25, 0.08, -0.25, 0.02)):
        m = (ii - npml - fi * sx) ** 2 + (jj - npml - fj * sy) ** 2 <= (rad * min(sx, sy)) ** 2
        e[m] *= 1.0 + de
        s[m] += ds
    pec = np.zeros((NY, NX), bool)
    ci, cj = npml + int(0.7 * sx), npml + int(0.6 * sy)
    r2 = (ii - ci) ** 2 + (jj - cj) ** 2
    pec |= (r2 <= 12 ** 2) & (r2 >= 9 ** 2)                        # hollow ring
    pec |= (ii - (npml + sx // 4)) ** 2 + (jj - (npml + 2 * sy // 3)) ** 2 <= 5 ** 2
    for a in (s, s0):
        a[pec] = 1.0e3
    src = np.array([[npml + sx // 3, npml + 2], [npml + sx // 2, npml + sy // 3]], np.int32)
    rec = np.zeros((2, 24, 2), np.int32)
    for k in range(2):
        rec[k, :12] = [[npml + 3 + r * (sx - 6) // 11, npml + 3] for r in range(12)]
        rec[k, 12:] = [[npml + sx - 4, npml + 3 + r * (sy - 6) // 11] for r in range(12)]
    w = I.wavelets(cfg)
    obs, _ = oracle_problem(cfg, e, s).forward(src, rec, w, nt)
    return cfg, e0, s0, pec, src, rec, w, obs.astype(np.float32)


@pytest.mark.parametrize("shape", [(150, 90, 10, 1000, 250e6, None),
                                   (1080, 960, 12, 800, 500e6, 120)],
                         ids=["depth4-170x110", "depth8-1104x984"])
def test_anisotropic_cells_with_conductor_inclusions(shape):
    """dx != dy on the GPU against the oracle, with sigma > 100 S/m cells:
    traces (all, and the late third of the window), misfit, gradients on the
    whole grid and per region (each CPML strip, the deep half, the interior
    away from sources and receivers), and exact zeros of the gradient in the
    conductor cells.  The larger grid has 2^20 cells and more, so its
    streaming passes run at temporal depth 8; its sources, receivers and
    conductors sit near the top-left corner, where the short window reaches
    (regions the waves never reach are zero on both sides).  The Ricker
    frequencies keep at least 25 cells per wavelength at f0 in the slowest
    layer, as the workloads do: on grids with only a few cells per
    wavelength the zero-lag sums cancel so strongly that their FP32
    accumulation alone reaches 1e-4 to 1e-3 of the gradient."""
    nx, ny, npml, nt, f0, span = shape
    cfg, e0, s0, pec, src, rec, w, obs = _conductor_case(nx, ny, npml, nt, 0.01, 0.0073,
                                                          f0, 17, span)
    P = oracle_problem(cfg, e0, s0)
    J, oge, ogs, otr = P.gradient_checkpointed(src, rec, w, obs, nt)
    mis, ge, gs, tr = Run(fwi.grid_from_config(cfg), src, rec, w, e0, s0).gradient(obs)
    tr, ge, gs = np_(tr), np_(ge), np_(gs)
    errs = {"traces": rel_l2(tr, otr), "late_traces": rel_l2(late_window(tr), late_window(otr)),
            "misfit": abs(float(mis.item()) - J) / J}
    print("aniso traces/misfit", errs, flush=True)
    assert errs["traces"] <= TR_TOL and errs["late_traces"] <= TR_TOL
    assert errs["misfit"] <= 1e-4
    check_gradients(ge, gs, oge, ogs, src, rec)
    regions = gradient_regions(ge.shape, cfg.npml, src, rec)
    for name, g, og in (("eps", ge, oge), ("sig", gs, ogs)):
        re = region_errors(g, og, regions)
        print("aniso", name, "regions", re, flush=True)
        for k, v in re.items():
            assert v <= GR_TOL, (name, k, v)
    assert np.all(ge[pec] == 0) and np.all(gs[pec] == 0)
    assert np.all(oge[pec] == 0) and np.all(ogs[pec] == 0)
