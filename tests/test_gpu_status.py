"""End-of-call finiteness status (FWI_ENONFINITE) through the C ABI: a NaN
or an infinity in the observed data or the model reaches the misfit,
gradients or traces, and the call reports it after writing its outputs;
clean inputs give FWI_OK.  Nothing here makes a kernel misbehave: NaN and
infinity are ordinary float inputs that the arithmetic carries along."""
import numpy as np
import pytest

from paper_2506_20513_amd import fwi
from paper_2506_20513_amd import inputs as I

pytestmark = pytest.mark.gpu


def _setup(nt=200):
    import torch
    cfg = I.config_tiny().with_(nt=nt)
    e, s, e0, s0 = I.model_for(cfg)
    src, rec = I.geometry(cfg)
    w = torch.from_numpy(I.wavelets(cfg)).cuda()
    geom = fwi.Geometry(src, rec, w)
    grid = fwi.grid_from_config(cfg)
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()  # noqa: E731
    obs = torch.zeros((cfg.nshots, cfg.nt, cfg.nrec), device="cuda")
    return cfg, grid, geom, w, dev(e0), dev(s0), obs


def _outs(cfg):
    import torch
    return (torch.empty(1, dtype=torch.float64, device="cuda"),
            torch.empty((cfg.NY, cfg.NX), device="cuda"),
            torch.empty((cfg.NY, cfg.NX), device="cuda"))


def test_gradient_reports_nonfinite_observed_data():
    import torch
    cfg, grid, geom, w, e0, s0, obs = _setup()
    ws = fwi.alloc_workspace(fwi.workspace_bytes(grid, geom, fwi.GRADIENT_WORKSPACE))
    mis, ge, gs = _outs(cfg)
    assert fwi.fwi_gradient(grid, geom, e0, s0, obs, mis, ge, gs, None, ws,
                            raise_on_error=False) == fwi.FWI_OK
    assert torch.isfinite(ge).all() and torch.isfinite(mis).all()
    for bad in (float("nan"), float("inf")):
        o = obs.clone()
        o[0, cfg.nt // 2, 3] = bad
        st = fwi.fwi_gradient(grid, geom, e0, s0, o, mis, ge, gs, None, ws,
                              raise_on_error=False)
        assert st == fwi.FWI_ENONFINITE, (bad, st)
        assert not torch.isfinite(mis).all()
        st = fwi.fwi_gradient_static(grid, geom, e0, s0, o, mis, ge, gs, None,
                                     raise_on_error=False)
        assert st == fwi.FWI_ENONFINITE, (bad, st)
    # a clean call on the same workspace afterwards is clean again
    assert fwi.fwi_gradient(grid, geom, e0, s0, obs, mis, ge, gs, None, ws,
                            raise_on_error=False) == fwi.FWI_OK
    with pytest.raises(fwi.FwiError) as err:
        o = obs.clone()
        o[0, 5, 0] = float("nan")
        fwi.fwi_gradient(grid, geom, e0, s0, o, mis, ge, gs, None, ws)
    assert err.value.status == fwi.FWI_ENONFINITE


def test_forward_and_adjoint_report_nonfinite_values():
    import torch
    cfg, grid, geom, w, e0, s0, obs = _setup()
    ws = fwi.alloc_workspace(fwi.workspace_bytes(grid, geom, fwi.FWI_SAVE_CHECKPOINT))
    tr = torch.empty((cfg.nshots, cfg.nt, cfg.nrec), device="cuda")
    mis, ge, gs = _outs(cfg)
    assert fwi.fdtd_forward(grid, geom, e0, s0, tr, fwi.FWI_SAVE_CHECKPOINT, ws,
                            raise_on_error=False) == fwi.FWI_OK
    res = tr.clone()
    assert fwi.fdtd_adjoint(grid, geom, e0, s0, res, ge, gs, None, fwi.FWI_SAVE_CHECKPOINT,
                            ws, raise_on_error=False) == fwi.FWI_OK
    res[0, 10, 0] = float("nan")
    assert fwi.fdtd_adjoint(grid, geom, e0, s0, res, ge, gs, None, fwi.FWI_SAVE_CHECKPOINT,
                            ws, raise_on_error=False) == fwi.FWI_ENONFINITE
    # a NaN permittivity next to the source reaches the receivers
    e_bad = e0.clone()
    si, sj = int(geom.src[0, 0]), int(geom.src[0, 1])
    e_bad[sj + 1, si] = float("nan")
    assert fwi.fdtd_forward(grid, geom, e_bad, s0, tr, fwi.FWI_SAVE_CHECKPOINT, ws,
                            raise_on_error=False) == fwi.FWI_ENONFINITE
    assert not torch.isfinite(tr).all()
