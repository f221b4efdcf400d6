"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every function include/fwi.h declares, sizes workspaces, and rejects bad
arguments with the documented status before any HIP call.  Every call here
is invalid on purpose or purely host-side (sizes), so nothing reaches the
GPU runtime."""
import ctypes
import math
import os
import re

import numpy as np
import pytest

from paper_2506_20513_amd import fwi
from paper_2506_20513_amd import inputs as I

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fwi.h")
NN_HEADER = os.path.join(ROOT, "include", "fwi_nn.h")

FAKE = 1 << 20        # a non-null, 256-aligned address that is never dereferenced


def header_functions(path=HEADER):
    text = open(path).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(\w+)\s*\(", text, flags=re.M)


@pytest.mark.parametrize("header", ["fwi.h", "fwi_nn.h", "fwi_tv.h"])
def test_library_exports_every_declared_function(header):
    from paper_2506_20513_amd import nn, tv
    names = header_functions(os.path.join(ROOT, "include", header))
    exported = {"fwi.h": fwi.EXPORTED, "fwi_nn.h": nn.EXPORTED, "fwi_tv.h": tv.EXPORTED}[header]
    assert set(names) == set(exported), names
    L = ctypes.CDLL(fwi.LIB_PATH)
    for n in names:
        assert hasattr(L, n), n


def test_strerror_covers_codes():
    for code in (0, -1, -2, -3, -4, -5, -6, -7):
        assert fwi.strerror(code) != "unknown status"
    assert fwi.strerror(-99) == "unknown status"


def _tiny():
    cfg = I.config_tiny()
    src, rec = I.geometry(cfg)
    return cfg, fwi.grid_from_config(cfg), fwi.Geometry(src, rec, FAKE)


def test_workspace_sizes_and_checkpoint_interval():
    cfg, grid, geom = _tiny()
    none = fwi.workspace_bytes(grid, geom, fwi.FWI_SAVE_NONE)
    ck = fwi.workspace_bytes(grid, geom, fwi.FWI_SAVE_CHECKPOINT)
    hist = fwi.workspace_bytes(grid, geom, fwi.FWI_SAVE_HISTORY)
    grad = fwi.workspace_bytes(grid, geom, fwi.GRADIENT_WORKSPACE)
    plane = cfg.NY * (-(-cfg.NX // 64) * 64) * 4
    assert none < ck < hist
    assert hist >= (cfg.nt + 1) * plane
    assert grad >= ck + 2 * cfg.nshots * cfg.nt * cfg.nrec * 4
    K = fwi.checkpoint_interval(grid, geom)
    assert 1 <= K <= cfg.nt
    assert abs(K - math.sqrt(3 * cfg.nt)) < 0.15 * math.sqrt(3 * cfg.nt)
    for v in (none, ck, hist, grad):
        assert v % 256 == 0


def test_workspace_large_config_fits_hbm():
    cfg = I.config_large()
    src, rec = I.geometry(cfg)
    grid = fwi.grid_from_config(cfg)
    geom = fwi.Geometry(src, rec, FAKE)
    grad = fwi.workspace_bytes(grid, geom, fwi.GRADIENT_WORKSPACE)
    assert grad < 200e9, grad / 1e9   # fits in 288 GB with room for the caller


def _status_forward(grid, geom, ws_bytes=None, save=fwi.FWI_SAVE_NONE, ptrs=(FAKE, FAKE, FAKE),
                    ws_addr=FAKE):
    if ws_bytes is None:
        ws_bytes = 0
    return fwi.fdtd_forward(grid, geom, ptrs[0], ptrs[1], ptrs[2], save, (ws_addr, ws_bytes),
                            stream=0, raise_on_error=False)


def test_forward_rejects_small_or_misaligned_workspace():
    _, grid, geom = _tiny()
    need = fwi.workspace_bytes(grid, geom, fwi.FWI_SAVE_NONE)
    assert _status_forward(grid, geom, need - 1) == fwi.FWI_ENOMEM
    assert _status_forward(grid, geom, need, ws_addr=FAKE + 4) == fwi.FWI_ENOMEM
    assert _status_forward(grid, geom, need, ws_addr=0) == fwi.FWI_ENOMEM


def test_forward_rejects_null_pointers_and_bad_mode():
    _, grid, geom = _tiny()
    assert _status_forward(grid, geom, 0, ptrs=(0, FAKE, FAKE)) == fwi.FWI_EINVAL
    assert _status_forward(grid, geom, 0, ptrs=(FAKE, 0, FAKE)) == fwi.FWI_EINVAL
    assert _status_forward(grid, geom, 0, ptrs=(FAKE, FAKE, 0)) == fwi.FWI_EINVAL
    assert _status_forward(grid, geom, 0, save=7) == fwi.FWI_EINVAL
    g2 = fwi.Geometry(geom.src, geom.rec, None)   # NULL wavelet
    assert _status_forward(grid, g2, 0) == fwi.FWI_EINVAL


def test_cfl_bound():
    cfg, grid, geom = _tiny()
    bound = 1.0 / (I.C0 * math.sqrt(1 / cfg.dx ** 2 + 1 / cfg.dy ** 2))
    grid.dt = bound * 1.001
    assert _status_forward(grid, geom) == fwi.FWI_ECFL
    out = ctypes.c_size_t()
    assert fwi.lib().fwi_workspace_bytes(ctypes.byref(grid), ctypes.byref(geom.c), 0,
                                         ctypes.byref(out)) == fwi.FWI_ECFL
    grid.dt = bound          # exactly at the bound is allowed
    assert _status_forward(grid, geom) == fwi.FWI_ENOMEM


@pytest.mark.parametrize("field,value", [("nx", 0), ("ny", -1), ("npml", -1), ("nt", 0),
                                         ("dx", 0.0), ("dy", float("nan")), ("dt", -1e-12),
                                         ("cpml_order", 0), ("cpml_order", 17),
                                         ("cpml_sigma_scale", -1.0), ("cpml_kappa_max", 0.5),
                                         ("cpml_alpha_max", float("inf"))])
def test_grid_parameter_checks(field, value):
    _, grid, geom = _tiny()
    setattr(grid, field, value)
    assert _status_forward(grid, geom) == fwi.FWI_EINVAL


def test_grid_size_limits():
    """Total grid sides 3 .. 2^20 and one shot's plane below 2^30 cells."""
    fake = fwi.Geometry(np.array([[5, 5]]), np.array([[[6, 6]]]), FAKE)
    dt = 1e-12
    # NX = 16384 (pitch 16384), NY = 65536: exactly 2^30 cells is rejected
    g = fwi.make_grid(16384, 65536, 0, 1, 0.01, 0.01, dt)
    assert _status_forward(g, fake) == fwi.FWI_EINVAL
    # one row fewer fits
    g = fwi.make_grid(16384, 65535, 0, 1, 0.01, 0.01, dt)
    out = ctypes.c_size_t()
    assert fwi.lib().fwi_workspace_bytes(ctypes.byref(g), ctypes.byref(fake.c), 0,
                                         ctypes.byref(out)) == fwi.FWI_OK
    # NX = 16321 rounds up to the same pitch
    g = fwi.make_grid(16321, 65536, 0, 1, 0.01, 0.01, dt)
    assert _status_forward(g, fake) == fwi.FWI_EINVAL
    g = fwi.make_grid(1 << 20, 8, 0, 1, 0.01, 0.01, dt)
    assert fwi.lib().fwi_workspace_bytes(ctypes.byref(g), ctypes.byref(fake.c), 0,
                                         ctypes.byref(out)) == fwi.FWI_OK
    g = fwi.make_grid((1 << 20) + 1, 8, 0, 1, 0.01, 0.01, dt)
    assert _status_forward(g, fake) == fwi.FWI_EINVAL
    g = fwi.make_grid(2, 3, 0, 1, 0.01, 0.01, dt)
    assert _status_forward(g, fake) == fwi.FWI_EINVAL


def test_geometry_checks():
    cfg, grid, geom = _tiny()
    p = cfg.npml
    bad_src = geom.src.copy()
    bad_src[0] = (p - 1, p + 1)               # inside the CPML
    assert _status_forward(grid, fwi.Geometry(bad_src, geom.rec, FAKE)) == fwi.FWI_EGEOM
    bad_rec = geom.rec.copy()
    bad_rec[0, 5] = (p + 3, cfg.NY - p)       # below the interior
    assert _status_forward(grid, fwi.Geometry(geom.src, bad_rec, FAKE)) == fwi.FWI_EGEOM
    # npml = 0: the PEC ring is excluded even though it is "interior"
    g0 = fwi.make_grid(20, 20, 0, 10, 0.01, 0.01, 1e-11)
    ring = fwi.Geometry(np.array([[0, 5]]), np.array([[[5, 5]]]), FAKE)
    assert _status_forward(g0, ring) == fwi.FWI_EGEOM
    ok = fwi.Geometry(np.array([[1, 5]]), np.array([[[18, 18]]]), FAKE)
    assert _status_forward(g0, ok) == fwi.FWI_ENOMEM
    # zero receivers / shots
    none = fwi.Geometry(geom.src, np.zeros((1, 0, 2), np.int32), FAKE)
    assert _status_forward(grid, none) == fwi.FWI_EINVAL


def test_adjoint_and_gradient_argument_checks():
    _, grid, geom = _tiny()
    L = fwi.lib()
    ws = (FAKE, 0)
    for mode in (fwi.FWI_SAVE_NONE, 5):
        st = fwi.fdtd_adjoint(grid, geom, FAKE, FAKE, FAKE, FAKE, FAKE, None, mode, ws,
                              stream=0, raise_on_error=False)
        assert st == fwi.FWI_EINVAL
    st = fwi.fdtd_adjoint(grid, geom, FAKE, FAKE, None, FAKE, FAKE, None,
                          fwi.FWI_SAVE_CHECKPOINT, ws, stream=0, raise_on_error=False)
    assert st == fwi.FWI_EINVAL
    st = fwi.fdtd_adjoint(grid, geom, FAKE, FAKE, FAKE, FAKE, FAKE, None,
                          fwi.FWI_SAVE_CHECKPOINT, ws, stream=0, raise_on_error=False)
    assert st == fwi.FWI_ENOMEM
    st = fwi.fwi_gradient(grid, geom, FAKE, FAKE, FAKE, None, FAKE, FAKE, None, ws,
                          stream=0, raise_on_error=False)
    assert st == fwi.FWI_EINVAL
    st = fwi.fwi_gradient(grid, geom, FAKE, FAKE, FAKE, FAKE, FAKE, FAKE, None, ws,
                          stream=0, raise_on_error=False)
    assert st == fwi.FWI_ENOMEM
    assert L.fwi_workspace_bytes(ctypes.byref(grid), ctypes.byref(geom.c), 0, None) == fwi.FWI_EINVAL
    assert L.fwi_workspace_bytes(None, ctypes.byref(geom.c), 0,
                                 ctypes.byref(ctypes.c_size_t())) == fwi.FWI_EINVAL


def _batch_problem(grid, geom, ptr=FAKE):
    return fwi.fwi_batch_problem(grid, geom.c, ptr, ptr, ptr, ptr, ptr, ptr)


def test_batch_argument_checks():
    """Batched plans validate every problem on the host, before any HIP call."""
    _, grid, geom = _tiny()
    L = fwi.lib()
    out = ctypes.c_size_t()
    arr = (fwi.fwi_batch_problem * 2)(_batch_problem(grid, geom), _batch_problem(grid, geom))
    assert L.fwi_batch_workspace_bytes(2, arr, ctypes.byref(out)) == fwi.FWI_OK
    one = (fwi.fwi_batch_problem * 1)(_batch_problem(grid, geom))
    out1 = ctypes.c_size_t()
    assert L.fwi_batch_workspace_bytes(1, one, ctypes.byref(out1)) == fwi.FWI_OK
    assert out.value > out1.value > 0
    assert L.fwi_batch_workspace_bytes(0, arr, ctypes.byref(out)) == fwi.FWI_EINVAL
    assert L.fwi_batch_workspace_bytes(2, arr, None) == fwi.FWI_EINVAL
    bad = (fwi.fwi_batch_problem * 2)(_batch_problem(grid, geom), _batch_problem(grid, geom, 0))
    assert L.fwi_batch_workspace_bytes(2, bad, ctypes.byref(out)) == fwi.FWI_EINVAL
    g2 = fwi_grid_copy(grid)
    g2.dt = grid.dt * 10
    cfl = (fwi.fwi_batch_problem * 2)(_batch_problem(grid, geom), _batch_problem(g2, geom))
    assert L.fwi_batch_workspace_bytes(2, cfl, ctypes.byref(out)) == fwi.FWI_ECFL
    # a workspace that is too small (or missing) is refused before any HIP call
    plan = ctypes.c_void_p()
    assert L.fwi_batch_plan_create(2, arr, FAKE, out.value - 1, 1, None,
                                   ctypes.byref(plan)) == fwi.FWI_ENOMEM
    assert L.fwi_batch_plan_create(2, arr, None, out.value, 1, None,
                                   ctypes.byref(plan)) == fwi.FWI_ENOMEM
    assert not plan.value
    assert L.fwi_batch_plan_run(None, 1, None) == fwi.FWI_EINVAL
    L.fwi_batch_plan_destroy(None)


def fwi_grid_copy(g):
    return fwi.fwi_grid.from_buffer_copy(g)


def test_nn_argument_checks():
    """The CNN entry points reject bad sizes, null pointers and misaligned
    operands with FWI_NN_EINVAL before launching anything."""
    from paper_2506_20513_amd import nn
    L = nn.lib()
    E = -1
    A = FAKE
    # channels must be multiples of 32, operands 16-byte aligned
    assert L.fwi_nn_conv3x3(A, A, None, A, 1, 8, 8, 16, 32, 1, None) == E
    assert L.fwi_nn_conv3x3(A, A, None, A, 1, 8, 8, 32, 48, 1, None) == E
    assert L.fwi_nn_conv3x3(A + 2, A, None, A, 1, 8, 8, 32, 32, 1, None) == E
    assert L.fwi_nn_conv3x3(A, A + 8, None, A, 1, 8, 8, 32, 32, 1, None) == E
    assert L.fwi_nn_conv3x3(None, A, None, A, 1, 8, 8, 32, 32, 1, None) == E
    assert L.fwi_nn_conv3x3(A, A, None, A, 0, 8, 8, 32, 32, 1, None) == E
    assert L.fwi_nn_conv3x3(A, A, None, A, 1 << 16, 1 << 15, 1 << 5, 32, 32, 1, None) == E
    assert L.fwi_nn_wgrad(A + 8, A, A, A, 1, 8, 8, 32, 64, 4, A, 1 << 30, None) == E
    # image sides above 2^15 (the kernels' exact division range)
    assert L.fwi_nn_conv3x3(A, A, None, A, 1, 32769, 1, 32, 32, 1, None) == E
    assert L.fwi_nn_conv3x3(A, A, None, A, 1, 1, 32769, 32, 32, 1, None) == E
    assert L.fwi_nn_wgrad(A, A, A, A, 1, 1, 32769, 32, 64, 4, A, 1 << 30, None) == E
    # several layers' flips: table checks (layers ascending and disjoint)
    I64, I32 = ctypes.c_int64, ctypes.c_int32
    off, ci, co = (I64 * 2)(0, 9 * 32 * 32), (I32 * 2)(32, 32), (I32 * 2)(32, 64)
    assert L.fwi_nn_flip_layers(A, A, 0, off, ci, co, None) == E
    assert L.fwi_nn_flip_layers(A, A, 33, off, ci, co, None) == E
    assert L.fwi_nn_flip_layers(None, A, 2, off, ci, co, None) == E
    assert L.fwi_nn_flip_layers(A, A, 2, None, ci, co, None) == E
    bad = (I64 * 2)(0, 9 * 32 * 32 - 1)
    assert L.fwi_nn_flip_layers(A, A, 2, bad, ci, co, None) == E
    assert L.fwi_nn_flip_layers(A, A, 2, (I64 * 2)(-1, 10000), ci, co, None) == E
    assert L.fwi_nn_flip_layers(A, A, 2, off, ci, (I32 * 2)(32, 0), None) == E
    # weight gradient: workspace size and split count
    need = L.fwi_nn_wgrad_workspace(32, 64, 4)
    assert need == (4 * 64 * 9 * 32 + 4 * 64) * 4
    assert L.fwi_nn_wgrad(A, A, A, A, 1, 8, 8, 32, 64, 4, A, need - 1, None) == E
    assert L.fwi_nn_wgrad(A, A, A, A, 1, 8, 8, 32, 64, 0, A, need, None) == E
    assert L.fwi_nn_wgrad(A, A, A, A, 1, 8, 8, 32, 64, 4, None, need, None) == E
    # pooling needs even sides; upsampling even output sides
    assert L.fwi_nn_pool2(A, A, 1, 7, 8, 32, None) == E
    assert L.fwi_nn_pool2_bwd(A, A, 1, 8, 9, 32, None) == E
    assert L.fwi_nn_up2_add(A, None, A, 1, 8, 5, 32, None) == E
    assert L.fwi_nn_mse(A, A, A, A, A, 10, 32, 33, None) == E
    assert L.fwi_nn_mse(A, A, A, A, A, 0, 32, 2, None) == E
    assert L.fwi_nn_adam(A, A, A, A, None, 10, 1e-3, 0.9, 0.999, 1e-8, 0, None) == E
    assert L.fwi_nn_pack4(A, A, A, 1, 8, 8, 3, None) == E
    assert L.fwi_nn_unpack2(A, A, A, 1, 8, 8, 1, None) == E
    # empty element-wise calls are no-ops
    assert L.fwi_nn_add(A, A, A, 0, None) == 0
    assert L.fwi_nn_relu_bwd(A, A, A, 0, None) == 0


def test_nn_parameter_layout():
    """Every parameter block of the network starts 128-byte aligned in the
    bf16 copy and the blocks tile the flat buffer without overlap."""
    from paper_2506_20513_amd import nn
    end = 0
    for (_, ci, co, _, _), (wo, bo) in zip(nn.LAYERS, nn.param_offsets()):
        assert wo >= end and wo % 64 == 0 and bo % 64 == 0
        assert bo >= wo + co * 9 * ci
        end = bo + co
    assert nn.param_count() >= end
    p = nn.init_params(seed=1, out_scale=0.1)
    assert p.shape == (nn.param_count(),) and np.isfinite(p).all()
    wo, _ = nn.param_offsets()[0]
    w0 = p[wo:wo + 32 * 9 * nn.CPAD].reshape(32, 3, 3, nn.CPAD)
    assert (w0[..., 4:] == 0).all()           # padded input channels carry nothing
    wo, _ = nn.param_offsets()[-1]
    wl = p[wo:wo + 32 * 9 * 32].reshape(32, 3, 3, 32)
    assert (wl[nn.NOUT:] == 0).all() and (wl[:nn.NOUT] != 0).any()
    p0 = nn.init_params(seed=1)               # default: starts as the zero predictor
    assert (p0[wo:wo + 32 * 9 * 32] == 0).all()


def test_tv_argument_checks():
    """fwi_tv_gradient rejects bad shapes and settings (FWI_EINVAL) and a
    missing, misaligned or short workspace (FWI_ENOMEM) before launching."""
    from paper_2506_20513_amd import tv
    L = tv.lib()
    f = lambda *v: (ctypes.c_float * len(v))(*v)
    one = f(1.0, 1.0)
    need = L.fwi_tv_workspace_bytes(2, 16, 24)
    assert need >= 6 * 2 * 16 * 24 * 4
    assert L.fwi_tv_workspace_bytes(0, 16, 24) == 0 and L.fwi_tv_workspace_bytes(5, 16, 24) == 0
    assert L.fwi_tv_workspace_bytes(1, 1, 24) == 0
    A = FAKE
    assert L.fwi_tv_gradient(A, A, 2, 16, 24, one, one, one, 0, A, need, None) == -1
    assert L.fwi_tv_gradient(None, A, 2, 16, 24, one, one, one, 3, A, need, None) == -1
    assert L.fwi_tv_gradient(A, A, 2, 16, 24, f(1.0, 0.0), one, one, 3, A, need, None) == -1
    assert L.fwi_tv_gradient(A, A, 2, 16, 24, one, f(-1.0, 1.0), one, 3, A, need, None) == -1
    assert L.fwi_tv_gradient(A, A, 5, 16, 24, one, one, one, 3, A, need, None) == -1
    assert L.fwi_tv_gradient(A, A, 2, 1, 24, one, one, one, 3, A, need, None) == -1
    assert L.fwi_tv_gradient(A, A, 2, 16, 24, one, one, one, 3, None, need, None) == -4
    assert L.fwi_tv_gradient(A, A, 2, 16, 24, one, one, one, 3, A + 64, need, None) == -4
    assert L.fwi_tv_gradient(A, A, 2, 16, 24, one, one, one, 3, A, need - 1, None) == -4


def test_checkpoint_interval_follows_the_temporal_depth():
    """Grids from 2^20 cells per shot on stream at depth 8, smaller ones at
    depth 4; the checkpoint interval is a multiple of the depth."""
    for cfg, depth in ((I.config_tiny(), 4), (I.config_survey(), 4), (I.config_large(), 8),
                       (I.config_tiny().with_(nx=1004, ny=1004, nt=203), 8)):
        src, rec = I.geometry(cfg)
        g = fwi.Geometry(src, rec, FAKE)
        k = fwi.checkpoint_interval(fwi.grid_from_config(cfg), g)
        assert k % depth == 0 and k <= cfg.nt, (cfg.name, k)


def test_static_gradient_host_checks():
    """fwi_gradient_static checks the problem's workspace against its static
    scratch and its pointers on the host, before any HIP call: the
    benchmark-size problem gets FWI_ESCRATCH, a null output FWI_EINVAL, a
    bad grid the same status as fwi_gradient."""
    cfg = I.config_large()
    src, rec = I.geometry(cfg)
    big = fwi.Geometry(src, rec, FAKE)
    grid = fwi.grid_from_config(cfg)
    assert fwi.workspace_bytes(grid, big, fwi.GRADIENT_WORKSPACE) > fwi.STATIC_SCRATCH_BYTES
    st = fwi.fwi_gradient_static(grid, big, FAKE, FAKE, FAKE, FAKE, FAKE, FAKE, None,
                                 stream=0, raise_on_error=False)
    assert st == fwi.FWI_ESCRATCH
    _, tgrid, tgeom = _tiny()
    assert fwi.workspace_bytes(tgrid, tgeom, fwi.GRADIENT_WORKSPACE) <= fwi.STATIC_SCRATCH_BYTES
    st = fwi.fwi_gradient_static(tgrid, tgeom, FAKE, FAKE, FAKE, None, FAKE, FAKE, None,
                                 stream=0, raise_on_error=False)
    assert st == fwi.FWI_EINVAL
    bad = fwi.grid_from_config(I.config_tiny().with_(nt=0))
    st = fwi.fwi_gradient_static(bad, tgeom, FAKE, FAKE, FAKE, FAKE, FAKE, FAKE, None,
                                 stream=0, raise_on_error=False)
    assert st == fwi.FWI_EINVAL
