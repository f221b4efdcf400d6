"""Drive the library's host code through whole calls on the CPU, for the
sanitizer build (run by tests/test_sanitizers.py in a process with the
AddressSanitizer runtime preloaded).  "Device" buffers are host buffers of
exactly the documented sizes (aligned_alloc), so every copy the host code
issues is checked against the real extent of its source and destination.
TEST INFRASTRUCTURE ONLY.

    python host_paths.py LIBRARY
"""
import ctypes
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

from paper_2506_20513_amd import fwi  # noqa: E402
from paper_2506_20513_amd import inputs as I  # noqa: E402

fwi.LIB_PATH = sys.argv[1]
libc = ctypes.CDLL(None)
libc.aligned_alloc.restype = ctypes.c_void_p
libc.aligned_alloc.argtypes = [ctypes.c_size_t, ctypes.c_size_t]
libc.free.argtypes = [ctypes.c_void_p]
held = []


def buf(nbytes):
    """A 256-byte aligned host block of exactly round_up(nbytes, 256) bytes."""
    n = max(256, (int(nbytes) + 255) // 256 * 256)
    p = libc.aligned_alloc(256, n)
    assert p
    ctypes.memset(p, 0, n)
    held.append(p)
    return p


def case(cfg, src, rec):
    S, R, nt = src.shape[0], rec.shape[1], cfg.nt
    w = buf(S * nt * 4)
    geom = fwi.Geometry(src, rec, w)
    grid = fwi.grid_from_config(cfg)
    plane = cfg.NX * cfg.NY * 4
    arrs = dict(eps=buf(plane), sig=buf(plane), ge=buf(plane), gs=buf(plane),
                tr=buf(S * nt * R * 4), obs=buf(S * nt * R * 4), mis=buf(8),
                sadj=buf(S * nt * 4))
    return grid, geom, arrs


def run_single(cfg, src, rec):
    grid, geom, a = case(cfg, src, rec)
    nb = fwi.workspace_bytes(grid, geom, fwi.GRADIENT_WORKSPACE)
    ws = (buf(nb), nb)
    fwi.fwi_gradient(grid, geom, a["eps"], a["sig"], a["obs"], a["mis"], a["ge"], a["gs"],
                     a["tr"], ws, stream=0)
    if nb <= fwi.STATIC_SCRATCH_BYTES:
        fwi.fwi_gradient_static(grid, geom, a["eps"], a["sig"], a["obs"], a["mis"], a["ge"],
                                a["gs"], a["tr"], stream=0)
    t = fwi.fwi_timing(sample_every=3)
    fwi.fwi_gradient_timed(grid, geom, a["eps"], a["sig"], a["obs"], a["mis"], a["ge"],
                           a["gs"], None, ws, t, stream=0)
    assert t.as_dict()["k_adj"]["launches"] > 0
    # shots in concurrent groups: the group layouts inside the same workspace
    for G in (2, 3, 4):
        if G <= src.shape[0]:
            t = fwi.fwi_timing(sample_every=2)
            fwi.fwi_gradient_ex(grid, geom, a["eps"], a["sig"], a["obs"], a["mis"], a["ge"],
                                a["gs"], a["tr"] if G != 3 else None, ws, timing=t,
                                shot_groups=G, stream=0)
            assert t.as_dict()["k_adj"]["launches"] > 0
    for mode in (fwi.FWI_SAVE_NONE, fwi.FWI_SAVE_CHECKPOINT, fwi.FWI_SAVE_HISTORY):
        nb = fwi.workspace_bytes(grid, geom, mode)
        ws = (buf(nb), nb)
        fwi.fdtd_forward(grid, geom, a["eps"], a["sig"], a["tr"], mode, ws, stream=0)
        if mode != fwi.FWI_SAVE_NONE:
            fwi.fdtd_adjoint(grid, geom, a["eps"], a["sig"], a["obs"], a["ge"], a["gs"],
                             a["sadj"], mode, ws, stream=0)


def run_batch(cfgs, geos, autotune):
    probs = []
    for cfg, (src, rec) in zip(cfgs, geos):
        grid, geom, a = case(cfg, src, rec)
        probs.append(fwi.BatchProblem(grid, geom, a["eps"], a["sig"], a["obs"], a["mis"],
                                      a["ge"], a["gs"]))
    nb = fwi.batch_workspace_bytes(probs)
    plan = fwi.BatchPlan(probs, (buf(nb), nb), autotune=autotune, stream=0)
    info = plan.info()
    assert info["nproblems"] == len(cfgs) and not info["graph"], info
    plan.run(stream=0)
    plan.close()


def overflow_check():
    """A workspace half the size the call is told it has: the host code's
    own copies run past the buffer, which the sanitizer must report (this
    shows that the harness would see such a mistake)."""
    cfg = I.config_tiny().with_(nt=20)
    src, rec = I.geometry(cfg)
    grid, geom, a = case(cfg, src, rec)
    nb = fwi.workspace_bytes(grid, geom, fwi.GRADIENT_WORKSPACE)
    fwi.fwi_gradient(grid, geom, a["eps"], a["sig"], a["obs"], a["mis"], a["ge"], a["gs"],
                     a["tr"], (buf(nb // 2), nb), stream=0)
    print("overflow not detected", flush=True)


def main():
    if len(sys.argv) > 2 and sys.argv[2] == "--overflow-check":
        return overflow_check()
    tiny = I.config_tiny().with_(nt=61)
    src, rec = I.geometry(tiny)
    run_single(tiny, src, rec)
    # ragged grid, two shots, duplicate receivers, receivers on many rows in
    # reverse order, a receiver on the source cell, no CPML
    odd = I.RunConfig("odd-37x23", 37, 23, 0, 45, 0.01, 0.01, 1e9, 2, 6)
    s2 = np.array([[5, 4], [30, 17]], np.int32)
    r2 = np.array([[[5, 4], [10, 10], [10, 10], [33, 20], [1, 19], [2, 1]],
                   [[10, 10], [2, 21], [10, 10], [30, 17], [2, 2], [35, 3]]], np.int32)
    run_single(odd, s2, r2)
    # a grid large enough for the depth-8 passes, few steps
    big = I.config_tiny().with_(nx=1004, ny=1004, nt=19)
    sb, rb = I.geometry(big)
    run_single(big, sb, rb)
    # batches of uneven problems, with and without the band autotuner
    cfgs = [I.config_tiny().with_(nt=37), odd.with_(nt=29),
            I.RunConfig("small-90x70", 90, 70, 10, 44, 0.02, 0.02, 2e8, 3, 16)]
    geos = [I.geometry(cfgs[0]), (s2, r2), I.geometry(cfgs[2])]
    run_batch(cfgs, geos, autotune=True)
    run_batch(cfgs, geos, autotune=False)
    run_batch(cfgs, geos, autotune=fwi.FWI_BATCH_DEPTH8)
    for p in held:
        libc.free(p)
    print("host paths ok", flush=True)


if __name__ == "__main__":
    main()
