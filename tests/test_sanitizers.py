"""AddressSanitizer and UndefinedBehaviorSanitizer builds of the CPU-side
code, run on the CPU:

* the FP64 oracle (oracle/fdtd_oracle.c), under a set of its pins;
* the library's host code (fwi_host.cpp, fwi_batch.cpp, fwi_static.hip:
  validation, workspace layout, geometry sorting, the pass loops and
  checkpoint copies, the batch schedule builder and its autotuner loop),
  built with g++ against a host-only stand-in for the HIP runtime
  (tests/host_asan) and driven through whole calls with "device" buffers of
  exactly their documented sizes, plus the host-side ABI checks.

Each run happens in a child process with the AddressSanitizer runtime
preloaded; any report fails the test.  One run gives the call a workspace
half the size it is told, to show that the harness sees an overrun."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2506_20513_amd", "csrc")
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
       "-fno-omit-frame-pointer", "-g", "-O1"]
REPORT = ("ERROR: AddressSanitizer", "runtime error:", "ERROR: LeakSanitizer")


def _asan_runtime():
    try:
        p = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True,
                           text=True, check=True).stdout.strip()
    except (OSError, subprocess.CalledProcessError):
        return None
    return p if os.path.isabs(p) and os.path.exists(p) else None


ASAN = _asan_runtime()
pytestmark = pytest.mark.skipif(ASAN is None, reason="gcc's AddressSanitizer runtime not found")


def _run(args, timeout=600):
    env = dict(os.environ, LD_PRELOAD=ASAN, ASAN_OPTIONS="detect_leaks=0",
               UBSAN_OPTIONS="print_stacktrace=1", OMP_NUM_THREADS="4")
    return subprocess.run([sys.executable, *args], cwd=ROOT, env=env, capture_output=True,
                          text=True, timeout=timeout)


def _clean(p):
    out = p.stdout + p.stderr
    assert p.returncode == 0 and not any(r in out for r in REPORT), out[-4000:]
    return out


@pytest.fixture(scope="module")
def host_lib(tmp_path_factory):
    so = str(tmp_path_factory.mktemp("asan") / "libfwi_host_asan.so")
    cmd = ["g++", "-std=c++17", "-fPIC", "-shared", "-pthread", "-Wall", "-Wno-unused-function", *SAN,
           "-I", os.path.join(ROOT, "tests", "host_asan"), "-I", os.path.join(ROOT, "include"),
           "-I", CSRC, os.path.join(ROOT, "tests", "host_asan", "hip_host_stub.cpp"),
           os.path.join(CSRC, "fwi_host.cpp"), os.path.join(CSRC, "fwi_batch.cpp"),
           "-x", "c++", os.path.join(CSRC, "fwi_static.hip"), "-o", so]
    subprocess.run(cmd, check=True)
    return so


def test_host_code_whole_calls_under_sanitizers(host_lib):
    out = _clean(_run([os.path.join("tests", "host_asan", "host_paths.py"), host_lib]))
    assert "host paths ok" in out


def test_sanitizer_sees_a_workspace_overrun(host_lib):
    p = _run([os.path.join("tests", "host_asan", "host_paths.py"), host_lib, "--overflow-check"])
    assert p.returncode != 0 and "heap-buffer-overflow" in p.stderr, p.stderr[-2000:]


def test_host_abi_checks_under_sanitizers(host_lib):
    code = ("import sys; sys.path.insert(0, {root!r}); "
            "from paper_2506_20513_amd import fwi; fwi.LIB_PATH = {so!r}; import pytest; "
            "sys.exit(pytest.main(['-q', '-p', 'no:cacheprovider', 'tests/test_abi_host.py', "
            "'-k', 'not nn and not tv and not exports']))").format(root=ROOT, so=host_lib)
    out = _clean(_run(["-c", code]))
    assert " passed" in out


def test_oracle_pins_under_sanitizers(tmp_path):
    import oracle
    src = os.path.join(ROOT, "oracle", "fdtd_oracle.c")
    so = str(tmp_path / "liboracle_asan.so")
    subprocess.run(["gcc", "-fopenmp", "-fPIC", "-shared", "-std=c99", *SAN, "-o", so, src, "-lm"],
                   check=True)
    assert os.path.exists(oracle.build(force=False))
    code = f"""
import sys
sys.path.insert(0, {ROOT!r})
import numpy as np
import oracle
from tests import oracle_pins as pins
with oracle.use_library({so!r}):
    for name, (v, bound) in [("energy", pins.pec_energy_drift(300, dy_ratio=0.73)),
                             ("decay", pins.lossy_decay()),
                             ("dot", pins.dot_product(0.73)),
                             ("fd", pins.fd_gradient(0.73)),
                             ("transpose", pins.transpose_symmetry()),
                             ("pec", pins.pec_material_box()),
                             ("reciprocity", pins.reciprocity(8))]:
        assert v <= bound, (name, v, bound)
    c = pins.fd_setup()
    P = oracle.Problem(c["eps0"], c["sig0"], c["npml"], c["dx"], c["dy"], c["dt"], **c["kw"])
    a = P.gradient(c["src"], c["rec"], c["w"], c["obs"], c["nt"])
    b = P.gradient_checkpointed(c["src"], c["rec"], c["w"], c["obs"], c["nt"], 37)
    assert all(np.array_equal(x, y) for x, y in zip(a[1:], b[1:]))
print("oracle pins ok")
"""
    out = _clean(_run(["-c", code]))
    assert "oracle pins ok" in out
