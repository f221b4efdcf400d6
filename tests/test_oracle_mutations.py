"""Plant plausible mistakes in copies of the oracle (on the CPU) and check
that at least one pin catches each.  This is what makes the pins a real
check: a dropped term, a wrong sign or index, or a transposed operand in the
forward or adjoint recursion must fail one of them."""
import os

import pytest

import oracle
from tests import oracle_pins as pins

SRC = os.path.join(os.path.dirname(oracle.__file__), "fdtd_oracle.c")

# (name, exact text in the source, replacement, pins expected to catch it)
MUTATIONS = [
    ("H-sign", "Hy[k] += ch * (de", "Hy[k] -= ch * (de", ["energy", "hankel"]),
    ("E-index", "(Hy[k] - Hy[k - 1]) / p->dx", "(Hy[k + 1] - Hy[k]) / p->dx", ["energy", "hankel"]),
    ("source-sign", "E[k] -= p->Cs[k] * w[n]", "E[k] += p->Cs[k] * w[n]", ["hankel"]),
    ("source-scale", "w[n] / (p->dx * p->dy)", "w[n] / p->dx", ["hankel"]),
    ("explicit-loss", "Ca[k] = EB / EA;", "Ca[k] = 1.0 - sigma[k] * dt / (ORC_EPS0 * eps_r[k]);", ["decay"]),
    ("drop-cpml-memory", "psi_ex[k] = p->bEx[i] * psi_ex[k] + p->aEx[i] * ddx;",
     "psi_ex[k] = 0.0 * ddx;", ["cpml"]),
    ("adjoint-transposed-diff", "double ax = tmpx[k] - (i + 1 < NX ? tmpx[k + 1] : 0.0);",
     "double ax = tmpx[k] - (i >= 1 ? tmpx[k - 1] : 0.0);", ["dot"]),
    ("adjoint-drop-Ca", "lE[k] = p->Ca[k] * lE[k];", "lE[k] = lE[k];", ["dot"]),
    ("adjoint-psi-sign", "double t = phi_hy[k] + h;", "double t = phi_hy[k] - h;", ["dot"]),
    ("imaging-sign", "S1[k] += lE[k] * (En1[k] - En[k]);", "S1[k] += lE[k] * (En[k] - En1[k]);", ["fd"]),
    ("imaging-lag", "S2[k] += lE[k] * (En1[k] + En[k]);", "S2[k] += lE[k] * (En1[k] + En1[k]);", ["fd"]),
    # each spacing swapped for the other axis' one, forward and adjoint
    ("Hx-diff-dx", "double de = (E[k + NX] - E[k]) / p->dy;", "double de = (E[k + NX] - E[k]) / p->dx;",
     ["energy-aniso", "hankel-aniso", "transpose"]),
    ("Hy-diff-dy", "double de = (E[k + 1] - E[k]) / p->dx;", "double de = (E[k + 1] - E[k]) / p->dy;",
     ["energy-aniso", "hankel-aniso", "transpose"]),
    ("E-ddx-dy", "double ddx = (Hy[k] - Hy[k - 1]) / p->dx;", "double ddx = (Hy[k] - Hy[k - 1]) / p->dy;",
     ["energy-aniso", "hankel-aniso", "transpose"]),
    ("E-ddy-dx", "double ddy = (Hx[k] - Hx[k - NX]) / p->dy;", "double ddy = (Hx[k] - Hx[k - NX]) / p->dx;",
     ["energy-aniso", "hankel-aniso", "transpose"]),
    ("adj-lHy-dy", "lHy[k] += ax / p->dx;", "lHy[k] += ax / p->dy;", ["dot-aniso", "transpose"]),
    ("adj-lHx-dx", "lHx[k] += ay / p->dy;", "lHx[k] += ay / p->dx;", ["dot-aniso", "transpose"]),
    ("adj-lE-x-dy", "lE[k] += (tmpx[k - 1] - tmpx[k]) / p->dx +", "lE[k] += (tmpx[k - 1] - tmpx[k]) / p->dy +",
     ["dot-aniso", "transpose"]),
    ("adj-lE-y-dx", "(tmpy[k - NX] - tmpy[k]) / p->dy;", "(tmpy[k - NX] - tmpy[k]) / p->dx;",
     ["dot-aniso", "transpose"]),
    # the perfect-conductor rule: threshold moved above the test's 1e3 S/m,
    # or a conductor cell that still takes the curl
    ("pec-threshold", "#define ORC_PEC_SIGMA 100.0", "#define ORC_PEC_SIGMA 1.0e4", ["pec"]),
    ("pec-curl-kept", "Cs[k] = 0.0;", "Cs[k] = 1.0 / (ORC_EPS0 * eps_r[k] / dt);", ["pec"]),
]
# Not planted: dropping the sigma > 100 test in orc_gradient_finalize.  Ez is
# identically zero in a perfect-conductor cell, so both correlation sums
# there are exactly zero and the branch cannot change any result.

# Mistakes in the Python marshalling (oracle.py): which spacing builds which
# axis' CPML profile.
PY_MUTATIONS = [
    ("profile-y-uses-dx", "self.py = cpml_profile(self.NY, npml, self.dy, self.dt, *cp)",
     "self.py = cpml_profile(self.NY, npml, self.dx, self.dt, *cp)", ["transpose"]),
    ("profile-x-uses-dy", "self.px = cpml_profile(self.NX, npml, self.dx, self.dt, *cp)",
     "self.px = cpml_profile(self.NX, npml, self.dy, self.dt, *cp)", ["transpose"]),
]

PINS = {
    "energy": lambda: pins.pec_energy_drift(600),
    "hankel": lambda: (pins.hankel_trace_error(0.006), 1e-2),
    "decay": pins.lossy_decay,
    "cpml": pins.cpml_reflection,
    "dot": pins.dot_product,
    "fd": pins.fd_gradient,
    "energy-aniso": lambda: pins.pec_energy_drift(600, dy_ratio=0.73),
    "hankel-aniso": lambda: (max(pins.hankel_trace_errors(0.006, 0.0044)), 1e-2),
    "dot-aniso": lambda: pins.dot_product(0.73),
    "transpose": pins.transpose_symmetry,
    "pec": pins.pec_material_box,
}


def _caught(catchers):
    caught = []
    for pin in catchers:
        try:
            v, bound = PINS[pin]()
            failed = not (v <= bound)
        except (FloatingPointError, ValueError, ZeroDivisionError):
            failed = True
        if failed:
            caught.append(pin)
    return caught


@pytest.mark.parametrize("name,old,new,catchers", MUTATIONS, ids=[m[0] for m in MUTATIONS])
def test_pins_catch_planted_mistake(tmp_path, name, old, new, catchers):
    src = open(SRC).read()
    assert src.count(old) == 1, f"mutation anchor not unique/present: {old!r}"
    mpath = tmp_path / "mutant.c"
    mpath.write_text(src.replace(old, new))
    so = oracle.compile_source(str(mpath), str(tmp_path / "libmutant.so"))
    with oracle.use_library(so):
        caught = _caught(catchers)
    assert caught, f"no pin caught mutation {name}"


@pytest.mark.parametrize("name,old,new,catchers", PY_MUTATIONS, ids=[m[0] for m in PY_MUTATIONS])
def test_pins_catch_planted_python_mistake(monkeypatch, name, old, new, catchers):
    """The same for the numpy marshalling: a mutated copy of oracle.py is
    loaded as a module of its own and put in place of the oracle the pins
    call."""
    import types

    from oracle import oracle as oracle_module
    path = oracle_module.__file__
    src = open(path).read()
    assert src.count(old) == 1, f"mutation anchor not unique/present: {old!r}"
    mod = types.ModuleType("oracle_mutant")
    mod.__file__ = path
    exec(compile(src.replace(old, new), path, "exec"), mod.__dict__)
    monkeypatch.setattr(pins, "oracle", mod)
    caught = _caught(catchers)
    assert caught, f"no pin caught mutation {name}"


def test_unmutated_oracle_passes_every_pin():
    """The mutation checks above mean something only if the pins they use
    hold for the oracle as written."""
    assert _caught(list(PINS)) == []
