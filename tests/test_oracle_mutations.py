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
]

PINS = {
    "energy": lambda: pins.pec_energy_drift(600),
    "hankel": lambda: (pins.hankel_trace_error(0.006), 1e-2),
    "decay": pins.lossy_decay,
    "cpml": pins.cpml_reflection,
    "dot": pins.dot_product,
    "fd": pins.fd_gradient,
}


@pytest.mark.parametrize("name,old,new,catchers", MUTATIONS, ids=[m[0] for m in MUTATIONS])
def test_pins_catch_planted_mistake(tmp_path, name, old, new, catchers):
    src = open(SRC).read()
    assert src.count(old) == 1, f"mutation anchor not unique/present: {old!r}"
    mpath = tmp_path / "mutant.c"
    mpath.write_text(src.replace(old, new))
    so = oracle.compile_source(str(mpath), str(tmp_path / "libmutant.so"))
    caught = []
    with oracle.use_library(so):
        for pin in catchers:
            try:
                v, bound = PINS[pin]()
                failed = not (v <= bound)
            except (FloatingPointError, ValueError, ZeroDivisionError):
                failed = True
            if failed:
                caught.append(pin)
    assert caught, f"no pin caught mutation {name}"
