"""The FP64 oracle against facts outside itself (see oracle_pins.py)."""
import math

import numpy as np
import pytest

import oracle
from tests import oracle_pins as pins


def test_hankel_line_source_second_order():
    e_coarse, e_fine = pins.hankel_error()
    # about 1e-2 or better at >= 20 cells per wavelength at 2.5 f0
    assert e_coarse < 1e-2, e_coarse
    # halving dx and dt must cut the error ~4x (order 1.8 .. 2.2)
    ratio = e_coarse / e_fine
    assert 2 ** 1.8 <= ratio <= 2 ** 2.2, (e_coarse, e_fine, ratio)


@pytest.mark.parametrize("dy_ratio", [1.0, 0.73])
def test_pec_cavity_energy_conserved(dy_ratio):
    v, bound = pins.pec_energy_drift(dy_ratio=dy_ratio)
    assert v <= bound, v


def test_hankel_line_source_anisotropic_cells():
    """dy = 0.733 dx: receivers along x and along y both match the analytic
    field and both converge at second order."""
    coarse, fine = pins.hankel_error_aniso()
    for ec, ef in zip(coarse, fine):
        assert ec < 1e-2, coarse
        assert 2 ** 1.8 <= ec / ef <= 2 ** 2.2, (coarse, fine)


def test_transpose_symmetry_anisotropic_cells():
    v, bound = pins.transpose_symmetry()
    assert v <= bound, v


def test_pec_material_ring_equals_pec_box():
    v, bound = pins.pec_material_box()
    assert v <= bound, v


def test_pec_material_threshold():
    """sigma just above 100 S/m is a perfect conductor, just below it is
    not (Sec. 3.2, coefficient kernel)."""
    P = oracle.Problem(np.full((3, 2), 4.0), np.array([[0.0, 100.0], [100.0001, 1e3],
                                                       [99.999, 50.0]]), 0, 0.01, 0.01, 1e-11)
    pec = P.Ca == 0.0
    assert np.array_equal(pec, [[False, False], [True, True], [False, False]])
    assert np.array_equal(P.Cs == 0.0, pec)


def test_uniform_lossy_decay_rate():
    v, bound = pins.lossy_decay()
    assert v <= bound, v


@pytest.mark.parametrize("npml", [0, 8])
def test_reciprocity(npml):
    v, bound = pins.reciprocity(npml)
    assert v <= bound, v


@pytest.mark.parametrize("dy_ratio", [1.0, 0.73])
def test_adjoint_dot_product(dy_ratio):
    v, bound = pins.dot_product(dy_ratio)
    assert v <= bound, v


@pytest.mark.parametrize("dy_ratio", [1.0, 0.73])
def test_gradient_central_differences(dy_ratio):
    v, bound = pins.fd_gradient(dy_ratio)
    assert v <= bound, v


def test_cpml_reflection_bound():
    v, bound = pins.cpml_reflection()
    assert v <= bound, v


def test_misfit_is_half_sum_of_squares():
    c = pins.fd_setup()
    P = oracle.Problem(c["eps0"], c["sig0"], c["npml"], c["dx"], c["dx"], c["dt"], **c["kw"])
    J, _, _, tr = P.gradient(c["src"], c["rec"], c["w"], c["obs"], c["nt"])
    assert J == pytest.approx(0.5 * float(np.sum((tr - c["obs"]) ** 2)), rel=1e-15)


def test_cpml_profile_shape():
    """Profile reading: zero conductivity (a = 0, kappa = 1) in the interior,
    graded to the outer edge, symmetric low/high sides."""
    n, npml = 30, 6
    bE, aE, kE, bH, aH, kH = oracle.cpml_profile(n, npml, 0.01, 2e-11, 3, 1.0, 5.0, 1e-3)
    assert np.all(aE[npml:n - npml] == 0) and np.all(kE[npml:n - npml] == 1)
    assert np.all(aH[npml:n - 1 - npml] == 0)
    assert np.all(aE[1:npml] < 0) and np.all(aH[:npml] < 0)
    assert np.allclose(aE[:npml], aE[::-1][:npml], rtol=1e-14, atol=0)
    assert np.allclose(aH[:npml], aH[n - 2::-1][:npml], rtol=1e-14, atol=0)
    assert np.all(np.diff(kE[:npml + 1]) > 0)  # 1/kappa grows towards the interior


@pytest.mark.parametrize("K", [1, 7, 37, 150, 400, None])
def test_checkpointed_gradient_equals_history(K):
    """The segment-checkpoint mode re-runs the same recursions in the same
    order, so it must reproduce the full-history gradient bit for bit for
    any interval, including K = 1, K not dividing nt and K >= nt."""
    c = pins.fd_setup(0.73)
    P = oracle.Problem(c["eps0"], c["sig0"], c["npml"], c["dx"], c["dy"], c["dt"], **c["kw"])
    a = P.gradient(c["src"], c["rec"], c["w"], c["obs"], c["nt"])
    b = P.gradient_checkpointed(c["src"], c["rec"], c["w"], c["obs"], c["nt"], K)
    assert a[0] == b[0]
    for x, y in zip(a[1:], b[1:]):
        assert np.array_equal(x, y)
