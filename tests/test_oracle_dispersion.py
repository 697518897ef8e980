"""Pins of the element matrices through plane-wave analysis of the assembled operator."""
import numpy as np
import pytest

from oracle import dispersion as dsp
from oracle import element as el

RHO, VS, VP = 2000.0, 1000.0, 2000.0
MU = RHO * VS ** 2
LAM = RHO * VP ** 2 - 2 * MU


def _ovfem(h=1.0):
    Kl, Km = el.ovfem_reference()
    return h * (LAM * Kl + MU * Km)


@pytest.mark.parametrize("kh", [0.2, 2 * np.pi / 10, 2 * np.pi / 5, 2.0])
@pytest.mark.parametrize("which", ["ovfem", "trilinear"])
def test_axis_aligned_waves_follow_the_1d_closed_form(kh, which):
    """Along a grid axis both elements reduce to the 1D lattice: c_h / c = sin(kh/2) / (kh/2)."""
    h = 1.0
    K = _ovfem(h) if which == "ovfem" else el.trilinear_stiffness(LAM, MU, h)
    c = dsp.phase_velocities(K, RHO, h, (0, 0, 1), kh)
    ratio = np.sin(kh / 2) / (kh / 2)
    assert np.allclose(c, [VS * ratio, VS * ratio, VP * ratio], rtol=1e-12)


@pytest.mark.parametrize("direction", [(1, 1, 1), (1, 2, 3), (1, 1, 0)])
def test_second_order_convergence_of_phase_velocity(direction):
    h = 1.0
    K = _ovfem(h)
    errs = []
    for kh in (0.2, 0.1):
        c = dsp.phase_velocities(K, RHO, h, direction, kh)
        errs.append(np.abs(c / np.array([VS, VS, VP]) - 1.0))
    ratio = errs[0] / errs[1]
    assert np.all((ratio > 3.9) & (ratio < 4.1)), ratio


@pytest.mark.parametrize("ppw", [10, 5])
def test_ovfem_less_dispersive_than_trilinear_off_axis(ppw):
    """OVFEM suppresses the dispersion of the lumped trilinear element (Sec. 2, Sec. 3 Table 2)."""
    h, kh = 1.0, 2 * np.pi / ppw
    ref = np.array([VS, VS, VP])
    eo = np.abs(dsp.phase_velocities(_ovfem(h), RHO, h, (1, 1, 1), kh) / ref - 1)
    et = np.abs(dsp.phase_velocities(el.trilinear_stiffness(LAM, MU, h), RHO, h, (1, 1, 1), kh) / ref - 1)
    assert np.all(eo < et)
    # P wave also along a face diagonal
    eo2 = abs(dsp.phase_velocities(_ovfem(h), RHO, h, (1, 1, 0), kh)[2] / VP - 1)
    et2 = abs(dsp.phase_velocities(el.trilinear_stiffness(LAM, MU, h), RHO, h, (1, 1, 0), kh)[2] / VP - 1)
    assert eo2 < et2


def test_highest_lattice_frequency_gives_cfl_h_over_vp():
    """omega_max = 2 Vp / h on the lattice (Vp = 2 Vs), so central differences need dt < h / Vp."""
    h = 1.0
    w = dsp.max_frequency(_ovfem(h), RHO, h, n=8)
    assert w == pytest.approx(2 * VP / h, rel=1e-12)


def test_equal_dispersion_accuracy_fixture():
    """tests/golden/equal_dispersion_accuracy.json is what the oracle computes, OVFEM is
    the more accurate element at equal resolution, and both errors fall at second order."""
    import importlib.util
    import json
    import os
    here = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
    spec = importlib.util.spec_from_file_location("mk", os.path.join(here, "make_equal_dispersion_accuracy.py"))
    mk = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mk)
    fx = json.load(open(os.path.join(here, "equal_dispersion_accuracy.json")))
    rows = {r["ppw_ovfem"]: r for r in fx["rows"]}
    dirs = mk.directions()
    again = mk.equal_accuracy(10, dirs, iters=40)
    for k in ("rms_phase_error", "ppw_trilinear", "cost_factor"):
        assert again[k] == pytest.approx(rows[10][k], rel=1e-12)
    assert rows[10]["ppw_trilinear"] > 10 and rows[10]["cost_factor"] > 1
    assert rows[5]["rms_phase_error"] / rows[10]["rms_phase_error"] == pytest.approx(4.0, rel=0.1)
    assert rows[10]["rms_phase_error"] / rows[20]["rms_phase_error"] == pytest.approx(4.0, rel=0.02)


@pytest.mark.parametrize("which,ppw,s_ratio,p_ratio", [
    ("ovfem", 10, 0.99850, 0.98035),
    ("trilinear", 10, 0.97833, 0.97025),
    ("ovfem", 5, 0.99253, None),
    ("trilinear", 5, 0.91639, None),
])
def test_diagonal_phase_velocities_match_an_independent_bloch_computation(which, ppw, s_ratio, p_ratio):
    """Semi-discrete phase velocities along (1, 1, 1) at ppw grid points per wavelength
    (Vp = 2 Vs), against values of a separate computation of the plane-wave symbol from the
    exact element integrals (five digits): a transposed block, a wrong phase sign or a wrong
    element weight moves them in the third digit or earlier."""
    h = 1.0
    K = _ovfem(h) if which == "ovfem" else el.trilinear_stiffness(LAM, MU, h)
    c = dsp.phase_velocities(K, RHO, h, (1, 1, 1), 2 * np.pi / ppw)
    assert abs(c[0] / VS - s_ratio) < 6e-6 and abs(c[1] / VS - s_ratio) < 6e-6
    if p_ratio is not None:
        assert abs(c[2] / VP - p_ratio) < 6e-6
