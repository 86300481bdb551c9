"""Pins of the oracle's effective algorithmic tangents (Sec. 3.3: the
derivatives of the effective stress and coupling term with respect to the
macro strain and temperature).

* central finite differences of the effective stress and coupling term: the
  increment is re-solved from a copy of the step-n state with the macro
  strain perturbed along each Mandel direction, or the temperature perturbed
  (a plastic increment of a PA66 / E-glass cell); these re-solves share
  nothing with the linearized solves but the cell problem itself;
* d<sigma>/dE is symmetric and positive definite (the local PA66 tangent is
  symmetric, the projection keeps it so);
* with linear phases d<sigma>/dE is the effective stiffness;
* a homogeneous thermoelastic cell has the closed forms
  d<sigma>/dtheta = -C[alpha], d<D>/dE = -theta C[alpha] / dt and
  d<D>/dtheta = -C[alpha] : (E - E^n) / dt.
"""
import copy

import numpy as np

from oracle import solver, tensor
from paper_2109_14403_amd import workloads as W


def solve_from(cell, st, strain_m, theta=None):
    c = copy.deepcopy(cell)
    out = c.solve_increment(tensor.mandel_to_components(strain_m), st.theta if theta is None else theta, st.grad,
                            st.dt, tol=1e-13, cg_rtol=1e-6)
    return tensor.components_to_mandel(out["stress"]), out["coupling"]


def plastic_cell():
    rng = np.random.default_rng(4)
    img = (rng.random((8, 8, 8)) < 0.3).astype(np.uint8)
    cell = solver.Cell(img, [W.pa66(), W.e_glass()])
    hist = W.history_shear_tension()
    for st in hist[:5]:
        cell.solve_increment(st.strain, st.theta, st.grad, st.dt, tol=1e-13, cg_rtol=1e-6)
    return cell, hist[5]


def test_tangent_matches_finite_differences():
    cell, st = plastic_cell()
    before = copy.deepcopy(cell)
    out = cell.solve_increment(st.strain, st.theta, st.grad, st.dt, tol=1e-13, cg_rtol=1e-6)
    assert out["dissipation"] > 0.0
    Cbar = cell.algorithmic_tangent(tol=1e-13)
    E = tensor.components_to_mandel(st.strain)
    h = 1e-7
    fd = np.zeros((6, 6))
    for j in range(6):
        dE = np.zeros(6)
        dE[j] = h
        fd[:, j] = (solve_from(before, st, E + dE)[0] - solve_from(before, st, E - dE)[0]) / (2 * h)
    err = np.abs(fd - Cbar).max() / np.abs(Cbar).max()
    assert err < 1e-5, err


def test_tangent_symmetric_positive_definite():
    cell, st = plastic_cell()
    cell.solve_increment(st.strain, st.theta, st.grad, st.dt, tol=1e-13, cg_rtol=1e-6)
    Cbar = cell.algorithmic_tangent(tol=1e-13)
    assert np.abs(Cbar - Cbar.T).max() <= 1e-9 * np.abs(Cbar).max()
    assert np.linalg.eigvalsh(0.5 * (Cbar + Cbar.T)).min() > 0.0


def test_linear_phases_tangent_is_effective_stiffness():
    wl = W.small_sphere_workload()
    cell = solver.Cell(wl.phases, wl.laws)
    st = wl.history[0]
    cell.solve_increment(st.strain, st.theta, st.grad, st.dt, tol=1e-12)
    assert np.allclose(cell.algorithmic_tangent(), cell.effective_stiffness(), rtol=1e-10, atol=1e-8)


def test_temperature_and_coupling_tangents_match_finite_differences():
    cell, st = plastic_cell()
    before = copy.deepcopy(cell)
    cell.solve_increment(st.strain, st.theta, st.grad, st.dt, tol=1e-13, cg_rtol=1e-6)
    t = cell.algorithmic_tangents(tol=1e-13)
    E = tensor.components_to_mandel(st.strain)
    ht = 1e-3
    sp, Dp = solve_from(before, st, E, st.theta + ht)
    sm, Dm = solve_from(before, st, E, st.theta - ht)
    fd_s = (sp - sm) / (2 * ht)
    fd_D = (Dp - Dm) / (2 * ht)
    print("dsdt", t["dsdt"], fd_s, "dDdt", t["dDdt"], fd_D)
    assert np.abs(fd_s - t["dsdt"]).max() <= 1e-5 * np.abs(fd_s).max()
    assert abs(fd_D - t["dDdt"]) <= 1e-5 * abs(fd_D)
    h = 1e-7
    fd_e = np.zeros(6)
    for j in range(6):
        dE = np.zeros(6)
        dE[j] = h
        fd_e[j] = (solve_from(before, st, E + dE)[1] - solve_from(before, st, E - dE)[1]) / (2 * h)
    print("dDde", t["dDde"], fd_e)
    assert np.abs(fd_e - t["dDde"]).max() <= 1e-5 * np.abs(fd_e).max()
    assert np.allclose(t["dsde"], cell.algorithmic_tangent(tol=1e-13), rtol=1e-9, atol=1e-6)


def test_homogeneous_thermoelastic_closed_forms():
    glass = W.e_glass()
    cell = solver.Cell(np.zeros((4, 4, 4), dtype=np.uint8), [glass])
    E0 = np.array([1e-3, -2e-4, 3e-4, 1e-4, 0.0, -5e-5])
    cell.solve_increment(E0, 320.0, np.zeros(3), 2.0)
    E1 = E0 + np.array([2e-4, 1e-4, -1e-4, 0.0, 3e-5, 0.0])
    theta, dt = 340.0, 0.5
    cell.solve_increment(E1, theta, np.zeros(3), dt)
    t = cell.algorithmic_tangents()
    K, G = tensor.bulk_shear(glass["E"], glass["nu"])
    Ca = 3.0 * K * glass["alpha0"] * np.array([1.0, 1, 1, 0, 0, 0])
    dEm = tensor.components_to_mandel(E1 - E0)
    assert np.allclose(t["dsde"], tensor.isotropic(K, G), rtol=1e-12, atol=1e-6)
    assert np.allclose(t["dsdt"], -Ca, rtol=1e-12, atol=0)
    assert np.allclose(t["dDde"], -theta * Ca / dt, rtol=1e-12, atol=0)
    assert np.isclose(t["dDdt"], -(Ca @ dEm) / dt, rtol=1e-12)
