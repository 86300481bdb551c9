"""Pins of the oracle's effective algorithmic tangent d<sigma>/dE.

* central finite differences of the effective stress: the increment is
  re-solved from a copy of the step-n state with the macro strain perturbed
  along each Mandel direction (a plastic increment of a PA66 / E-glass cell);
* C_bar is symmetric and positive definite (the local PA66 tangent is
  symmetric, the projection keeps it so);
* with linear phases it is the effective stiffness.
"""
import copy

import numpy as np

from oracle import solver, tensor
from paper_2109_14403_amd import workloads as W


def solve_from(cell, st, strain_m):
    c = copy.deepcopy(cell)
    out = c.solve_increment(tensor.mandel_to_components(strain_m), st.theta, st.grad, st.dt, tol=1e-13,
                            cg_rtol=1e-6)
    return tensor.components_to_mandel(out["stress"])


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
        fd[:, j] = (solve_from(before, st, E + dE) - solve_from(before, st, E - dE)) / (2 * h)
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
