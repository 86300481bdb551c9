"""Pins of the oracle's mixed boundary conditions and adiabatic heat balance
(the paper's single-point virtual experiments: stress-free lateral
directions; c (theta - theta^n) / dt = <D> at one macroscopic point).

* homogeneous isotropic thermoelastic cell under uniaxial stress: the lateral
  strains of the closed form, with thermal expansion;
* two-phase laminate under uniaxial stress: the effective law
  sigma = C_b (E - alpha_b dtheta) with C_b from the laminate equation of
  Sec. 3.2 and alpha_b from Levin's formula, both independent of the cell
  solver;
* homogeneous thermoelastic cell, adiabatic, strain-controlled: the implicit
  heat balance c0 (theta - theta^n) = -theta 3K alpha tr(dE) in closed form;
* the same cell adiabatic under uniaxial stress: a 2 x 2 nonlinear system
  (lateral strain, theta) solved here by Newton;
* a plastic PA66 / E-glass cell: the prescribed stress components are met,
  the heat balance holds, and the committed state is that of a strain
  controlled increment at the reported strain and temperature.
"""
import copy

import numpy as np
import pytest

from oracle import solver, tensor
from paper_2109_14403_amd import workloads as W

from test_oracle_cell import MAT_A, MAT_B, laminate_equation_stiffness, levin_expansion

LATERAL = [False, True, True, True, True, True]   # only E11 prescribed


def test_homogeneous_uniaxial_stress_closed_form():
    cell = solver.Cell(np.zeros((4, 4, 4), dtype=np.uint8), [MAT_A])
    e11, theta = 2e-3, 313.0
    out = cell.solve_load([e11, 0, 0, 0, 0, 0], np.zeros(6), LATERAL, theta, [0, 0, 0], 1.0, tol=1e-12)
    a, nu, E = MAT_A["alpha0"], MAT_A["nu"], MAT_A["E"]
    th = a * (theta - MAT_A["theta0"])
    expect = np.array([e11, th - nu * (e11 - th), th - nu * (e11 - th), 0, 0, 0])
    assert np.allclose(out["strain"], expect, rtol=1e-10, atol=1e-15)
    assert np.isclose(out["stress"][0], E * (e11 - th), rtol=1e-10)
    assert np.abs(out["stress"][1:]).max() <= 1e-9 * abs(out["stress"][0])


@pytest.mark.parametrize("axis,load", [(0, 0), (1, 0), (2, 5)])
def test_laminate_mixed_conditions_match_effective_law(axis, load):
    img = W.laminate((8, 8, 8), [2, 6], axis=axis)
    cell = solver.Cell(img, [MAT_A, MAT_B])
    la = cell.laws
    lam = 0.5 * min(np.linalg.eigvalsh(la[0].C).min(), np.linalg.eigvalsh(la[1].C).min())
    Cb = laminate_equation_stiffness(la[1].C, la[0].C, img.mean(), np.eye(3)[axis], lam)
    ab = levin_expansion(Cb, la)
    dth = 25.0
    mask = [True] * 6
    mask[load] = False
    strain = np.zeros(6)
    strain[load] = 1.5e-3
    out = cell.solve_load(strain, np.zeros(6), mask, MAT_A["theta0"] + dth, [0, 0, 0], 1.0, tol=1e-13)
    # effective law, Mandel: S_f = 0 fixes the free strains
    Em = tensor.components_to_mandel(strain)
    f = [c for c in range(6) if mask[c]]
    rhs = -(Cb[np.ix_(f, [load])] @ (Em[[load]] - ab[[load]] * dth)) + Cb[np.ix_(f, f)] @ (ab[f] * dth)
    Ef = np.linalg.solve(Cb[np.ix_(f, f)], rhs)
    expect = Em.copy()
    expect[f] = Ef
    s_expect = Cb @ (expect - ab * dth)
    assert np.allclose(tensor.components_to_mandel(out["strain"]), expect, rtol=1e-8, atol=1e-12)
    assert np.allclose(tensor.components_to_mandel(out["stress"]), s_expect, rtol=1e-8,
                       atol=1e-8 * np.abs(s_expect).max())


def test_homogeneous_adiabatic_closed_form():
    cell = solver.Cell(np.zeros((4, 4, 4), dtype=np.uint8), [MAT_A])
    K, _ = tensor.bulk_shear(MAT_A["E"], MAT_A["nu"])
    c0, a = MAT_A["c0"], MAT_A["alpha0"]
    theta_n = 300.0
    for strain, dt in ((np.array([2e-3, 1e-3, -5e-4, 1e-4, 0, 0]), 0.5), (np.array([-1e-3, 0, 2e-3, 0, 3e-4, 0]), 2.0)):
        dtr = strain[:3].sum() - tensor.mandel_to_components(cell.E_n)[:3].sum()
        out = cell.solve_load(strain, np.zeros(6), [False] * 6, theta_n, [0, 0, 0], dt, adiabatic=True, tol=1e-12)
        expect = theta_n * c0 / (c0 + 3 * K * a * dtr)
        assert np.isclose(out["theta"], expect, rtol=1e-12)
        assert out["stagger_iterations"] >= 2
        theta_n = out["theta"]


def test_homogeneous_adiabatic_uniaxial_stress():
    cell = solver.Cell(np.zeros((4, 4, 4), dtype=np.uint8), [MAT_A])
    K, G = tensor.bulk_shear(MAT_A["E"], MAT_A["nu"])
    c0, a, t0 = MAT_A["c0"], MAT_A["alpha0"], MAT_A["theta0"]
    e11, theta_n, dt = 3e-3, 295.0, 1.0
    out = cell.solve_load([e11, 0, 0, 0, 0, 0], np.zeros(6), LATERAL, theta_n, [0, 0, 0], dt, adiabatic=True,
                          tol=1e-12)

    # unknowns: lateral strain x (= eps22 = eps33), theta
    def F(u):
        x, th = u
        tr = e11 + 2 * x
        s22 = 3 * K * (tr / 3 - a * (th - t0)) + 2 * G * (x - tr / 3)
        heat = c0 * (th - theta_n) + th * 3 * K * a * tr
        return np.array([s22, heat])

    u = np.array([0.0, theta_n])
    for _ in range(30):
        J = np.zeros((2, 2))
        for k in range(2):
            h = np.zeros(2)
            h[k] = 1e-7 * max(abs(u[k]), 1.0)
            J[:, k] = (F(u + h) - F(u - h)) / (2 * h[k])
        u = u - np.linalg.solve(J, F(u))
    assert np.isclose(out["strain"][1], u[0], rtol=1e-9) and np.isclose(out["strain"][2], u[0], rtol=1e-9)
    assert np.isclose(out["theta"], u[1], rtol=1e-12)


def test_plastic_cell_mixed_adiabatic_properties():
    rng = np.random.default_rng(4)
    img = (rng.random((8, 8, 8)) < 0.3).astype(np.uint8)
    laws = [W.pa66(), W.e_glass()]
    cell = solver.Cell(img, laws)
    theta = 293.15
    for k in range(1, 5):
        before = copy.deepcopy(cell)
        out = cell.solve_load([0.006 * k, 0, 0, 0, 0, 0], np.zeros(6), LATERAL, theta, [0, 0, 0], 2.0,
                              adiabatic=True, tol=1e-12)
        s = out["stress"]
        assert np.abs(s[1:]).max() <= 1e-9 * abs(s[0])
        # heat balance at the reported temperature (up to the staggering tolerance)
        assert abs(out["heat_capacity"] * (out["theta"] - theta) - 2.0 * out["coupling"]) <= 1e-8 * out["heat_capacity"]
        # the committed increment is the strain-controlled one at (E, theta)
        ref = before.solve_increment(out["strain"], out["theta"], [0, 0, 0], 2.0, tol=1e-12)
        assert np.allclose(ref["stress"], s, rtol=1e-9, atol=1e-9 * np.abs(s).max())
        for i in cell.state:      # before now holds the strain-controlled increment's commit
            assert np.allclose(cell.state[i]["ep"], before.state[i]["ep"], atol=1e-14)
        theta = out["theta"]
    # plastic flow, and a temperature change (tension cools by the thermoelastic coupling)
    assert out["dissipation"] > 0.0 and abs(theta - 293.15) > 0.1
