"""Pins of the oracle's direct DMN (Sec. 3).

* depth 1 is one laminate: it equals the FFT oracle's effective stiffness of
  the same laminate microstructure (an independent solver);
* any parameters: the prediction lies between the Voigt and Reuss bounds of
  the phase fractions the weights give, and equal phases give that phase;
* autograd gradients of the loss against central finite differences;
* online evaluation with linear elastic phases reproduces the offline linear
  homogenization (stress and d<sigma>/dE), through Newton's method on the
  jumps instead of the laminate equation;
* online with the same PA66 law in both phases is the point law, with zero
  jumps;
* the online d<sigma>/dE, d<sigma>/dtheta, d<D>/dE and d<D>/dtheta against
  finite differences of re-evaluated increments; dissipation >= 0;
* a DMN of one thermoelastic law: d<sigma>/dtheta = -C[alpha],
  d<D>/dE = -theta C[alpha] / dt, d<D>/dtheta = -C[alpha] : dE / dt.
"""
import copy

import numpy as np
import pytest
import torch

from oracle import dmn, solver, tensor
from oracle.laws import PA66
from paper_2109_14403_amd import workloads as W

from test_oracle_cell import MAT_A, MAT_B

RNG = np.random.default_rng(8)


def iso(K, G):
    return tensor.isotropic(K, G)


def random_params(K):
    m = RNG.standard_normal((2 ** K - 1, 3))
    v = RNG.uniform(0.0, 1.0, 2 ** K)
    return m, v / v.sum()


def test_depth_one_is_the_fft_laminate():
    img = W.laminate((8, 8, 8), [2, 6], axis=0)      # normal e1; phase 1 (B) on 4 of 8 layers
    cell = solver.Cell(img, [MAT_A, MAT_B])
    fft = cell.effective_stiffness(tol=1e-13)
    CA, CB = cell.laws[0].C, cell.laws[1].C
    c_b = img.mean()
    # leaf 0 = first input, leaf 1 = second input
    got = dmn.homogenize_np(CB[None], CA[None], np.array([[3.0, 0.0, 0.0]]), np.array([c_b, 1 - c_b]))[0]
    assert np.allclose(got, fft, rtol=1e-9, atol=1e-9 * np.abs(fft).max())


@pytest.mark.parametrize("K", [2, 4, 6])
def test_bounds_and_equal_phases(K):
    m, v = random_params(K)
    C1 = iso(30.0, 20.0)[None]
    C2 = iso(2.0, 0.7)[None]
    D = dmn.homogenize_np(C1, C2, m, v)[0]
    w = np.maximum(v, 0)
    c1 = w[0::2].sum() / w.sum()
    voigt = c1 * C1[0] + (1 - c1) * C2[0]
    reuss = np.linalg.inv(c1 * np.linalg.inv(C1[0]) + (1 - c1) * np.linalg.inv(C2[0]))
    assert np.linalg.eigvalsh(voigt - D).min() >= -1e-10 * np.abs(voigt).max()
    assert np.linalg.eigvalsh(D - reuss).min() >= -1e-10 * np.abs(voigt).max()
    assert np.allclose(D, D.T, atol=1e-10 * np.abs(D).max())
    same = dmn.homogenize_np(C1, C1, m, v)[0]
    assert np.allclose(same, C1[0], rtol=1e-10, atol=1e-10 * np.abs(C1).max())


def test_gradients_match_finite_differences():
    K = 3
    m, v = random_params(K)
    v[2] = -0.05                                  # one clamped weight
    B = 4
    C1 = np.stack([iso(*RNG.uniform([5, 3], [40, 30])) for _ in range(B)])
    C2 = np.stack([iso(*RNG.uniform([1, 0.3], [4, 2])) for _ in range(B)])
    Cbar = dmn.homogenize_np(C1, C2, RNG.standard_normal(m.shape), np.full(2 ** K, 1.0 / 2 ** K)) * 1.03
    J, gm, gv = dmn.loss_and_grad(C1, C2, Cbar, m, v)
    h = 1e-6
    f = lambda mm, vv: dmn.loss_and_grad(C1, C2, Cbar, mm, vv)[0]
    for idx in [(0, 0), (3, 2), (6, 1)]:
        mp, mm = m.copy(), m.copy()
        mp[idx] += h
        mm[idx] -= h
        assert np.isclose((f(mp, v) - f(mm, v)) / (2 * h), gm[idx], rtol=1e-5, atol=1e-9)
    for i in [0, 2, 5]:
        vp, vm = v.copy(), v.copy()
        vp[i] += h
        vm[i] -= h
        assert np.isclose((f(m, vp) - f(m, vm)) / (2 * h), gv[i], rtol=1e-5, atol=1e-9)
    assert gv[2] == 0.0                           # clamped weight: no gradient


def glass(E=70e3, nu=0.22):
    return dict(kind="thermoelastic", E=E, nu=nu, alpha0=5e-6, kappa0=1.0, c0=2.0, theta0=293.15)


def test_online_linear_phases_match_offline():
    K = 4
    m, v = random_params(K)
    l1, l2 = glass(), glass(3e3, 0.35)
    net = dmn.OnlineDMN(m, v, l1, l2, tol=1e-13)
    C1 = tensor.isotropic(*tensor.bulk_shear(l1["E"], l1["nu"]))
    C2 = tensor.isotropic(*tensor.bulk_shear(l2["E"], l2["nu"]))
    D = dmn.homogenize_np(C1[None], C2[None], m, v)[0]
    strain = np.array([2e-3, -1e-3, 5e-4, 3e-4, 0.0, -2e-4])
    out = net.step(strain, 293.15, 1.0)                  # theta0: no thermal strain
    expect = tensor.mandel_to_components(D @ tensor.components_to_mandel(strain))
    assert np.allclose(out["stress"], expect, rtol=1e-9, atol=1e-9 * np.abs(expect).max())
    assert np.allclose(out["dsde"], D, rtol=1e-9, atol=1e-9 * np.abs(D).max())


def test_online_same_pa66_phases_is_the_point_law():
    K = 3
    m, v = random_params(K)
    p = W.pa66()
    net = dmn.OnlineDMN(m, v, p, p, tol=1e-12)
    law = PA66(p)
    st = law.initial_state(1)
    en = np.zeros((6, 1))
    for strain, th in (([0.01, 0, 0, 0, 0, 0.004], 300.0), ([0.025, 0, 0, 0, 0, 0.01], 320.0)):
        out = net.step(np.array(strain, dtype=float), th, 2.0)
        E = tensor.components_to_mandel(np.array(strain, dtype=float))[:, None]
        pt = law.update(E, en, st, th, 2.0)
        st, en = pt["state"], E
        assert np.allclose(out["stress"], tensor.mandel_to_components(pt["sigma"][:, 0]), rtol=1e-9)
        assert np.isclose(out["coupling"], pt["coupling"][0], rtol=1e-9)
        assert np.abs(net.a).max() <= 1e-12
    assert pt["delta"][0] > 0


def test_online_tangent_matches_finite_differences():
    K = 3
    m, v = random_params(K)
    net = dmn.OnlineDMN(m, v, W.e_glass(), W.pa66(), tol=1e-12)
    for k in range(1, 4):
        net.step(np.array([0.008 * k, 0, 0, 0, 0, 0.003 * k]), 300.0, 2.0)
    before = copy.deepcopy(net)
    strain = np.array([0.032, 0.001, 0, 0, 0, 0.012])
    out = net.step(strain, 300.0, 2.0)
    assert out["dissipation"] > 0.0
    E = tensor.components_to_mandel(strain)
    h = 1e-7
    fd = np.zeros((6, 6))
    for j in range(6):
        res = []
        for sgn in (1, -1):
            n2 = copy.deepcopy(before)
            Ej = E.copy()
            Ej[j] += sgn * h
            res.append(tensor.components_to_mandel(n2.step(tensor.mandel_to_components(Ej), 300.0, 2.0)["stress"]))
        fd[:, j] = (res[0] - res[1]) / (2 * h)
    assert np.abs(fd - out["dsde"]).max() <= 1e-5 * np.abs(fd).max()


def test_online_temperature_and_coupling_tangents_match_finite_differences():
    K = 3
    m, v = random_params(K)
    net = dmn.OnlineDMN(m, v, W.e_glass(), W.pa66(), tol=1e-12)
    for k in range(1, 4):
        net.step(np.array([0.008 * k, 0, 0, 0, 0, 0.003 * k]), 300.0 + k, 2.0)
    before = copy.deepcopy(net)
    strain = np.array([0.032, 0.001, 0, 0, 0, 0.012])
    th = 305.0
    out = net.step(strain, th, 2.0, all_tangents=True)
    assert out["dissipation"] > 0.0
    E = tensor.components_to_mandel(strain)

    def again(Em, t):
        n2 = copy.deepcopy(before)
        r = n2.step(tensor.mandel_to_components(Em), t, 2.0)
        return tensor.components_to_mandel(r["stress"]), r["coupling"]

    ht = 1e-3
    sp, Dp = again(E, th + ht)
    sm, Dm = again(E, th - ht)
    assert np.abs((sp - sm) / (2 * ht) - out["dsdt"]).max() <= 1e-5 * np.abs(out["dsdt"]).max()
    assert abs((Dp - Dm) / (2 * ht) - out["dDdt"]) <= 1e-5 * abs(out["dDdt"])
    h = 1e-7
    fd = np.zeros(6)
    for j in range(6):
        dE = np.zeros(6)
        dE[j] = h
        fd[j] = (again(E + dE, th)[1] - again(E - dE, th)[1]) / (2 * h)
    assert np.abs(fd - out["dDde"]).max() <= 1e-5 * np.abs(fd).max()


def test_online_thermoelastic_closed_forms():
    K = 3
    m, v = random_params(K)
    g = glass()
    net = dmn.OnlineDMN(m, v, g, g, tol=1e-13)
    E0 = np.array([1e-3, -2e-4, 3e-4, 1e-4, 0.0, -5e-5])
    net.step(E0, 320.0, 2.0)
    E1 = E0 + np.array([2e-4, 1e-4, -1e-4, 0.0, 3e-5, 0.0])
    out = net.step(E1, 340.0, 0.5, all_tangents=True)
    K_, G_ = tensor.bulk_shear(g["E"], g["nu"])
    Ca = 3 * K_ * g["alpha0"] * np.array([1.0, 1, 1, 0, 0, 0])
    wsum = np.maximum(v, 0).sum()
    assert np.allclose(out["dsdt"], -Ca * wsum, rtol=1e-10)
    assert np.allclose(out["dDde"], -340.0 * Ca / 0.5 * wsum, rtol=1e-10)
    assert np.isclose(out["dDdt"], -(Ca @ tensor.components_to_mandel(E1 - E0)) / 0.5 * wsum, rtol=1e-9)
