"""Pins of the oracle's cell-problem solver against exact results.

* homogeneous material: the effective response is the local law;
* laminates with even layer thickness: the effective stiffness satisfies the
  laminate equation of Sec. 3.2 exactly; the conductivity is the harmonic
  mean across and the arithmetic mean along the layers;
* two-phase thermoelasticity: Levin's formula for the effective expansion;
* any geometry: Voigt/Reuss bounds; for the cubic-symmetric centred sphere
  the Hashin-Shtrikman bounds on bulk modulus and conductivity and cubic
  symmetry of the effective tensors;
* converged fields are equilibrated in Fourier space.
"""
import numpy as np
import pytest

from oracle import fourier, green, solver, tensor
from paper_2109_14403_amd import workloads as W


def te(E, nu, alpha, kappa, c0=2.0, theta0=293.0):
    return dict(kind="thermoelastic", E=E, nu=nu, alpha0=alpha, kappa0=kappa, c0=c0, theta0=theta0)


MAT_A = te(3.0e3, 0.35, 6e-5, 0.2)
MAT_B = te(70.0e3, 0.22, 5e-6, 1.0)


@pytest.mark.parametrize("scheme", ["basic", "newton"])
def test_homogeneous_thermoelastic(scheme):
    phases = np.zeros((6, 6, 6), dtype=np.uint8)
    cell = solver.Cell(phases, [MAT_A])
    strain = np.array([1e-3, -2e-4, 3e-4, 1e-4, -5e-5, 2e-4])
    theta, dt = 313.0, 2.0
    out = cell.solve_increment(strain, theta, [1.0, -2.0, 0.5], dt, scheme=scheme, tol=1e-12)
    K, G = tensor.bulk_shear(MAT_A["E"], MAT_A["nu"])
    tr = strain[:3].sum()
    dth = theta - MAT_A["theta0"]
    expect = 2 * G * strain
    expect[:3] += (3 * K * (tr / 3 - MAT_A["alpha0"] * dth) - 2 * G * tr / 3)
    assert np.allclose(out["stress"], expect, rtol=1e-12, atol=1e-12)
    assert np.allclose(cell.last["eps"], tensor.components_to_mandel(strain)[:, None, None, None], atol=1e-15)
    assert out["iterations"] <= 1
    assert np.allclose(out["heat_flux"], -0.2 * np.array([1.0, -2.0, 0.5]))
    assert np.isclose(out["coupling"], -theta * 3 * K * MAT_A["alpha0"] * tr / dt)
    assert out["dissipation"] == 0.0
    assert out["heat_capacity"] == MAT_A["c0"]


def test_free_thermal_expansion_is_stress_free():
    phases = np.zeros((4, 4, 4), dtype=np.uint8)
    cell = solver.Cell(phases, [MAT_A])
    a = MAT_A["alpha0"] * 20.0
    out = cell.solve_increment(np.array([a, a, a, 0, 0, 0]), 313.0, [0, 0, 0], 1.0, tol=1e-12)
    assert np.allclose(out["stress"], 0.0, atol=1e-12)


def test_homogeneous_pa66_equals_point_law():
    from oracle.laws import PA66
    p = W.pa66()
    phases = np.zeros((4, 4, 4), dtype=np.uint8)
    cell = solver.Cell(phases, [p])
    law = PA66(p)
    st = law.initial_state(1)
    eps_n = np.zeros((6, 1))
    for k, (e11, e12, th) in enumerate([(0.01, 0.004, 300.0), (0.02, 0.008, 320.0), (0.03, 0.01, 340.0)]):
        strain = np.array([e11, 0, 0, 0, 0, e12])
        out = cell.solve_increment(strain, th, [0, 0, 0], 2.0, tol=1e-12)
        E = tensor.components_to_mandel(strain)[:, None]
        pt = law.update(E, eps_n, st, th, 2.0)
        st, eps_n = pt["state"], E
        assert np.allclose(out["stress"], tensor.mandel_to_components(pt["sigma"][:, 0]), rtol=1e-10, atol=1e-10)
        assert np.isclose(out["dissipation"], pt["dissipation"][0], rtol=1e-10)
        assert np.isclose(out["coupling"], pt["coupling"][0], rtol=1e-10)
    assert pt["delta"][0] > 0.0     # the last increment flows plastically


def laminate_equation_stiffness(C1, C2, c1, n, lam):
    """Solve (P + lam [Cb - lam I]^-1)^-1 = c1 (P + lam [C1 - lam I]^-1)^-1 + c2 (...)^-1 for Cb
    (Sec. 3.2, laminate homogenization)."""
    I = np.eye(6)
    nn = np.asarray(n, dtype=float)
    P = np.array([green.projector(I[:, j:j + 1], nn[:, None])[:, 0] for j in range(6)]).T
    A = lambda C: np.linalg.inv(P + lam * np.linalg.inv(C - lam * I))
    rhs = c1 * A(C1) + (1.0 - c1) * A(C2)
    return lam * I + lam * np.linalg.inv(np.linalg.inv(rhs) - P)


@pytest.mark.parametrize("axis,n,bounds", [(0, 8, [2, 6]), (1, 10, [0, 4]), (2, 12, [2, 4, 8, 10])])
def test_laminate_stiffness_and_conductivity(axis, n, bounds):
    shape = [n, n, n]
    img = W.laminate(tuple(shape), bounds, axis=axis)
    cell = solver.Cell(img, [MAT_A, MAT_B])
    Cb = cell.effective_stiffness(tol=1e-13)
    c_b = img.mean()
    la = cell.laws
    lam = 0.5 * min(np.linalg.eigvalsh(la[0].C).min(), np.linalg.eigvalsh(la[1].C).min())
    direction = np.eye(3)[axis]
    expect = laminate_equation_stiffness(la[1].C, la[0].C, c_b, direction, lam)
    assert np.allclose(Cb, expect, rtol=1e-9, atol=1e-9 * np.abs(expect).max())
    kb = cell.effective_conductivity(tol=1e-13)
    harm = 1.0 / (c_b / 1.0 + (1 - c_b) / 0.2)
    arith = c_b * 1.0 + (1 - c_b) * 0.2
    expect_k = np.full(3, arith)
    expect_k[axis] = harm
    assert np.allclose(kb, np.diag(expect_k), atol=1e-10)


def test_odd_grid_laminate():
    img = W.laminate((9, 5, 5), [0, 4], axis=0)     # 4 of 9 layers: any thickness is exact on odd n
    cell = solver.Cell(img, [MAT_A, MAT_B])
    Cb = cell.effective_stiffness(tol=1e-13)
    la = cell.laws
    lam = 0.5 * min(np.linalg.eigvalsh(la[0].C).min(), np.linalg.eigvalsh(la[1].C).min())
    expect = laminate_equation_stiffness(la[1].C, la[0].C, img.mean(), [1, 0, 0], lam)
    assert np.allclose(Cb, expect, rtol=1e-9, atol=1e-9 * np.abs(expect).max())


def levin_expansion(Cb, laws):
    """Levin: alpha_b = alpha1 + (Sb - S1)(S2 - S1)^-1 (alpha2 - alpha1), S = C^-1."""
    S1, S2 = np.linalg.inv(laws[0].C), np.linalg.inv(laws[1].C)
    Sb = np.linalg.inv(Cb)
    return laws[0].alpha + (Sb - S1) @ np.linalg.inv(S2 - S1) @ (laws[1].alpha - laws[0].alpha)


@pytest.mark.parametrize("geometry", ["laminate", "sphere"])
def test_levin_effective_expansion(geometry):
    if geometry == "laminate":
        img = W.laminate((8, 8, 8), [2, 6], axis=1)
    else:
        img = W.centred_sphere(8, 2.6)
    cell = solver.Cell(img, [MAT_A, MAT_B])
    Cb = cell.effective_stiffness(tol=1e-13)
    dth = 40.0
    out = cell.solve_increment(np.zeros(6), MAT_A["theta0"] + dth, [0, 0, 0], 1.0, tol=1e-13,
                               cg_rtol=1e-6)
    alpha_b = -np.linalg.solve(Cb, tensor.components_to_mandel(out["stress"])) / dth
    assert np.allclose(alpha_b, levin_expansion(Cb, cell.laws), rtol=1e-8, atol=1e-13)


@pytest.fixture(scope="module")
def sphere16():
    wl = W.small_sphere_workload()
    cell = solver.Cell(wl.phases, wl.laws)
    return cell, cell.effective_stiffness(tol=1e-12), cell.effective_conductivity(tol=1e-12), wl


def hs_bulk(K1, G1, K2, G2, c2):
    """Hashin-Shtrikman bulk bounds (phase 2 stiffer)."""
    c1 = 1 - c2
    lo = K1 + c2 / (1 / (K2 - K1) + 3 * c1 / (3 * K1 + 4 * G1))
    hi = K2 + c1 / (1 / (K1 - K2) + 3 * c2 / (3 * K2 + 4 * G2))
    return lo, hi


def hs_conductivity(k1, k2, c2):
    c1 = 1 - c2
    lo = k1 + c2 / (1 / (k2 - k1) + c1 / (3 * k1))
    hi = k2 + c1 / (1 / (k1 - k2) + c2 / (3 * k2))
    return lo, hi


def test_sphere_bounds_and_symmetry(sphere16):
    cell, Cb, kb, wl = sphere16
    la = cell.laws
    c2 = wl.phases.mean()
    assert wl.phases.sum() == 840
    Cv = (1 - c2) * la[0].C + c2 * la[1].C
    Cr = np.linalg.inv((1 - c2) * np.linalg.inv(la[0].C) + c2 * np.linalg.inv(la[1].C))
    assert np.linalg.eigvalsh(Cv - Cb).min() > 0
    assert np.linalg.eigvalsh(Cb - Cr).min() > 0
    assert np.allclose(Cb, Cb.T, atol=1e-9 * np.abs(Cb).max())
    # cubic symmetry
    d = np.diag(Cb)
    assert np.allclose(d[:3], d[0], rtol=1e-9) and np.allclose(d[3:], d[3], rtol=1e-9)
    assert np.isclose(Cb[0, 1], Cb[0, 2], rtol=1e-9) and np.isclose(Cb[1, 2], Cb[0, 1], rtol=1e-9)
    assert np.abs(Cb[:3, 3:]).max() < 1e-9 * np.abs(Cb).max()
    # bulk modulus of the cubic effective tensor within the Hashin-Shtrikman bounds
    Kb = Cb[:3, :3].sum() / 9.0
    lo, hi = hs_bulk(la[0].K, la[0].G, la[1].K, la[1].G, c2)
    assert lo < Kb < hi
    # cubic conductivity is isotropic, within Hashin-Shtrikman
    assert np.allclose(kb, kb[0, 0] * np.eye(3), atol=1e-10)
    klo, khi = hs_conductivity(0.2, 1.0, c2)
    assert klo < kb[0, 0] < khi


def test_basic_scheme_and_newton_agree_on_sphere(sphere16):
    _, _, _, wl = sphere16
    a = solver.Cell(wl.phases, wl.laws)
    b = solver.Cell(wl.phases, wl.laws)
    for st in wl.history[:2]:
        ra = a.solve_increment(st.strain, st.theta, st.grad, st.dt, scheme="basic", tol=1e-11)
        rb = b.solve_increment(st.strain, st.theta, st.grad, st.dt, scheme="newton", tol=1e-11)
        assert np.allclose(ra["stress"], rb["stress"], rtol=1e-8, atol=1e-8)
        assert np.allclose(ra["heat_flux"], rb["heat_flux"], rtol=1e-8)
        assert np.isclose(ra["coupling"], rb["coupling"], rtol=1e-8)


def test_effective_response_uses_effective_stiffness(sphere16):
    """Linear thermoelastic composite: <sigma> = Cb (E - alpha_b dth)."""
    cell0, Cb, kb, wl = sphere16
    cell = solver.Cell(wl.phases, wl.laws)
    st = wl.history[0]
    out = cell.solve_increment(st.strain, st.theta, st.grad, st.dt, scheme="newton", tol=1e-12,
                               cg_rtol=1e-6)
    alpha_b = levin_expansion(Cb, cell.laws)
    E = tensor.components_to_mandel(st.strain)
    expect = Cb @ (E - alpha_b * (st.theta - 293.0))
    assert np.allclose(tensor.components_to_mandel(out["stress"]), expect, rtol=1e-8, atol=1e-8)
    assert np.allclose(out["heat_flux"], -kb @ st.grad, rtol=1e-8)


def test_equilibrium_in_fourier_space():
    wl = W.sphere_composite_workload(16, seed=2)
    cell = solver.Cell(wl.phases, wl.laws)
    tol = 1e-9
    for st in wl.history[:3]:
        cell.solve_increment(st.strain, st.theta, st.grad, st.dt, tol=tol)
    sig = cell.last["sigma"]
    S = fourier.fft3(sig)
    t = tensor.mandel_to_matrix(S)
    div = np.einsum("ij...,j...->i...", t, cell.n)
    rel = np.abs(div).max() / (sig[0].size * np.linalg.norm(sig.reshape(6, -1).mean(1)))
    assert rel <= 10 * tol
    assert np.all(cell.last["dissipation"] >= 0.0)
