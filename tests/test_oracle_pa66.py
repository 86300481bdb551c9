"""Pins of the oracle's PA66 law (Sec. 4) against what the paper fixes.

* the stress is the strain derivative of the printed free energy;
* the entropy part of the coupling term and the heat capacity are the
  temperature derivatives of that free energy;
* viscoelastic branches relax exponentially with the printed relaxation
  times and WLF shift (implicit Euler converges to the exact ODE solution);
* steady viscoplastic flow under a constant shear rate reaches the overstress
  of the printed flow rule; for vanishing viscosity the consistency
  condition sigma_eq = sigma_Y + H holds;
* dissipation is non-negative; the algorithmic tangent is the derivative of
  the incremental stress (central differences).
"""
import numpy as np
import pytest

from oracle import tensor
from oracle.laws import PA66, Thermoelastic
from paper_2109_14403_amd import workloads as W


def random_state(law, m, rng, scale=2e-3):
    st = law.initial_state(m)
    st["ep"] = rng.uniform(0.0, 0.02, size=m)
    st["evp"] = tensor.deviator(rng.normal(scale=scale, size=(6, m)))
    st["ev"] = rng.normal(scale=scale, size=(law.N, 6, m))
    return st


def test_stress_is_free_energy_derivative():
    law = PA66(W.pa66())
    rng = np.random.default_rng(0)
    m = 5
    st = random_state(law, m, rng)
    eps = rng.normal(scale=5e-3, size=(6, m))
    theta = 331.0
    sig = law.stress_from_state(eps, st["evp"], st["ev"], theta)
    h = 1e-6
    fd = np.zeros_like(sig)
    for a in range(6):
        ep = eps.copy(); ep[a] += h
        em = eps.copy(); em[a] -= h
        fd[a] = (law.free_energy(ep, st, theta) - law.free_energy(em, st, theta)) / (2 * h)
    assert np.allclose(sig, fd, rtol=1e-6, atol=1e-6)


def test_thermoelastic_stress_and_coupling_from_free_energy():
    law = Thermoelastic(W.e_glass())
    rng = np.random.default_rng(1)
    eps = rng.normal(scale=1e-3, size=(6, 3))
    eps_n = rng.normal(scale=1e-3, size=(6, 3))
    theta, dt, h = 320.0, 0.5, 1e-6
    fd = np.zeros_like(eps)
    for a in range(6):
        ep = eps.copy(); ep[a] += h
        em = eps.copy(); em[a] -= h
        fd[a] = (law.free_energy(ep, theta) - law.free_energy(em, theta)) / (2 * h)
    assert np.allclose(law.stress(eps, theta), fd, rtol=1e-6, atol=1e-4)
    # D = theta d2psi/dtheta deps : eps_dot; psi is linear in theta -> difference quotient is exact
    ht = 1e-3
    dpsi = lambda e: (law.free_energy(e, theta + ht) - law.free_energy(e, theta - ht)) / (2 * ht)
    D_fd = theta * (dpsi(eps) - dpsi(eps_n)) / dt
    assert np.allclose(law.coupling(eps, eps_n, theta, dt), D_fd, rtol=1e-5)


def test_heat_capacity_from_free_energy():
    law = PA66(W.pa66())
    st = law.initial_state(1)
    eps = np.full((6, 1), 1e-3)
    theta, h = 340.0, 1e-2
    f = lambda t: law.free_energy(eps, st, t)[0]
    d2 = (f(theta + h) - 2 * f(theta) + f(theta - h)) / h ** 2
    assert np.isclose(-theta * d2, W.pa66()["c0"], rtol=1e-4)


def one_branch_params(theta_ref=298.15):
    p = W.pa66()
    p["E_i"] = [400.0]
    p["log10_tau_i"] = [0.0]
    p["sigma_y0"] = 1e12        # no viscoplastic flow
    p["theta_ref"] = theta_ref
    return p


@pytest.mark.parametrize("theta", [298.15, 330.0])
def test_maxwell_relaxation_converges_to_exponential(theta):
    p = one_branch_params()
    law = PA66(p)
    d = theta - p["theta_ref"]
    a = 10.0 ** (-p["C1"] * d / (p["C2"] + d))           # WLF, Sec. 4
    tau = 1.0
    tauG = tau * 2.0 * (1.0 + p["nu"])                   # tau E / G
    tauK = tau * 3.0 * (1.0 - 2.0 * p["nu"])             # tau E / K
    T = 0.7 * a * tauG
    for steps in (400, 800):
        dt = T / steps
        eps = np.zeros((6, 1))
        eps[5, 0] = 2e-3 * np.sqrt(2)                     # shear step, held
        eps[0, 0] = 1e-3                                  # plus a volumetric part
        st = law.initial_state(1)
        eps_n = np.zeros((6, 1))
        for _ in range(steps):
            out = law.update(eps, eps_n, st, theta, dt)
            st, eps_n = out["state"], eps
        ev = st["ev"][0][:, 0]
        dev_expect = tensor.deviator(eps[:, 0]) * (1.0 - np.exp(-T / (a * tauG)))
        sph_expect = (eps[0, 0] / 3 - p["alpha0"] * (theta - p["theta0"])) * (1.0 - np.exp(-T / (a * tauK)))
        err_dev = np.abs(tensor.deviator(ev) - dev_expect).max() / np.abs(dev_expect).max()
        err_sph = abs(ev[:3].sum() / 3 - sph_expect) / abs(sph_expect)
        if steps == 400:
            e1 = (err_dev, err_sph)
    # first-order convergence of implicit Euler towards the exact exponential
    assert err_dev < 2e-3 and err_sph < 2e-3
    assert 1.7 < e1[0] / err_dev < 2.3 and 1.7 < e1[1] / err_sph < 2.3


def perzyna_params(k_h=0.0, eta0=74.0):
    p = W.pa66()
    p["E_i"] = []
    p["log10_tau_i"] = []
    p["k_h"] = k_h
    p["eta0"] = eta0
    return p


def test_steady_viscoplastic_shear_flow():
    p = perzyna_params()
    law = PA66(p)
    theta = 310.0
    rate = 1e-3                                   # d eps_12 / dt
    dt = 0.05
    st = law.initial_state(1)
    eps_n = np.zeros((6, 1))
    for k in range(1, 4001):
        eps = np.zeros((6, 1))
        eps[5, 0] = np.sqrt(2) * rate * k * dt
        out = law.update(eps, eps_n, st, theta, dt)
        st, eps_n = out["state"], eps
    s12 = out["sigma"][5, 0] / np.sqrt(2)
    sY = np.exp(-p["beta1"] * (theta - p["theta_ref"])) * p["sigma_y0"]
    eta = np.exp(-p["beta2"] * (theta - p["theta_ref"])) * p["eta0"]
    ep_rate = 2.0 * rate / np.sqrt(3.0)
    seq = sY + sY * (eta * ep_rate / sY) ** (1.0 / p["m"])
    assert np.isclose(np.sqrt(3.0) * s12, seq, rtol=1e-9)
    assert np.isclose(out["delta"][0] / dt, ep_rate, rtol=1e-9)


def test_rate_independent_limit_consistency():
    p = perzyna_params(k_h=103.0, eta0=1e-7)
    law = PA66(p)
    theta = 300.0
    st = law.initial_state(1)
    eps_n = np.zeros((6, 1))
    for k in range(1, 60):
        eps = np.zeros((6, 1))
        eps[0, 0] = 1e-3 * k
        eps[5, 0] = 5e-4 * k
        out = law.update(eps, eps_n, st, theta, 1.0)
        st, eps_n = out["state"], eps
    s = tensor.deviator(out["sigma"][:, 0])
    seq = np.sqrt(1.5) * np.linalg.norm(s)
    g1 = np.exp(-p["beta1"] * (theta - p["theta_ref"]))
    assert st["ep"][0] > 0.01
    assert np.isclose(seq, g1 * (p["sigma_y0"] + p["k_h"] * st["ep"][0] ** p["n_h"]), rtol=1e-4)
    # flow direction is the deviatoric stress direction
    devp = st["evp"][:, 0]
    assert abs(np.dot(devp, s) / (np.linalg.norm(devp) * np.linalg.norm(s))) > 0.99


def test_dissipation_nonnegative_and_tangent_matches_finite_differences():
    law = PA66(W.pa66())
    rng = np.random.default_rng(7)
    m = 40
    st = random_state(law, m, rng)
    eps_n = rng.normal(scale=3e-3, size=(6, m))
    st["ep"][: m // 2] = 0.0
    eps = eps_n + rng.normal(size=(6, m)) * np.logspace(-5, -1.5, m)[None]
    for theta, dt in [(300.0, 2.0), (370.0, 0.5), (293.15, 1e-3)]:
        out = law.update(eps, eps_n, st, theta, dt)
        assert np.all(out["dissipation"] >= 0.0)
        assert np.any(out["delta"] > 0) and np.any(out["delta"] == 0)
        h = 1e-7
        fd = np.zeros((6, 6, m))
        for b in range(6):
            ep = eps.copy(); ep[b] += h
            em = eps.copy(); em[b] -= h
            fd[:, b] = (law.update(ep, eps_n, st, theta, dt)["sigma"]
                        - law.update(em, eps_n, st, theta, dt)["sigma"]) / (2 * h)
        scale = np.abs(out["tangent"]).max()
        assert np.abs(out["tangent"] - fd).max() <= 1e-5 * scale


def test_coupling_entropy_part_from_free_energy_without_plastic_flow():
    p = W.pa66()
    p["sigma_y0"] = 1e12
    law = PA66(p)
    rng = np.random.default_rng(4)
    m = 4
    st = random_state(law, m, rng)
    st["ep"][:] = 0.0
    st["evp"][:] = 0.0
    eps_n = rng.normal(scale=3e-3, size=(6, m))
    eps = eps_n + rng.normal(scale=3e-3, size=(6, m))
    theta, dt, h = 340.0, 0.3, 1e-3
    out = law.update(eps, eps_n, st, theta, dt)
    dpsi = lambda e, s: (law.free_energy(e, s, theta + h) - law.free_energy(e, s, theta - h)) / (2 * h)
    entropy = theta * (dpsi(eps, out["state"]) - dpsi(eps_n, st)) / dt
    assert np.allclose(out["coupling"] - out["dissipation"], entropy, rtol=1e-6, atol=1e-9)
