"""Pins of the oracle's PA66 dissipation and coupling term (Sec. 4) against
the printed free energy, with no use of the oracle's own 𝒟 / D formulas.

The paper defines the dissipation as minus the internal-variable derivative of
the free energy times the rates (Sec. 2, effective dissipation; Sec. 3.3,
phase-wise dissipation), and for PA66 it prints the evaluated form
σ_Y ε̇_p + Σ σ_v,i : ε̇_v,i (Sec. 4, dissipation). The coupling term is the
dissipation plus θ times the mixed temperature derivatives of the free energy
along the rates (Sec. 4, coupling term). Each check below derives its expected
value from central differences of ``PA66.free_energy`` (the printed Helmholtz
energy, eq. helmholtz_PA66 plus the heat part) or from a closed-form steady
state, and each is chosen so that a plausible slip in the oracle fails it:

* Maxwell part: branch stresses at step n instead of n+1 (the implicit
  reading, A9) fails the gradient pin and the energy-balance sign;
* plastic part: a wrong factor on σ_Y ε̇_p fails the rate-independent limit
  and the steady shear flow;
* coupling: a flipped sign or factor on the softening term θ ∂H/∂θ ε̇_p
  fails the difference quotient of ∂ψ/∂θ.
"""
import numpy as np
import pytest

from oracle import tensor
from oracle.laws import PA66
from paper_2109_14403_amd import workloads as W


def _state_copy(st):
    return dict(ep=st["ep"].copy(), evp=st["evp"].copy(), ev=st["ev"].copy())


def free_energy_gradient_z(law, eps, st, theta, h=1e-7):
    """Central differences of the free energy in every internal variable
    (ε_p, the six Mandel components of ε_vp, those of each ε_v,i)."""
    grad = dict(ep=np.zeros_like(st["ep"]), evp=np.zeros_like(st["evp"]), ev=np.zeros_like(st["ev"]))
    # ε_p: forward-safe central difference where ε_p > h (H is an ε_p power law)
    sp = _state_copy(st); sm = _state_copy(st)
    live = st["ep"] > 2 * h
    sp["ep"] = np.where(live, st["ep"] + h, st["ep"])
    sm["ep"] = np.where(live, st["ep"] - h, st["ep"])
    grad["ep"] = np.where(live, (law.free_energy(eps, sp, theta) - law.free_energy(eps, sm, theta)) / (2 * h), 0.0)
    for a in range(6):
        sp = _state_copy(st); sm = _state_copy(st)
        sp["evp"][a] += h; sm["evp"][a] -= h
        grad["evp"][a] = (law.free_energy(eps, sp, theta) - law.free_energy(eps, sm, theta)) / (2 * h)
    for i in range(law.N):
        for a in range(6):
            sp = _state_copy(st); sm = _state_copy(st)
            sp["ev"][i, a] += h; sm["ev"][i, a] -= h
            grad["ev"][i, a] = (law.free_energy(eps, sp, theta) - law.free_energy(eps, sm, theta)) / (2 * h)
    return grad


def dpsi_dtheta(law, eps, st, theta, h=1e-3):
    return (law.free_energy(eps, st, theta + h) - law.free_energy(eps, st, theta - h)) / (2 * h)


def plastic_start(law, m, rng, ep0=0.05):
    """Step-n state with accumulated plastic strain and loaded Maxwell branches."""
    st = law.initial_state(m)
    st["ep"] = np.full(m, ep0)
    st["evp"] = tensor.deviator(rng.normal(scale=2e-3, size=(6, m)))
    st["ev"] = rng.normal(scale=1e-3, size=(law.N, 6, m))
    return st


def test_maxwell_dissipation_is_free_energy_gradient_at_new_state():
    """Without plastic flow: 𝒟 = -Σ ∂ψ/∂ε_v,i(z^{n+1}) · Δε_v,i / Δt (branch stresses
    at the new time level, reading A9)."""
    p = W.pa66()
    p["sigma_y0"] = 1e12
    law = PA66(p)
    rng = np.random.default_rng(11)
    m = 6
    st = plastic_start(law, m, rng, ep0=0.0)
    st["evp"][:] = 0.0
    eps_n = rng.normal(scale=3e-3, size=(6, m))
    eps = eps_n + rng.normal(scale=2e-3, size=(6, m))
    for theta, dt in [(300.0, 0.8), (350.0, 2.0), (372.0, 1e-2)]:
        out = law.update(eps, eps_n, st, theta, dt)
        assert np.all(out["delta"] == 0.0)
        g = free_energy_gradient_z(law, eps, out["state"], theta)
        expect = -(g["ev"] * (out["state"]["ev"] - st["ev"])).sum(axis=(0, 1)) / dt
        assert np.all(expect > 0.0)
        assert np.allclose(out["dissipation"], expect, rtol=1e-6, atol=0.0)
        # the same product at the old state differs visibly: the pin tells n from n+1
        g_old = free_energy_gradient_z(law, eps, st, theta)
        old = -(g_old["ev"] * (out["state"]["ev"] - st["ev"])).sum(axis=(0, 1)) / dt
        assert np.all(np.abs(old - expect) > 1e-3 * np.abs(expect))


@pytest.mark.parametrize("theta", [298.15, 340.0])
def test_maxwell_relaxation_energy_balance(theta):
    """Held strain, fixed θ, no plastic flow: the work input is zero, so the
    dissipated energy Σ 𝒟 Δt approaches the drop of the free energy at first
    order in Δt, from below (implicit Euler with branch stresses at n+1; per
    step the gap is the quadratic remainder ½ Δε_v : C_i Δε_v ≥ 0)."""
    p = W.pa66()
    p["sigma_y0"] = 1e12
    # three branches whose relaxation times the steps resolve at both temperatures
    p["E_i"] = p["E_i"][5:8]
    p["log10_tau_i"] = p["log10_tau_i"][5:8]
    law = PA66(p)
    eps = np.zeros((6, 1))
    eps[0, 0] = 2e-3
    eps[5, 0] = 1.5e-3 * np.sqrt(2)
    d = theta - p["theta_ref"]
    a = 10.0 ** (-p["C1"] * d / (p["C2"] + d))           # WLF shift (Sec. 4)
    T = 2.0 * a * 10.0 ** p["log10_tau_i"][1] * 2.0 * (1.0 + p["nu"])
    gaps = []
    for steps in (400, 800, 1600):
        dt = T / steps
        st = law.initial_state(1)
        psi0 = law.free_energy(eps, st, theta)[0]
        eps_n = eps.copy()                        # the strain is applied before t = 0
        total = 0.0
        for _ in range(steps):
            out = law.update(eps, eps_n, st, theta, dt)
            total += out["dissipation"][0] * dt
            st_prev, st = st, out["state"]
            # exact per-step identity of a quadratic energy
            step_drop = law.free_energy(eps, st_prev, theta)[0] - law.free_energy(eps, st, theta)[0]
            mirror = _state_copy(st)
            mirror["ev"] = 2 * st["ev"] - st_prev["ev"]
            quad = 0.5 * (law.free_energy(eps, st_prev, theta)[0] - 2 * law.free_energy(eps, st, theta)[0]
                          + law.free_energy(eps, mirror, theta)[0])
            assert quad > 0.0
            assert abs(step_drop - out["dissipation"][0] * dt - quad) <= 1e-7 * abs(step_drop) + 1e-15
        drop = psi0 - law.free_energy(eps, st, theta)[0]
        assert drop > 0.0
        gaps.append(drop - total)
    assert all(g > 0.0 for g in gaps)
    assert gaps[-1] < 2e-2 * drop
    assert 1.7 < gaps[0] / gaps[1] < 2.3 and 1.7 < gaps[1] / gaps[2] < 2.3


def test_plastic_dissipation_in_rate_independent_limit():
    """The general definition -∂ψ/∂z · ż (Sec. 2) and the printed PA66 form
    σ_Y ε̇_p + Σ σ_v,i : ε̇_v,i (Sec. 4) differ by the overstress times ε̇_p
    (reading A5). As the viscosity vanishes the overstress does, so the two
    must meet: at η₀ → 0 the oracle's 𝒟 equals the free-energy gradient
    product over all internal variables, and the gap shrinks like η₀^{1/m}."""
    m = 4
    rel = []
    for scale in (1e-4, 1e-8):
        p = W.pa66()
        p["eta0"] = p["eta0"] * scale
        law = PA66(p)
        st = plastic_start(law, m, np.random.default_rng(5), ep0=0.03)
        r2 = np.random.default_rng(6)
        eps_n = r2.normal(scale=3e-3, size=(6, m))
        push = tensor.deviator(r2.normal(size=(6, m)))
        eps = eps_n + 4e-2 * push / tensor.norm(push)
        theta, dt = 320.0, 1.0
        out = law.update(eps, eps_n, st, theta, dt)
        assert np.all(out["delta"] > 0.0)
        new = out["state"]
        g = free_energy_gradient_z(law, eps, new, theta)
        general = -((g["ep"] * (new["ep"] - st["ep"]))
                    + (g["evp"] * (new["evp"] - st["evp"])).sum(0)
                    + (g["ev"] * (new["ev"] - st["ev"])).sum(axis=(0, 1))) / dt
        gap = general - out["dissipation"]
        assert np.all(gap > -1e-6 * general)
        rel.append(gap / general)
    rel = np.array(rel)
    assert np.all(np.abs(rel[1]) < 1e-4)
    # gap ∝ η₀^{1/m} with m = 2: a factor 1e4 in η₀ is 1e2 in the gap
    ratio = rel[0] / rel[1]
    assert np.all((ratio > 50.0) & (ratio < 200.0))


def test_steady_shear_flow_dissipation_without_branches():
    """No Maxwell branches, no hardening, constant shear rate: at steady state
    all plastic, ε̇_p = 2 γ̇ / √3 for ε̇_12 = γ̇, and the printed dissipation is
    the yield stress of the softening law times that rate. The shear keeps the
    trace at zero and H ≡ 0, so the coupling term equals the dissipation."""
    p = W.pa66()
    p["E_i"] = []
    p["log10_tau_i"] = []
    p["k_h"] = 0.0
    law = PA66(p)
    theta, rate, dt = 345.0, 2e-3, 0.05
    st = law.initial_state(1)
    eps_n = np.zeros((6, 1))
    for k in range(1, 3001):
        eps = np.zeros((6, 1))
        eps[5, 0] = np.sqrt(2) * rate * k * dt
        out = law.update(eps, eps_n, st, theta, dt)
        st, eps_n = out["state"], eps
    sY = np.exp(-p["beta1"] * (theta - p["theta_ref"])) * p["sigma_y0"]   # Sec. 4 yield stress table value
    ep_rate = 2.0 * rate / np.sqrt(3.0)
    assert np.isclose(out["dissipation"][0], sY * ep_rate, rtol=1e-9)
    assert np.isclose(out["coupling"][0], out["dissipation"][0], rtol=1e-12)


@pytest.mark.parametrize("theta, push_size", [(305.0, 3e-2), (360.0, 2e-2)])
def test_coupling_with_plastic_flow_from_free_energy(theta, push_size):
    """D - 𝒟 = θ (∂²ψ/∂θ∂ε : ε̇ + ∂²ψ/∂θ∂z · ż) (Sec. 4, coupling term). ∂ψ/∂θ is
    linear in ε, ε_vp and ε_v,i, so its difference quotient between the two
    states is exact for those parts; the hardening energy ∫H contributes
    ∫ ∂H/∂θ dε_p, which the implicit step takes at ε_p^{n+1}: an O(Δε_p / ε_p)
    relative error on the softening part only. The states start at ε_p = 5 %
    and the plastic increments stay below 2e-3."""
    law = PA66(W.pa66())
    rng = np.random.default_rng(21)
    m = 5
    st = plastic_start(law, m, rng, ep0=0.05)
    eps_n = rng.normal(scale=3e-3, size=(6, m))
    # a large deviatoric push over a short step: plastic flow with small increments
    push = tensor.deviator(rng.normal(size=(6, m)))
    eps = eps_n + push_size * push / tensor.norm(push)
    dt = 1e-5
    out = law.update(eps, eps_n, st, theta, dt)
    new = out["state"]
    assert np.all(out["delta"] > 0.0) and np.all(out["delta"] < 2e-3)
    entropy = theta * (dpsi_dtheta(law, eps, new, theta) - dpsi_dtheta(law, eps_n, st, theta)) / dt
    # the softening part alone: ∂ψ/∂θ moved only through ε_p
    only_ep = _state_copy(st)
    only_ep["ep"] = new["ep"]
    soft = theta * (dpsi_dtheta(law, eps_n, only_ep, theta) - dpsi_dtheta(law, eps_n, st, theta)) / dt
    err = (out["coupling"] - out["dissipation"]) - entropy
    bound = 0.2 * (out["delta"] / new["ep"]) * np.abs(soft) + 1e-7 * np.abs(entropy)
    # sharp enough that a 5 % slip in the softening term (let alone its sign) fails
    assert np.all(bound < 0.05 * np.abs(soft))
    assert np.all(np.abs(err) <= bound), (err / np.abs(soft), out["delta"])
