"""Constitutive laws of the paper's Sec. 4, evaluated voxel by voxel in float64.

Both laws are non-isothermal generalized standard materials (Sec. 2): the
stress is the strain derivative of the Helmholtz free energy and the
internal variables follow Biot's equation. Time is discretised by implicit
Euler (Sec. 3.3, condensed incremental potential): rates are
(x^{n+1} - x^n) / dt and every quantity is taken at the new time level.
The micro temperature is homogeneous and equal to the macro temperature
theta (Sec. 2, micro cell problem).

Arrays: strains and stresses are Mandel vectors of shape (6, M) for M voxels;
tangents are (6, 6, M).
"""
from __future__ import annotations

import numpy as np

from . import tensor
from .tensor import IDENTITY2, P1, P2


class Thermoelastic:
    """Isotropic linear thermoelastic law (Sec. 4, E-glass fibres):
    psi = 1/2 eps:C eps - eps:C[alpha (theta - theta0)] + psi_heat(theta),
    sigma = C[eps - alpha (theta - theta0)], C = 3K P1 + 2G P2, alpha = alpha0 I,
    D = -theta eps_dot : C[alpha] (Gough-Joule), dissipation = 0, c = c0."""

    inelastic = False

    def __init__(self, p: dict):
        self.p = dict(p)
        self.K, self.G = tensor.bulk_shear(p["E"], p["nu"])
        self.C = tensor.isotropic(self.K, self.G)
        self.alpha = p["alpha0"] * IDENTITY2
        self.kappa = p["kappa0"]
        self.c0 = p["c0"]
        self.theta0 = p["theta0"]

    def stress(self, eps, theta):
        th = (theta - self.theta0) * self.alpha
        return self.C @ (eps - th[:, None])

    def tangent(self, m):
        return np.repeat(self.C[:, :, None], m, axis=2)

    def coupling(self, eps, eps_n, theta, dt):
        rate = (eps - eps_n) / dt
        return -theta * ((self.C @ self.alpha) @ rate)

    def free_energy(self, eps, theta):
        th = (theta - self.theta0) * self.alpha
        mech = 0.5 * np.einsum("a...,ab,b...->...", eps, self.C, eps) - eps.T @ (self.C @ th)
        return mech + heat_energy(self.c0, self.theta0, theta)


def heat_energy(c0, theta0, theta):
    """psi_heat = c0 [(theta - theta0) - theta ln(theta / theta0)] (Sec. 4)."""
    return c0 * ((theta - theta0) - theta * np.log(theta / theta0))


class PA66:
    """Thermo-viscoelastic / viscoplastic PA66 law (Sec. 4, eq. helmholtz_PA66 ff.).

    Internal variables z = [eps_p, eps_vp, eps_v_1 .. eps_v_N]:
    accumulated plastic strain, deviatoric viscoplastic strain and the N
    viscous strains of the generalized Maxwell model.
    """

    inelastic = True

    def __init__(self, p: dict):
        self.p = dict(p)
        self.N = len(p["E_i"])
        nu = p["nu"]
        self.Kinf, self.Ginf = tensor.bulk_shear(p["E"], nu)
        self.Cinf = tensor.isotropic(self.Kinf, self.Ginf)
        self.E_i = np.asarray(p["E_i"], dtype=np.float64)
        self.tau_i = 10.0 ** np.asarray(p["log10_tau_i"], dtype=np.float64)
        self.K_i = self.E_i / (3.0 * (1.0 - 2.0 * nu))
        self.G_i = self.E_i / (2.0 * (1.0 + nu))
        self.C_i = [tensor.isotropic(k, g) for k, g in zip(self.K_i, self.G_i)]
        # volumetric and deviatoric relaxation times tau_K = tau E / K, tau_G = tau E / G
        self.tauK = self.tau_i * self.E_i / self.K_i
        self.tauG = self.tau_i * self.E_i / self.G_i
        self.alpha = p["alpha0"] * IDENTITY2
        self.kappa = p["kappa0"]
        self.c0 = p["c0"]
        self.theta0 = p["theta0"]

    # ---- temperature functions -------------------------------------------
    def shift(self, theta):
        """WLF: log10 a = -C1 (theta - theta_ref) / (C2 + theta - theta_ref)."""
        d = theta - self.p["theta_ref"]
        return 10.0 ** (-self.p["C1"] * d / (self.p["C2"] + d))

    def softening(self, theta, beta):
        """Gamma(theta, beta) = exp(-beta (theta - theta_ref))."""
        return np.exp(-beta * (theta - self.p["theta_ref"]))

    def yield_stress(self, theta):
        return self.softening(theta, self.p["beta1"]) * self.p["sigma_y0"]

    def hardening(self, theta, ep):
        return self.softening(theta, self.p["beta1"]) * self.p["k_h"] * np.power(ep, self.p["n_h"])

    def viscosity(self, theta):
        return self.softening(theta, self.p["beta2"]) * self.p["eta0"]

    # ---- state ------------------------------------------------------------
    def initial_state(self, m):
        return dict(ep=np.zeros(m), evp=np.zeros((6, m)), ev=np.zeros((self.N, 6, m)))

    # ---- viscous branch update -------------------------------------------
    def branch_matrices(self, theta, dt):
        """Implicit Euler of eps_v_i' = F_i[sigma_v_i], sigma_v_i = C_i[e - eps_v_i],
        e = eps - eps_vp - alpha (theta - theta0), F_i = V_i^+ (pseudo-inverse),
        V_i = a(theta) (3 K_i tau_K P1 + 2 G_i tau_G P2):
        (I + dt F_i C_i) eps_v^{n+1} = eps_v^n + dt F_i C_i e.
        Returns (B_i, M_i) with eps_v^{n+1} = B_i eps_v^n + M_i e."""
        a = self.shift(theta)
        out = []
        for i in range(self.N):
            V = a * (3.0 * self.K_i[i] * self.tauK[i] * P1 + 2.0 * self.G_i[i] * self.tauG[i] * P2)
            F = np.linalg.pinv(V)
            A = np.eye(6) + dt * F @ self.C_i[i]
            B = np.linalg.inv(A)
            out.append((B, B @ (dt * F @ self.C_i[i])))
        return out

    def stress_from_state(self, eps, evp, ev, theta):
        """sigma = C_inf[eps - eps_vp - alpha dth] + sum C_i[eps - eps_vp - eps_v_i - alpha dth]."""
        th = ((theta - self.theta0) * self.alpha)[:, None]
        e = eps - evp - th
        sig = self.Cinf @ e
        for i in range(self.N):
            sig = sig + self.C_i[i] @ (e - ev[i])
        return sig

    def free_energy(self, eps, state, theta):
        """Helmholtz free energy, eq. helmholtz_PA66 plus the heat part."""
        th = ((theta - self.theta0) * self.alpha)[:, None]
        e = eps - state["evp"]
        psi = 0.5 * (e * (self.Cinf @ e)).sum(0) - (e * (self.Cinf @ th)).sum(0)
        g1 = self.softening(theta, self.p["beta1"])
        psi = psi + g1 * self.p["k_h"] * np.power(state["ep"], self.p["n_h"] + 1.0) / (self.p["n_h"] + 1.0)
        for i in range(self.N):
            ei = e - state["ev"][i]
            psi = psi + 0.5 * (ei * (self.C_i[i] @ ei)).sum(0) - (ei * (self.C_i[i] @ th)).sum(0)
        return psi + heat_energy(self.c0, self.theta0, theta)

    def update(self, eps, eps_n, state, theta, dt, bisect_steps=200):
        """One implicit Euler step at fixed strain eps (6, M) from state z^n.

        Returns dict(sigma, tangent, state, dissipation, coupling, delta)."""
        m = eps.shape[1]
        mats = self.branch_matrices(theta, dt)
        th = ((theta - self.theta0) * self.alpha)[:, None]
        sY = self.yield_stress(theta)
        eta = self.viscosity(theta)
        mexp = self.p["m"]
        ep_n = state["ep"]
        evp_n = state["evp"]
        ev_n = state["ev"]

        def branches(evp):
            e = eps - evp - th
            return np.stack([B @ ev_n[i] + M @ e for i, (B, M) in enumerate(mats)]) if self.N else \
                np.zeros((0, 6, m))

        # trial: no viscoplastic increment
        ev_tr = branches(evp_n)
        s_tr = tensor.deviator(self.stress_from_state(eps, evp_n, ev_tr, theta))
        s_norm = tensor.norm(s_tr)
        seq_tr = np.sqrt(1.5) * s_norm
        f = seq_tr - sY - self.hardening(theta, ep_n)
        plastic = f > 0.0
        Nd = np.where(s_norm > 0.0, s_tr / np.where(s_norm > 0.0, s_norm, 1.0), 0.0)

        # change of the deviatoric stress per unit plastic increment, from the stress formula
        ev_1 = branches(evp_n + np.sqrt(1.5) * Nd)
        dS = tensor.deviator(self.stress_from_state(eps, evp_n + np.sqrt(1.5) * Nd, ev_1, theta)) - s_tr
        slope = np.sqrt(1.5) * tensor.norm(dS)           # = -d sigma_eq / d delta

        def g(delta, idx):
            seq = np.sqrt(1.5) * tensor.norm(s_tr[:, idx] + delta * dS[:, idx])
            over = (seq - sY - self.hardening(theta, ep_n[idx] + delta)) / sY
            return delta - dt * (sY / eta) * np.power(np.maximum(over, 0.0), mexp)

        delta = np.zeros(m)
        idx = np.nonzero(plastic)[0]
        if idx.size:
            lo = np.zeros(idx.size)
            hi = f[idx] / slope[idx]
            for _ in range(bisect_steps):
                mid = 0.5 * (lo + hi)
                gm = g(mid, idx)
                lo = np.where(gm < 0.0, mid, lo)
                hi = np.where(gm < 0.0, hi, mid)
                if np.all(hi - lo <= 1e-15 * np.maximum(hi, 1e-300)):
                    break
            delta[idx] = 0.5 * (lo + hi)

        ep = ep_n + delta
        evp = evp_n + np.sqrt(1.5) * delta[None] * Nd
        ev = branches(evp)
        sig = self.stress_from_state(eps, evp, ev, theta)

        # ---- algorithmic tangent ------------------------------------------
        Cve = self.Cinf.copy()
        for i, (B, M) in enumerate(mats):
            Cve = Cve + self.C_i[i] @ (np.eye(6) - M)
        tangent = np.repeat(Cve[:, :, None], m, axis=2)
        if idx.size:
            PC = P2 @ Cve                                   # d s_tr / d eps
            Np = Nd[:, idx]
            sn = s_norm[idx]
            dN = np.einsum("abk,bc->ack", (np.eye(6)[:, :, None] - np.einsum("ak,bk->abk", Np, Np))
                           / sn[None, None], PC)
            dseq = np.sqrt(1.5) * np.einsum("ak,ab->bk", Np, PC)
            dl = delta[idx]
            over = (np.sqrt(1.5) * tensor.norm(s_tr[:, idx] + dl * dS[:, idx]) - sY
                    - self.hardening(theta, ep[idx])) / sY
            c = dt * sY / eta
            dH = (self.softening(theta, self.p["beta1"]) * self.p["k_h"] * self.p["n_h"]
                  * np.power(ep[idx], self.p["n_h"] - 1.0))
            w = c * mexp * np.power(np.maximum(over, 0.0), mexp - 1.0) / sY
            g_d = 1.0 + w * (slope[idx] + dH)
            ddelta = (w / g_d)[None] * dseq                  # d delta / d eps
            devp = np.sqrt(1.5) * (np.einsum("ak,bk->abk", Np, ddelta) + dl[None, None] * dN)
            tangent[:, :, idx] = np.einsum("ab,bck->ack", Cve, np.eye(6)[:, :, None] - devp)

        # ---- dissipation and thermomechanical coupling ---------------------
        e_new = eps - evp - th
        ep_rate = delta / dt
        diss = self.yield_stress(theta) * ep_rate
        for i in range(self.N):
            sv = self.C_i[i] @ (e_new - ev[i])
            diss = diss + (sv * (ev[i] - ev_n[i])).sum(0) / dt
        eps_rate = (eps - eps_n) / dt
        evp_rate = (evp - evp_n) / dt
        Ca = self.Cinf @ self.alpha
        coup = -theta * ((eps_rate - evp_rate) * Ca[:, None]).sum(0)
        for i in range(self.N):
            Cia = self.C_i[i] @ self.alpha
            coup = coup - theta * ((eps_rate - evp_rate - (ev[i] - ev_n[i]) / dt) * Cia[:, None]).sum(0)
        dHdth = -self.p["beta1"] * self.hardening(theta, ep)
        coup = coup + theta * dHdth * ep_rate + diss

        return dict(sigma=sig, tangent=tangent, state=dict(ep=ep, evp=evp, ev=ev),
                    dissipation=diss, coupling=coup, delta=delta)


def make_law(p: dict):
    kind = p["kind"]
    if kind == "thermoelastic":
        return Thermoelastic(p)
    if kind == "pa66":
        return PA66(p)
    raise ValueError(f"unknown law kind {kind}")
