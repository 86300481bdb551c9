"""The thermomechanical cell problem on a periodic voxel grid, plainly.

Sec. 2 (micro cell problem): for a prescribed macro strain E and a
homogeneous temperature theta, find a periodic displacement fluctuation u
such that div sigma(E + grad_s u, theta, z) = 0. On the voxel grid with the
trigonometric collocation of Moulinec and Suquet (cited in Sec. 5.2/5.4) this
is: find a strain field eps with mean E whose fluctuation is compatible
(P(n) eps^ = eps^ for xi != 0) and whose stress is equilibrated
(P(n) sigma^ = 0 for xi != 0), with P(n) the projector of the laminate
equation in Sec. 3.2.

Heat conduction (the effective conductivity of Sec. 6) is the analogous
linear problem for the temperature gradient g with mean grad(theta):
curl-free fluctuation and div(kappa g) = 0. The heat flux is q = -kappa g.

Effective outputs (Sec. 2): <sigma>, <q>, the dissipation <D_diss>, the
coupling term <D> and the heat capacity <c0>, all volume averages.
"""
from __future__ import annotations

import copy

import numpy as np

from . import fourier, green, tensor
from .laws import make_law


def field_norm(a):
    return float(np.sqrt((a * a).sum()))


def conjugate_gradient(apply, b, x0=None, rtol=1e-10, maxit=10000):
    """Textbook CG for a symmetric positive (semi-)definite operator; stops when
    ||b - A x|| <= rtol ||b||. Returns (x, iterations)."""
    x = np.zeros_like(b) if x0 is None else x0.copy()
    r = b - apply(x) if x0 is not None else b.copy()
    bn = field_norm(b)
    if bn == 0.0:
        return x, 0
    p = r.copy()
    rr = float((r * r).sum())
    for it in range(maxit):
        if np.sqrt(rr) <= rtol * bn:
            return x, it
        Ap = apply(p)
        alpha = rr / float((p * Ap).sum())
        x = x + alpha * p
        r = r - alpha * Ap
        rr_new = float((r * r).sum())
        p = r + (rr_new / rr) * p
        rr = rr_new
    return x, maxit


class Cell:
    """A voxel microstructure with one constitutive law per phase id."""

    def __init__(self, phases, laws, lengths=(1.0, 1.0, 1.0), discretization="ms"):
        """discretization: "ms" (Moulinec-Suquet collocation, directions
        xi / |xi|) or "rotated" (the modified wave vectors of the rotated
        finite-difference scheme, fourier.rotated_wavevectors; Newton-CG and
        CG only)."""
        self.phases = np.asarray(phases, dtype=np.uint8)
        self.shape = self.phases.shape
        self.laws = [make_law(p) for p in laws]
        self.masks = [self.phases == i for i in range(len(self.laws))]
        if discretization not in ("ms", "rotated"):
            raise ValueError(f"unknown discretization {discretization}")
        self.discretization = discretization
        if discretization == "ms":
            self.n = fourier.directions(self.shape, lengths)
        else:
            self.n = fourier.rotated_directions(self.shape, lengths)
        self.nvox = self.phases.size
        self.eps_n = np.zeros((6,) + self.shape)
        self.E_n = np.zeros(6)
        self.g = None
        self.state = {i: law.initial_state(int(self.masks[i].sum()))
                      for i, law in enumerate(self.laws) if law.inelastic}
        self.kappa = np.zeros(self.shape)
        self.c0 = np.zeros(self.shape)
        for i, law in enumerate(self.laws):
            self.kappa[self.masks[i]] = law.kappa
            self.c0[self.masks[i]] = law.c0
        self.last = {}

    # ---- constitutive evaluation over the whole grid --------------------
    def evaluate(self, eps, theta, dt, with_tangent=True):
        sig = np.zeros_like(eps)
        tan = np.zeros((6, 6) + self.shape) if with_tangent else None
        diss = np.zeros(self.shape)
        coup = np.zeros(self.shape)
        new_state = {}
        for i, law in enumerate(self.laws):
            msk = self.masks[i]
            if not msk.any():
                continue
            e = eps[:, msk]
            en = self.eps_n[:, msk]
            if law.inelastic:
                out = law.update(e, en, self.state[i], theta, dt)
                sig[:, msk] = out["sigma"]
                if with_tangent:
                    tan[:, :, msk] = out["tangent"]
                diss[msk] = out["dissipation"]
                coup[msk] = out["coupling"]
                new_state[i] = out["state"]
            else:
                sig[:, msk] = law.stress(e, theta)
                if with_tangent:
                    tan[:, :, msk] = law.C[:, :, None]
                coup[msk] = law.coupling(e, en, theta, dt)
        return sig, tan, diss, coup, new_state

    def reference_medium(self, theta, dt):
        """Moulinec-Suquet mean rule: lam0, mu0 = midpoints of the phase Lame constants
        (instantaneous viscoelastic moduli for the PA66)."""
        lams, mus = [], []
        for law in self.laws:
            if law.inelastic:
                mats = law.branch_matrices(theta, dt)
                Cve = law.Cinf.copy()
                for i, (B, M) in enumerate(mats):
                    Cve = Cve + law.C_i[i] @ (np.eye(6) - M)
                K = Cve[0, 0] / 3.0 + 2.0 * Cve[0, 1] / 3.0
                G = 0.5 * Cve[3, 3]
            else:
                K, G = law.K, law.G
            lams.append(K - 2.0 * G / 3.0)
            mus.append(G)
        return 0.5 * (min(lams) + max(lams)), 0.5 * (min(mus) + max(mus))

    # ---- mechanical solvers -------------------------------------------
    def project(self, field):
        if self.discretization == "rotated":
            return fourier.ifft3(green.projector_hermitian(fourier.fft3(field), self.n))
        return fourier.ifft3(green.projector(fourier.fft3(field), self.n))

    def project_gradient(self, field):
        if self.discretization == "rotated":
            return fourier.ifft3(green.gradient_projector_hermitian(fourier.fft3(field), self.n))
        return fourier.ifft3(green.gradient_projector(fourier.fft3(field), self.n))

    def _basic(self, eps, theta, dt, tol, maxit):
        if self.discretization != "ms":
            raise ValueError("the basic scheme is built for the Moulinec-Suquet discretization only")
        lam0, mu0 = self.reference_medium(theta, dt)
        for it in range(1, maxit + 1):
            sig = self.evaluate(eps, theta, dt, with_tangent=False)[0]
            d = fourier.ifft3(green.gamma_isotropic(fourier.fft3(sig), self.n, lam0, mu0))
            eps = eps - d
            err = field_norm(d) / max(field_norm(eps), 1e-300)
            if err <= tol:
                return eps, dict(iterations=it, residual=err, converged=True)
        return eps, dict(iterations=maxit, residual=err, converged=False)

    def _newton(self, eps, theta, dt, tol, max_newton, cg_rtol):
        krylov = 0
        res = np.inf
        for it in range(max_newton + 1):
            sig, tan, *_ = self.evaluate(eps, theta, dt)
            R = self.project(sig)
            sn = field_norm(sig)
            res = field_norm(R) / sn if sn > 0.0 else 0.0
            if res <= tol:
                return eps, dict(iterations=it, krylov=krylov, residual=res, converged=True)
            if it == max_newton:
                break
            apply = lambda v: self.project(np.einsum("ab...,b...->a...", tan, v))
            d, k = conjugate_gradient(apply, -R, rtol=cg_rtol)
            krylov += k
            eps = eps + d
        return eps, dict(iterations=max_newton, krylov=krylov, residual=res, converged=False)

    # ---- heat conduction ------------------------------------------------
    def _thermal(self, grad, scheme, tol, maxit):
        G = np.asarray(grad, dtype=np.float64)
        if self.g is None:
            self.g = np.zeros((3,) + self.shape)
        g = self.g + G[:, None, None, None]
        if scheme == "basic":
            k0 = 0.5 * (self.kappa.min() + self.kappa.max())
            its = 0
            for its in range(1, maxit + 1):
                d = fourier.ifft3(green.gamma_conduction(fourier.fft3(self.kappa[None] * g), self.n, k0))
                g = g - d
                if field_norm(d) <= tol * max(field_norm(g), 1e-300):
                    break
        else:
            proj = self.project_gradient
            b = -proj(self.kappa[None] * G[:, None, None, None])
            apply = lambda v: proj(self.kappa[None] * v)
            x0 = self.g
            if field_norm(b) == 0.0:
                gt, its = np.zeros_like(b), 0
            else:
                gt, its = conjugate_gradient(apply, b, x0=x0, rtol=tol)
            g = gt + G[:, None, None, None]
        self.g = g - G[:, None, None, None]
        q = -self.kappa[None] * g
        return q.reshape(3, -1).mean(axis=1), its

    # ---- one load increment ---------------------------------------------
    def solve_increment(self, strain, theta, grad, dt, scheme="newton", tol=1e-10,
                        maxit=2000, max_newton=50, cg_rtol=1e-3, thermal_tol=None):
        """strain: (6,) components (11, 22, 33, 23, 13, 12); returns effective outputs."""
        E = tensor.components_to_mandel(strain)
        eps = self.eps_n + (E - self.E_n)[:, None, None, None]
        if scheme == "basic":
            eps, info = self._basic(eps, theta, dt, tol, maxit)
        else:
            eps, info = self._newton(eps, theta, dt, tol, max_newton, cg_rtol)
        sig, tan, diss, coup, new_state = self.evaluate(eps, theta, dt, with_tangent=True)
        q, th_its = self._thermal(grad, scheme, tol if thermal_tol is None else thermal_tol, maxit)
        # the algorithmic tangent field at the converged strain and what the
        # point partials need (state n and eps^n, before the commit)
        self.last = dict(eps=eps, sigma=sig, dissipation=diss, coupling=coup, tangent=tan,
                         eps_n=self.eps_n, state_n=dict(self.state), theta=theta, dt=dt)
        self.eps_n = eps
        self.E_n = E
        self.state.update(new_state)
        out = dict(
            stress=tensor.mandel_to_components(sig.reshape(6, -1).mean(axis=1)),
            heat_flux=q,
            dissipation=float(diss.mean()),
            coupling=float(coup.mean()),
            heat_capacity=float(self.c0.mean()),
            thermal_iterations=th_its,
        )
        out.update(info)
        return out

    # ---- mixed boundary conditions, adiabatic heat balance -----------------
    def solve_load(self, strain, stress, mask, theta_n, grad, dt, adiabatic=False, tol=1e-10, cg_rtol=1e-6,
                   stress_tol=1e-10, theta_tol=1e-9, max_outer=30, max_stagger=30):
        """One increment of the paper's single-point virtual experiments:
        mixed boundary conditions (the components with mask[c] True are
        stress-controlled with target stress[c], the others strain-controlled;
        Sec. 5.4 and the appendix use them for stress-free lateral directions)
        and, if adiabatic, the macroscopic heat equation of Sec. 2 at one point
        without source or flux divergence, c (theta - theta^n) / dt = <D>,
        solved by the implicit staggered scheme: mechanics at fixed theta,
        then theta from the heat equation, until theta is stationary.

        The stress-controlled macro strain components follow from an outer
        chord iteration with the effective algorithmic tangent of its first
        iterate; every outer and staggered iterate re-solves the increment
        from state n. strain,
        stress: (6,) tensor components. Returns the outputs of
        solve_increment plus the macro strain (components), theta and the
        numbers of staggered and outer iterations; commits like
        solve_increment."""
        mask = np.asarray(mask, dtype=bool)
        free = np.nonzero(mask)[0]
        Em = tensor.components_to_mandel(np.asarray(strain, dtype=np.float64))
        Sm = tensor.components_to_mandel(np.asarray(stress, dtype=np.float64))
        E = Em.copy()
        E[free] = self.E_n[free]          # start from the last mean strain of those components
        theta = float(theta_n)
        base = copy.deepcopy(self)
        outer_total = 0
        stagger = 0
        C = None
        for stagger in range(1, max_stagger + 1):
            for _ in range(max_outer):
                trial = copy.deepcopy(base)
                out = trial.solve_increment(tensor.mandel_to_components(E), theta, grad, dt, tol=tol,
                                            cg_rtol=cg_rtol)
                outer_total += 1
                if free.size == 0:
                    break
                s = tensor.components_to_mandel(out["stress"])
                res = s[free] - Sm[free]
                if np.abs(res).max() <= stress_tol * max(np.abs(s).max(), 1.0):
                    break
                if C is None:
                    C = trial.algorithmic_tangent(tol=1e-13)
                E[free] -= np.linalg.solve(C[np.ix_(free, free)], res)
            else:
                raise RuntimeError("mixed boundary conditions: outer Newton did not converge")
            if not adiabatic:
                break
            theta_next = float(theta_n) + dt * out["coupling"] / out["heat_capacity"]
            if abs(theta_next - theta) <= theta_tol:
                break
            theta = theta_next
        else:
            raise RuntimeError("adiabatic staggering did not converge")
        out = self.solve_increment(tensor.mandel_to_components(E), theta, grad, dt, tol=tol, cg_rtol=cg_rtol)
        out.update(strain=tensor.mandel_to_components(E), theta=theta, stagger_iterations=stagger,
                   outer_iterations=outer_total)
        return out

    # ---- linear effective properties -------------------------------------
    def linearized_solve(self, C, E, s0=None, tol=1e-12):
        """Strain field x with mean E (Mandel) and a compatible fluctuation d
        that solves the linearized cell problem P[C x + s0] = 0 (Sec. 2, cell
        problem; Sec. 3.3, the linear systems of the strain-jump derivatives,
        with the voxels in place of the DMN phases). Returns (x, C x + s0)."""
        apply_C = lambda v: np.einsum("ab...,b...->a...", C, v)
        eps = np.broadcast_to(np.asarray(E, dtype=np.float64)[:, None, None, None], (6,) + self.shape).copy()
        rhs = apply_C(eps) if s0 is None else apply_C(eps) + s0
        d, _ = conjugate_gradient(lambda v: self.project(apply_C(v)), -self.project(rhs), rtol=tol)
        x = eps + d
        return x, apply_C(x) if s0 is None else apply_C(x) + s0

    def homogenized_tangent(self, C, tol=1e-12):
        """Effective 6 x 6 Mandel matrix of a local linear map C(x) (6, 6, ...):
        column j is <C x_j> for the solution x_j with mean E_j (unit macro
        strain j)."""
        Cbar = np.zeros((6, 6))
        for j in range(6):
            E = np.zeros(6)
            E[j] = 1.0
            Cbar[:, j] = self.linearized_solve(C, E, tol=tol)[1].reshape(6, -1).mean(axis=1)
        return Cbar

    def point_partials(self, h_eps=1e-6, h_theta=1e-3):
        """Per-voxel partial derivatives of the local laws at the converged
        strain of the last increment, from state n: d sigma / d theta (6,
        Mandel), d D / d eps (6, Mandel) and d D / d theta of the coupling
        term D. Thermoelastic phases in closed form; the PA66 law by central
        differences of its implicit Euler update, steps h_eps (Mandel strain)
        and h_theta [K]."""
        L = self.last
        eps, eps_n, theta, dt = L["eps"], L["eps_n"], L["theta"], L["dt"]
        dsdt = np.zeros((6,) + self.shape)
        dDde = np.zeros((6,) + self.shape)
        dDdt = np.zeros(self.shape)
        for i, law in enumerate(self.laws):
            msk = self.masks[i]
            if not msk.any():
                continue
            e = eps[:, msk]
            en = eps_n[:, msk]
            if law.inelastic:
                st = L["state_n"][i]
                up = law.update(e, en, st, theta + h_theta, dt)
                dn = law.update(e, en, st, theta - h_theta, dt)
                dsdt[:, msk] = (up["sigma"] - dn["sigma"]) / (2.0 * h_theta)
                dDdt[msk] = (up["coupling"] - dn["coupling"]) / (2.0 * h_theta)
                for c in range(6):
                    ep = e.copy()
                    em = e.copy()
                    ep[c] += h_eps
                    em[c] -= h_eps
                    Dp = law.update(ep, en, st, theta, dt)["coupling"]
                    Dm = law.update(em, en, st, theta, dt)["coupling"]
                    dDde[c, msk] = (Dp - Dm) / (2.0 * h_eps)
            else:
                Ca = law.C @ law.alpha                 # C[alpha]
                dsdt[:, msk] = -Ca[:, None]
                dDde[:, msk] = (-theta / dt) * Ca[:, None]
                dDdt[msk] = -(Ca @ (e - en)) / dt
        return dsdt, dDde, dDdt

    def algorithmic_tangents(self, tol=1e-12, h_eps=1e-6, h_theta=1e-3):
        """The four effective algorithmic tangents of the last increment
        (Sec. 3.3, derivatives of the effective stress and coupling term with
        respect to the macro strain and temperature), Mandel components:
        dsde (6, 6) = d<sigma>/dE, dsdt (6,) = d<sigma>/dtheta,
        dDde (6,) = d<D>/dE, dDdt = d<D>/dtheta. The strain-jump derivatives
        of the paper become the fluctuation fields of the linearized cell
        problem: x_j (mean E_j) for dE_j and x_t (mean 0, source d sigma /
        d theta) for dtheta, all with the converged algorithmic tangent."""
        C = self.last["tangent"]
        dsdt_v, dDde_v, dDdt_v = self.point_partials(h_eps, h_theta)
        dsde = np.zeros((6, 6))
        dDde = np.zeros(6)
        for j in range(6):
            E = np.zeros(6)
            E[j] = 1.0
            x, s = self.linearized_solve(C, E, tol=tol)
            dsde[:, j] = s.reshape(6, -1).mean(axis=1)
            dDde[j] = (dDde_v * x).sum(axis=0).mean()
        x, s = self.linearized_solve(C, np.zeros(6), s0=dsdt_v, tol=tol)
        dsdt = s.reshape(6, -1).mean(axis=1)
        dDdt = float((dDdt_v + (dDde_v * x).sum(axis=0)).mean())
        return dict(dsde=dsde, dsdt=dsdt, dDde=dDde, dDdt=dDdt)

    def effective_stiffness(self, tol=1e-12):
        """6 x 6 Mandel effective stiffness of the thermoelastic phases (all
        laws linear), by six unit macro strains."""
        C = np.zeros((6, 6) + self.shape)
        for i, law in enumerate(self.laws):
            C[:, :, self.masks[i]] = law.C[:, :, None]
        return self.homogenized_tangent(C, tol)

    def algorithmic_tangent(self, tol=1e-12):
        """d<sigma>/dE (6 x 6 Mandel) at the converged state of the last
        increment: the homogenized algorithmic tangent of the local laws
        (the effective algorithmic tangent a macroscopic Newton method needs,
        Sec. 3.3)."""
        return self.homogenized_tangent(self.last["tangent"], tol)

    def effective_conductivity(self, tol=1e-12):
        kb = np.zeros((3, 3))
        for j in range(3):
            G = np.zeros(3)
            G[j] = 1.0
            self.g = None
            q, _ = self._thermal(G, "cg", tol, 10000)
            kb[:, j] = -q
        self.g = None
        return kb
