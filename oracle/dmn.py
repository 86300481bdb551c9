"""Direct deep material network (Sec. 3), plainly: test infrastructure only.

Tree (Sec. 3.1): a perfect rooted binary tree of depth K whose nodes are
two-phase laminates. Level k = 1..K holds 2^(k-1) nodes; node i of level k
has the children 2i-1, 2i of level k+1; the 2^K leaves (level K+1) carry the
input weights w = <v>_+ and alternate between phase 1 (odd leaves) and
phase 2 (even leaves). A node's volume fractions are its children's summed
leaf weights, normalized. Parameter order of the directions: level K first,
the root last (the paper's vector of lamination directions). Indices here are
0-based: leaf l is phase 1 for even l.

Readings where the paper is silent:
* directions are free 3-vectors m, normalized to n = m / |m| inside;
* a node whose two children carry zero weight gets the fractions (1/2, 1/2);
* the laminate equation's lambda is half the smallest eigenvalue of the two
  input stiffnesses of the sample (below every stiffness in the tree, which
  the bounds keep between the inputs).

Offline (Sec. 3.2): the linear homogenization function through the laminate
equation, the loss J with its mixing penalty, gradients by torch autograd
(FP64, CPU). Online (Sec. 3.3): Newton's method on the displacement jumps
with the dense system A^T W C A and the backtracking of the paper's
algorithm; effective stress, coupling term, dissipation and d<sigma>/dE.
"""
from __future__ import annotations

import numpy as np
import torch

from . import tensor

_DT = torch.float64


def _basis():
    """The 6 Mandel basis tensors as 3x3 matrices."""
    return torch.tensor(np.stack([tensor.mandel_to_matrix(np.eye(6)[:, j]) for j in range(6)]), dtype=_DT)


_E = None


def projector_matrix(n):
    """6x6 Mandel matrix of P(n) (Sec. 3.2): P tau = n (x) tau n + tau n (x) n - (n . tau n) n (x) n.
    n: (..., 3) unit vectors. Columns are P applied to the Mandel basis."""
    global _E
    if _E is None:
        _E = _basis()
    Tn = torch.einsum("jab,...b->...ja", _E, n)                 # (..., 6, 3): E_j n
    ntn = (Tn * n[..., None, :]).sum(-1)                          # (..., 6)
    out = (n[..., None, :, None] * Tn[..., :, None, :] + Tn[..., :, :, None] * n[..., None, None, :]
           - ntn[..., :, None, None] * n[..., None, :, None] * n[..., None, None, :])   # (..., 6, 3, 3)
    w = torch.tensor([1.0, 1.0, 1.0, np.sqrt(2.0), np.sqrt(2.0), np.sqrt(2.0)], dtype=_DT)
    idx = [(0, 0), (1, 1), (2, 2), (1, 2), (0, 2), (0, 1)]
    rows = torch.stack([out[..., a, b] for a, b in idx], dim=-1) * w   # (..., 6 columns, 6 rows)
    return rows.transpose(-1, -2)


def laminate(C1, C2, c1, n, lam):
    """Effective stiffness of a two-phase laminate with normal n and fractions
    (c1, 1 - c1): the equation of Sec. 3.2,
    (P + lam [C - lam I]^-1)^-1 = c1 (P + lam [C1 - lam I]^-1)^-1 + c2 (P + lam [C2 - lam I]^-1)^-1.
    Batched over leading axes; lam (...,)."""
    I = torch.eye(6, dtype=_DT)
    P = projector_matrix(n)
    L = lam[..., None, None]
    A = lambda C: torch.linalg.inv(P + L * torch.linalg.inv(C - L * I))
    S = c1[..., None, None] * A(C1) + (1.0 - c1)[..., None, None] * A(C2)
    return L * I + L * torch.linalg.inv(torch.linalg.inv(S) - P)


def sample_lambda(C1, C2):
    e = torch.cat([torch.linalg.eigvalsh(C1), torch.linalg.eigvalsh(C2)], dim=-1)
    return 0.5 * e.min(dim=-1).values


def homogenize(C1, C2, m, v):
    """DMN linear homogenization function: C1, C2 (B, 6, 6), m (2^K - 1, 3)
    directions, v (2^K,) unconstrained weights. Returns (B, 6, 6)."""
    nleaf = v.shape[0]
    K = int(round(np.log2(nleaf)))
    w = torch.clamp(v, min=0.0)
    lam = sample_lambda(C1, C2)
    Cs = [C1 if l % 2 == 0 else C2 for l in range(nleaf)]
    Ws = [w[l] for l in range(nleaf)]
    off = 0
    for level in range(K, 0, -1):
        cnt = 2 ** (level - 1)
        nC, nW = [], []
        for j in range(cnt):
            wl, wr = Ws[2 * j], Ws[2 * j + 1]
            s = wl + wr
            c1 = torch.where(s > 0, wl / torch.where(s > 0, s, torch.ones_like(s)), torch.full_like(s, 0.5))
            mm = m[off + j]
            n = mm / torch.linalg.norm(mm)
            nC.append(laminate(Cs[2 * j], Cs[2 * j + 1], c1.expand(lam.shape), n, lam))
            nW.append(s)
        off += cnt
        Cs, Ws = nC, nW
    return Cs[0]


def loss(C1, C2, Cbar, m, v, q=10.0, penalty=1e3):
    """J of Sec. 3.2 with p = 1: (1/B) (sum_s e_s^q)^(1/q) + penalty (sum w - 1)^2,
    e_s = |Cbar_s - DMN_s|_1 / |Cbar_s|_1 over the Mandel components."""
    D = homogenize(C1, C2, m, v)
    e = (Cbar - D).abs().sum(dim=(-1, -2)) / Cbar.abs().sum(dim=(-1, -2))
    B = C1.shape[0]
    w = torch.clamp(v, min=0.0)
    return (e ** q).sum() ** (1.0 / q) / B + penalty * (w.sum() - 1.0) ** 2


def loss_and_grad(C1, C2, Cbar, m, v, q=10.0, penalty=1e3):
    """Loss and its gradients with respect to m and v (autograd, FP64)."""
    mt = torch.tensor(m, dtype=_DT, requires_grad=True)
    vt = torch.tensor(v, dtype=_DT, requires_grad=True)
    J = loss(torch.as_tensor(C1, dtype=_DT), torch.as_tensor(C2, dtype=_DT), torch.as_tensor(Cbar, dtype=_DT),
             mt, vt, q, penalty)
    J.backward()
    return float(J.detach()), mt.grad.numpy().copy(), vt.grad.numpy().copy()


def homogenize_np(C1, C2, m, v):
    with torch.no_grad():
        return homogenize(torch.as_tensor(C1, dtype=_DT), torch.as_tensor(C2, dtype=_DT),
                          torch.as_tensor(m, dtype=_DT), torch.as_tensor(v, dtype=_DT)).numpy()


# ---------------------------------------------------------------------------
# online evaluation (Sec. 3.3)
# ---------------------------------------------------------------------------
def sym_matrix(n):
    """6 x 3 Mandel matrix of a -> sym(a (x) n)."""
    out = np.zeros((6, 3))
    for k in range(3):
        a = np.zeros(3)
        a[k] = 1.0
        out[:, k] = tensor.matrix_to_mandel(0.5 * (np.outer(a, n) + np.outer(n, a)))
    return out


def kinematics(m, v):
    """A (6 * 2^K, 3 * (2^K - 1)) of the kinematics eps_leaf = E + A a (Sec. 3.3)
    and the leaf weights w: along the path from the root, a leaf in the first
    child's subtree of a node gets + c2 sym(a (x) n), in the second child's
    subtree - c1 sym(a (x) n)."""
    nleaf = len(v)
    K = int(round(np.log2(nleaf)))
    w = np.maximum(np.asarray(v, dtype=np.float64), 0.0)
    A = np.zeros((6 * nleaf, 3 * (nleaf - 1)))
    off = 0
    for level in range(K, 0, -1):
        cnt = 2 ** (level - 1)
        span = nleaf // cnt                      # leaves under a node of this level
        for j in range(cnt):
            node = off + j
            leaves = np.arange(j * span, (j + 1) * span)
            left, right = leaves[: span // 2], leaves[span // 2:]
            wl, wr = w[left].sum(), w[right].sum()
            c1 = wl / (wl + wr) if wl + wr > 0 else 0.5
            n = np.asarray(m[node], dtype=np.float64)
            Nm = sym_matrix(n / np.linalg.norm(n))
            for l in left:
                A[6 * l:6 * l + 6, 3 * node:3 * node + 3] += (1.0 - c1) * Nm
            for l in right:
                A[6 * l:6 * l + 6, 3 * node:3 * node + 3] -= c1 * Nm
        off += cnt
    return A, w


class OnlineDMN:
    """A DMN at one macroscopic point with the laws of its two phases (phase 1
    on odd leaves, phase 2 on even ones; the paper's glass fibres and PA66
    matrix) and their internal variables; Newton's method with backtracking
    on the displacement jumps as in the paper's online algorithm."""

    def __init__(self, m, v, law1, law2, tol=1e-10, maxit=50, maxbacktrack=8, gamma=0.5):
        from .laws import make_law
        self.A, self.w = kinematics(m, v)
        self.nleaf = len(v)
        self.laws = [make_law(law1), make_law(law2)]
        self.leaves = [np.arange(0, self.nleaf, 2), np.arange(1, self.nleaf, 2)]
        self.state = {p: self.laws[p].initial_state(len(self.leaves[p]))
                      for p in (0, 1) if self.laws[p].inelastic}
        self.a = np.zeros(3 * (self.nleaf - 1))
        self.eps_n = np.zeros((6, self.nleaf))
        self.tol, self.maxit, self.maxbacktrack, self.gamma = tol, maxit, maxbacktrack, gamma

    def leaf_strains(self, E, a):
        return (np.repeat(E[None], self.nleaf, axis=0).reshape(-1) + self.A @ a).reshape(self.nleaf, 6).T

    def evaluate(self, eps, theta, dt):
        sig = np.zeros((6, self.nleaf))
        tan = np.zeros((self.nleaf, 6, 6))
        coup = np.zeros(self.nleaf)
        diss = np.zeros(self.nleaf)
        new = {}
        for p in (0, 1):
            idx = self.leaves[p]
            law = self.laws[p]
            e, en = eps[:, idx], self.eps_n[:, idx]
            if law.inelastic:
                out = law.update(e, en, self.state[p], theta, dt)
                sig[:, idx] = out["sigma"]
                tan[idx] = np.moveaxis(out["tangent"], 2, 0)
                coup[idx] = out["coupling"]
                diss[idx] = out["dissipation"]
                new[p] = out["state"]
            else:
                sig[:, idx] = law.stress(e, theta)
                tan[idx] = law.C[None]
                coup[idx] = law.coupling(e, en, theta, dt)
        return sig, tan, coup, diss, new

    def residual(self, E, a, theta, dt):
        eps = self.leaf_strains(E, a)
        sig = self.evaluate(eps, theta, dt)[0]
        g = self.A.T @ (sig.T * self.w[:, None]).reshape(-1)
        sbar = sig @ self.w
        return np.linalg.norm(g) / ((self.nleaf - 1) * max(np.linalg.norm(sbar), 1e-300)), g

    def point_partials(self, eps, theta, dt, h_eps=1e-6, h_theta=1e-3):
        """Per-leaf d sigma / d theta (6), d D / d eps (6) and d D / d theta of
        the coupling term D at the leaf strains, from state n: closed form for
        thermoelastic phases, central differences of the PA66 update (steps
        h_eps in Mandel strain, h_theta in K)."""
        dsdt = np.zeros((6, self.nleaf))
        dDde = np.zeros((6, self.nleaf))
        dDdt = np.zeros(self.nleaf)
        for p in (0, 1):
            idx = self.leaves[p]
            law = self.laws[p]
            e, en = eps[:, idx], self.eps_n[:, idx]
            if law.inelastic:
                st = self.state[p]
                up = law.update(e, en, st, theta + h_theta, dt)
                dn = law.update(e, en, st, theta - h_theta, dt)
                dsdt[:, idx] = (up["sigma"] - dn["sigma"]) / (2.0 * h_theta)
                dDdt[idx] = (up["coupling"] - dn["coupling"]) / (2.0 * h_theta)
                for c in range(6):
                    ep, em = e.copy(), e.copy()
                    ep[c] += h_eps
                    em[c] -= h_eps
                    dDde[c, idx] = (law.update(ep, en, st, theta, dt)["coupling"]
                                    - law.update(em, en, st, theta, dt)["coupling"]) / (2.0 * h_eps)
            else:
                Ca = law.C @ law.alpha
                dsdt[:, idx] = -Ca[:, None]
                dDde[:, idx] = (-theta / dt) * Ca[:, None]
                dDdt[idx] = -(Ca @ (e - en)) / dt
        return dsdt, dDde, dDdt

    def step(self, strain, theta, dt, all_tangents=False):
        """One increment at the macro strain (6 tensor components), theta, dt.
        Commits the internal variables and the jumps; returns the effective
        stress (components), coupling term, dissipation, d<sigma>/dE (Mandel)
        and the Newton iterations; with all_tangents also d<sigma>/dtheta,
        d<D>/dE (Mandel) and d<D>/dtheta (Sec. 3.3: the strain-jump
        derivatives solve the Newton system with other right-hand sides)."""
        E = tensor.components_to_mandel(np.asarray(strain, dtype=np.float64))
        a = self.a.copy()                        # the jumps of the last increment
        res, g = self.residual(E, a, theta, dt)
        its = 0
        for its in range(1, self.maxit + 1):
            eps = self.leaf_strains(E, a)
            _, tan, *_ = self.evaluate(eps, theta, dt)
            Kmat = self.A.T @ self._blockdiag(tan) @ self.A
            # minimal-norm solution: the jump of a laminate with a weightless
            # side is a null mode and stays where it is
            da = np.linalg.lstsq(Kmat, -g, rcond=1e-13)[0]
            res_old = res
            a = a + da
            res, g = self.residual(E, a, theta, dt)
            for i in range(self.maxbacktrack):
                if res < res_old:
                    break
                a = a - self.gamma ** i * (1.0 - self.gamma) * da
                res, g = self.residual(E, a, theta, dt)
            if res < self.tol:
                break
        eps = self.leaf_strains(E, a)
        sig, tan, coup, diss, new = self.evaluate(eps, theta, dt)
        WC = self._blockdiag(tan)
        Kmat = self.A.T @ WC @ self.A
        one = np.tile(np.eye(6), (self.nleaf, 1))               # E -> every leaf
        dadE = -np.linalg.lstsq(Kmat, self.A.T @ WC @ one, rcond=1e-13)[0]
        dleaf = one + self.A @ dadE                              # d eps_leaf / dE
        Cbar = (np.tile(self.w.repeat(6)[:, None], (1, 6)) * (self._blockdiag_unweighted(tan) @ dleaf))
        Cbar = Cbar.reshape(self.nleaf, 6, 6).sum(axis=0)
        extra = {}
        if all_tangents:
            dsdt_l, dDde_l, dDdt_l = self.point_partials(eps, theta, dt)
            dadT = -np.linalg.lstsq(Kmat, self.A.T @ (self.w[:, None] * dsdt_l.T).reshape(-1), rcond=1e-13)[0]
            deps_dT = (self.A @ dadT).reshape(self.nleaf, 6).T
            dsdt = sum(self.w[l] * (dsdt_l[:, l] + tan[l] @ deps_dT[:, l]) for l in range(self.nleaf))
            dl = dleaf.reshape(self.nleaf, 6, 6)
            dDde = sum(self.w[l] * (dl[l].T @ dDde_l[:, l]) for l in range(self.nleaf))
            dDdt = sum(self.w[l] * (dDdt_l[l] + dDde_l[:, l] @ deps_dT[:, l]) for l in range(self.nleaf))
            extra = dict(dsdt=dsdt, dDde=dDde, dDdt=float(dDdt))
        self.state.update(new)
        self.eps_n = eps
        self.a = a
        return dict(stress=tensor.mandel_to_components(sig @ self.w), coupling=float(coup @ self.w),
                    dissipation=float(diss @ self.w), dsde=Cbar, newton_iters=its, residual=res, **extra)

    def _blockdiag(self, tan):
        out = np.zeros((6 * self.nleaf, 6 * self.nleaf))
        for l in range(self.nleaf):
            out[6 * l:6 * l + 6, 6 * l:6 * l + 6] = self.w[l] * tan[l]
        return out

    def _blockdiag_unweighted(self, tan):
        out = np.zeros((6 * self.nleaf, 6 * self.nleaf))
        for l in range(self.nleaf):
            out[6 * l:6 * l + 6, 6 * l:6 * l + 6] = tan[l]
        return out
