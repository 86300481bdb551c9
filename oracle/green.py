"""Green operators in Fourier space, applied frequency by frequency.

All operators act on Mandel vectors (mechanics) or 3-vectors (heat
conduction) stored as (6, ...) / (3, ...) complex arrays, with the direction
field n of shape (3, ...). Where n = 0 (zero frequency, or a frequency nulled
by the Nyquist reading) every operator returns zero: the mean of the
fluctuation is fixed separately.
"""
import numpy as np

from . import tensor


def _tau_n(t, n):
    """(tau n)_i = sum_j tau_ij n_j for a full tensor t (3, 3, ...)."""
    return np.einsum("ij...,j...->i...", t, n)


def projector(tau_m, n):
    """P(n) applied to tau (Sec. 3.2, projection operator of the laminate equation):
    (P tau)_mn = n_m (tau n)_n + (tau n)_m n_n - n_m n_n (n . tau n).
    P(n) is the orthogonal projector onto the compatible strains sym(a (x) n)."""
    t = tensor.mandel_to_matrix(tau_m)
    tn = _tau_n(t, n)
    ntn = (n * tn).sum(axis=0)
    out = (np.einsum("i...,j...->ij...", n, tn) + np.einsum("i...,j...->ij...", tn, n)
           - ntn[None, None] * np.einsum("i...,j...->ij...", n, n))
    return tensor.matrix_to_mandel(out)


def gamma_isotropic(tau_m, n, lam0, mu0):
    """Green operator of the isotropic reference medium (lam0, mu0), the
    Moulinec-Suquet operator cited in Sec. 5.2:
    Gamma tau = (n (x) tau n + tau n (x) n) / (2 mu0)
                - (lam0 + mu0) / (mu0 (lam0 + 2 mu0)) (n . tau n) n (x) n.
    It reduces to P(n) for (lam0, mu0) = (0, 1/2)."""
    t = tensor.mandel_to_matrix(tau_m)
    tn = _tau_n(t, n)
    ntn = (n * tn).sum(axis=0)
    c = (lam0 + mu0) / (mu0 * (lam0 + 2.0 * mu0))
    out = ((np.einsum("i...,j...->ij...", n, tn) + np.einsum("i...,j...->ij...", tn, n)) / (2.0 * mu0)
           - c * ntn[None, None] * np.einsum("i...,j...->ij...", n, n))
    return tensor.matrix_to_mandel(out)


def gradient_projector(q, n):
    """Q(n) q = n (n . q): orthogonal projector onto gradient fields."""
    return n * (n * q).sum(axis=0)[None]


def gamma_conduction(q, n, kappa0):
    """Green operator of a homogeneous conductor kappa0: n (n . q) / kappa0."""
    return gradient_projector(q, n) / kappa0


def projector_hermitian(tau_m, n):
    """Orthogonal projector (Hermitian inner product) onto sym(n (x) a),
    a complex, for a complex unit direction n (n-bar . n = 1):
    P tau = sym(n (x) u), u = 2 tau n-bar - n (n-bar . tau n-bar).
    It equals projector() for a real n."""
    t = tensor.mandel_to_matrix(tau_m)
    nb = np.conj(n)
    tn = _tau_n(t, nb)
    q = (nb * tn).sum(axis=0)
    u = 2.0 * tn - n * q[None]
    out = 0.5 * (np.einsum("i...,j...->ij...", n, u) + np.einsum("i...,j...->ij...", u, n))
    return tensor.matrix_to_mandel(out)


def gradient_projector_hermitian(q, n):
    """n (n-bar . q): orthogonal projector onto multiples of a complex unit n."""
    return n * (np.conj(n) * q).sum(axis=0)[None]
