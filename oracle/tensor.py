"""Second-order symmetric tensors in normalized Voigt-Mandel notation.

The paper measures stiffness norms in normalized Voigt-Mandel notation
(Sec. 3.2, loss function; Sec. 5.3, mean error). A symmetric tensor T is
stored as the 6-vector (T11, T22, T33, sqrt2 T23, sqrt2 T13, sqrt2 T12), so
that the Euclidean product of two such vectors equals the double contraction
T:S and fourth-order tensors with minor symmetries become 6 x 6 matrices.
"""
import numpy as np

SQ2 = np.sqrt(2.0)
# Mandel slot -> (i, j)
PAIRS = [(0, 0), (1, 1), (2, 2), (1, 2), (0, 2), (0, 1)]
WEIGHT = np.array([1.0, 1.0, 1.0, SQ2, SQ2, SQ2])

IDENTITY2 = np.array([1.0, 1.0, 1.0, 0.0, 0.0, 0.0])
P1 = np.outer(IDENTITY2, IDENTITY2) / 3.0           # spherical projector (Sec. 4)
P2 = np.eye(6) - P1                                  # deviatoric projector (Sec. 4)


def components_to_mandel(c):
    """(11, 22, 33, 23, 13, 12) tensor components -> Mandel vector (last axis)."""
    c = np.asarray(c, dtype=np.float64)
    return c * WEIGHT


def mandel_to_components(m):
    m = np.asarray(m)
    return m / WEIGHT


def mandel_to_matrix(m):
    """Mandel (6, ...) -> full tensor (3, 3, ...)."""
    m = np.asarray(m)
    t = np.zeros((3, 3) + m.shape[1:], dtype=m.dtype)
    for a, (i, j) in enumerate(PAIRS):
        v = m[a] / WEIGHT[a]
        t[i, j] = v
        t[j, i] = v
    return t


def matrix_to_mandel(t):
    """Full symmetric tensor (3, 3, ...) -> Mandel (6, ...)."""
    t = np.asarray(t)
    m = np.zeros((6,) + t.shape[2:], dtype=t.dtype)
    for a, (i, j) in enumerate(PAIRS):
        m[a] = WEIGHT[a] * 0.5 * (t[i, j] + t[j, i])
    return m


def fourth_to_mandel(C):
    """Fourth-order tensor C_ijkl with minor symmetries -> 6 x 6 Mandel matrix."""
    M = np.zeros((6, 6))
    for a, (i, j) in enumerate(PAIRS):
        for b, (k, l) in enumerate(PAIRS):
            M[a, b] = WEIGHT[a] * WEIGHT[b] * C[i, j, k, l]
    return M


def isotropic(K, G):
    """C = 3K P1 + 2G P2 (Sec. 4, E-glass fibres)."""
    return 3.0 * K * P1 + 2.0 * G * P2


def bulk_shear(E, nu):
    """K = E / (3(1 - 2 nu)), G = E / (2(1 + nu)) (Sec. 4)."""
    return E / (3.0 * (1.0 - 2.0 * nu)), E / (2.0 * (1.0 + nu))


def trace(m):
    return m[0] + m[1] + m[2]


def deviator(m):
    tr3 = trace(m) / 3.0
    out = np.array(m, dtype=np.float64, copy=True)
    out[0] -= tr3
    out[1] -= tr3
    out[2] -= tr3
    return out


def norm(m):
    return np.sqrt((np.asarray(m) ** 2).sum(axis=0))
