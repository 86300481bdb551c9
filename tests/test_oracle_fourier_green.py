"""Pins of the oracle's Fourier conventions and Green operators.

The DFT wrapper is pinned by a direct triple sum; the projector by the index
formula printed in Sec. 3.2 (laminate equation) and by its defining
properties; the isotropic-reference Green operator by its reduction to the
projector and its algebraic identities.
"""
import numpy as np
import pytest

from oracle import fourier, green, tensor


@pytest.mark.parametrize("shape", [(5, 5, 5), (4, 6, 5), (6, 6, 6), (3, 4, 2)])
def test_fft_matches_direct_sum(shape):
    rng = np.random.default_rng(11)
    f = rng.normal(size=(2,) + shape)
    F = fourier.fft3(f)
    D = fourier.dft_direct(f)
    assert np.max(np.abs(F - D)) <= 1e-12 * np.max(np.abs(D))
    assert np.allclose(fourier.ifft3(F), f, atol=1e-13)
    # Parseval
    assert np.isclose((np.abs(F) ** 2).sum() / np.prod(shape), (f * f).sum())


def test_integer_frequencies_and_nyquist():
    assert list(fourier.integer_frequencies(4)) == [0, 1, -2, -1]
    assert list(fourier.integer_frequencies(5)) == [0, 1, 2, -2, -1]
    xi = fourier.frequency_vectors((4, 4, 4), (1.0, 1.0, 1.0))
    # x frequency of index kx = 1 is 2 pi; the Nyquist index 2 is nulled
    assert np.isclose(xi[0, 0, 0, 1], 2 * np.pi)
    assert np.all(xi[0, :, :, 2] == 0.0)
    assert np.all(xi[1, :, 2, :] == 0.0)
    assert np.all(xi[2, 2, :, :] == 0.0)
    assert np.isclose(xi[0, 0, 0, 3], -2 * np.pi)
    xi_odd = fourier.frequency_vectors((3, 3, 3), (2.0, 1.0, 1.0))
    assert np.isclose(xi_odd[0, 0, 0, 1], np.pi)


def projector_index_formula(n):
    """P_mnop = 1/2 (n_m d_no n_p + n_n d_mo n_p + n_m d_np n_o + n_n d_mp n_o)
    - n_m n_n n_o n_p, written with explicit index loops (Sec. 3.2)."""
    d = np.eye(3)
    P = np.zeros((3, 3, 3, 3))
    for m in range(3):
        for nn in range(3):
            for o in range(3):
                for p in range(3):
                    P[m, nn, o, p] = 0.5 * (n[m] * d[nn, o] * n[p] + n[nn] * d[m, o] * n[p]
                                            + n[m] * d[nn, p] * n[o] + n[nn] * d[m, p] * n[o]) \
                        - n[m] * n[nn] * n[o] * n[p]
    return P


def operator_matrix(op, n):
    cols = []
    for j in range(6):
        e = np.zeros((6, 1))
        e[j, 0] = 1.0
        cols.append(op(e, n[:, None])[:, 0])
    return np.array(cols).T


def test_projector_matches_index_formula_and_is_orthogonal_projector():
    rng = np.random.default_rng(3)
    for _ in range(5):
        n = rng.normal(size=3)
        n /= np.linalg.norm(n)
        Pm = operator_matrix(green.projector, n)
        Pidx = tensor.fourth_to_mandel(projector_index_formula(n))
        assert np.allclose(Pm, Pidx, atol=1e-14)
        assert np.allclose(Pm @ Pm, Pm, atol=1e-14)
        assert np.allclose(Pm, Pm.T, atol=1e-14)
        assert np.isclose(np.trace(Pm), 3.0)
        # reproduces compatible strains sym(a (x) n)
        a = rng.normal(size=3)
        sym = 0.5 * (np.outer(a, n) + np.outer(n, a))
        v = tensor.matrix_to_mandel(sym[:, :, None])[:, 0]
        assert np.allclose(Pm @ v, v, atol=1e-14)
        # annihilates tensors with tau n = 0 (e.g. t1 (x) t2 + t2 (x) t1 with t_i ⟂ n)
        t1 = np.cross(n, a)
        t2 = np.cross(n, t1)
        tau = np.outer(t1, t2) + np.outer(t2, t1)
        assert np.allclose(Pm @ tensor.matrix_to_mandel(tau[:, :, None])[:, 0], 0.0, atol=1e-13)


def test_isotropic_green_operator_identities():
    rng = np.random.default_rng(5)
    n = rng.normal(size=3)
    n /= np.linalg.norm(n)
    G_half = operator_matrix(lambda t, nn: green.gamma_isotropic(t, nn, 0.0, 0.5), n)
    assert np.allclose(G_half, operator_matrix(green.projector, n), atol=1e-14)
    lam0, mu0 = 1.7, 0.9
    G = operator_matrix(lambda t, nn: green.gamma_isotropic(t, nn, lam0, mu0), n)
    C0 = tensor.isotropic(lam0 + 2 * mu0 / 3, mu0)
    assert np.allclose(G @ C0 @ G, G, atol=1e-13)
    # Gamma0 C0 is the (oblique) projector onto compatible strains: it fixes sym(a (x) n)
    a = rng.normal(size=3)
    v = tensor.matrix_to_mandel((0.5 * (np.outer(a, n) + np.outer(n, a)))[:, :, None])[:, 0]
    assert np.allclose(G @ C0 @ v, v, atol=1e-13)


def test_operators_vanish_at_zero_direction():
    tau = np.ones((6, 1)) + 1j
    z = np.zeros((3, 1))
    assert np.all(green.projector(tau, z) == 0)
    assert np.all(green.gamma_isotropic(tau, z, 1.0, 1.0) == 0)
    assert np.all(green.gradient_projector(np.ones((3, 1)), z) == 0)


def test_gradient_projector():
    rng = np.random.default_rng(9)
    n = rng.normal(size=3)
    n /= np.linalg.norm(n)
    Q = np.array([green.gradient_projector(np.eye(3)[:, j:j + 1], n[:, None])[:, 0] for j in range(3)]).T
    assert np.allclose(Q @ Q, Q)
    assert np.allclose(Q, np.outer(n, n))


def test_material_tables_match_fixture():
    import json
    import os
    from paper_2109_14403_amd import workloads as W
    fx = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "materials.json")))
    for name, fn in (("e_glass", W.e_glass), ("pa66", W.pa66)):
        p = fn()
        for k, v in fx[name].items():
            assert p[k] == v, (name, k)
