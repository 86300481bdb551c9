"""Pins of the rotated finite-difference discretization (modified wave
vectors; the "staggered grid" the paper cites for its stiffness samples).

* the symbol k_j is that of a real-space stencil: the difference of a corner
  displacement along j, averaged over the 4 cell edges parallel to j,
  applied with np.roll to random fields (no Fourier formula involved);
* the Hermitian projector keeps every strain field built by that stencil
  (range), is idempotent and self-adjoint on real fields, and maps real
  fields to real fields;
* it equals the Moulinec-Suquet projector for real directions;
* laminates with layers across a grid axis: the effective stiffness is the
  laminate equation of Sec. 3.2, exactly as for the collocation scheme;
* the rotated and the collocation schemes agree on the effective stiffness
  of a sphere composite to the discretization error (a few per cent at 16^3)
  and both within the Voigt / Reuss bounds.
"""
import numpy as np
import pytest

from oracle import fourier, green, solver, tensor
from paper_2109_14403_amd import workloads as W

from test_oracle_cell import MAT_A, MAT_B, laminate_equation_stiffness

RNG = np.random.default_rng(21)


def stencil_strain(u, lengths=(1.0, 1.0, 1.0)):
    """Rotated-scheme strain (Mandel, (6, nz, ny, nx)) of a corner displacement
    u (3, nz, ny, nx), u[i] the x_i component at corner (z, y, x): gradient
    d_j u_i at the cell centre x + 1/2 = mean over the 4 edges parallel to j
    of u_i(corner + e_j) - u_i(corner)."""
    nz, ny, nx = u.shape[1:]
    h = (lengths[0] / nx, lengths[1] / ny, lengths[2] / nz)
    ax = {0: 2, 1: 1, 2: 0}           # coordinate -> array axis
    sh = lambda f, j: np.roll(f, -1, axis=ax[j] + (f.ndim - 3))   # f(x + e_j)
    grad = np.zeros((3, 3, nz, ny, nx))
    for i in range(3):
        for j in range(3):
            d = (sh(u[i], j) - u[i]) / h[j]
            o = [l for l in range(3) if l != j]
            avg = 0.25 * (d + sh(d, o[0]) + sh(d, o[1]) + sh(sh(d, o[0]), o[1]))
            grad[i, j] = avg
    eps = 0.5 * (grad + grad.transpose(1, 0, 2, 3, 4))
    return tensor.matrix_to_mandel(eps)


@pytest.mark.parametrize("shape,lengths", [((6, 8, 10), (1.0, 1.0, 1.0)), ((5, 7, 4), (1.0, 2.0, 0.5))])
def test_symbol_matches_real_space_stencil(shape, lengths):
    u = RNG.standard_normal((3,) + shape)
    eps = stencil_strain(u, lengths)
    k = fourier.rotated_wavevectors(shape, lengths)
    uh = fourier.fft3(u)
    sym = 0.5 * (np.einsum("i...,j...->ij...", uh, k) + np.einsum("i...,j...->ij...", k, uh))
    assert np.allclose(fourier.fft3(eps), tensor.matrix_to_mandel(sym), atol=1e-9 * np.abs(uh).max())


@pytest.mark.parametrize("shape", [(6, 8, 10), (5, 7, 4), (8, 8, 8)])
def test_projector_range_idempotence_symmetry(shape):
    n = fourier.rotated_directions(shape)
    P = lambda f: fourier.ifft3(green.projector_hermitian(fourier.fft3(f), n))
    eps = stencil_strain(RNG.standard_normal((3,) + shape))
    eps -= eps.reshape(6, -1).mean(axis=1)[:, None, None, None]
    assert np.allclose(P(eps), eps, atol=1e-10)
    a = RNG.standard_normal((6,) + shape)
    b = RNG.standard_normal((6,) + shape)
    Pa = P(a)
    assert np.allclose(P(Pa), Pa, atol=1e-10)
    assert np.isclose((Pa * b).sum(), (a * P(b)).sum(), rtol=1e-10)
    full = np.fft.ifftn(green.projector_hermitian(fourier.fft3(a), n), axes=(-3, -2, -1))
    assert np.abs(full.imag).max() <= 1e-12 * np.abs(full.real).max()
    g = RNG.standard_normal((3,) + shape)
    Q = lambda f: fourier.ifft3(green.gradient_projector_hermitian(fourier.fft3(f), n))
    assert np.allclose(Q(Q(g)), Q(g), atol=1e-10)


def test_hermitian_projector_equals_real_for_real_directions():
    shape = (6, 6, 6)
    n = fourier.directions(shape)
    t = fourier.fft3(RNG.standard_normal((6,) + shape))
    assert np.allclose(green.projector_hermitian(t, n), green.projector(t, n), atol=1e-12)


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_laminate_exact_on_rotated_grid(axis):
    img = W.laminate((8, 8, 8), [2, 6], axis=axis)
    cell = solver.Cell(img, [MAT_A, MAT_B], discretization="rotated")
    Cb = cell.effective_stiffness(tol=1e-13)
    la = cell.laws
    lam = 0.5 * min(np.linalg.eigvalsh(la[0].C).min(), np.linalg.eigvalsh(la[1].C).min())
    expect = laminate_equation_stiffness(la[1].C, la[0].C, img.mean(), np.eye(3)[axis], lam)
    assert np.allclose(Cb, expect, rtol=1e-9, atol=1e-9 * np.abs(expect).max())


def test_sphere_rotated_close_to_collocation_and_bounded():
    img = W.centred_sphere(16, 5.8)
    ms = solver.Cell(img, [MAT_A, MAT_B]).effective_stiffness(tol=1e-11)
    rot = solver.Cell(img, [MAT_A, MAT_B], discretization="rotated").effective_stiffness(tol=1e-11)
    assert np.abs(rot - ms).max() <= 0.05 * np.abs(ms).max()
    assert not np.allclose(rot, ms, rtol=1e-6)      # a different discretization
    c = img.mean()
    CA, CB = tensor.isotropic(*tensor.bulk_shear(MAT_A["E"], MAT_A["nu"])), \
        tensor.isotropic(*tensor.bulk_shear(MAT_B["E"], MAT_B["nu"]))
    voigt = (1 - c) * CA + c * CB
    reuss = np.linalg.inv((1 - c) * np.linalg.inv(CA) + c * np.linalg.inv(CB))
    assert np.linalg.eigvalsh(voigt - rot).min() >= -1e-8 * np.abs(voigt).max()
    assert np.linalg.eigvalsh(rot - reuss).min() >= -1e-8 * np.abs(voigt).max()
