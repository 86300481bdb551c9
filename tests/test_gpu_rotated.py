"""The rotated finite-difference discretization (HOM_DISC_ROTATED) against
the oracle: the Hermitian projectors element by element through the FFT
pipeline, and whole increments of a PA66 / E-glass sphere composite, the
algorithmic tangent and a laminate's exactness."""
import numpy as np
import pytest

from oracle import fourier, green, solver
from paper_2109_14403_amd import hom
from paper_2109_14403_amd import workloads as W

from test_gpu_solver import FP32_BOUND, compare
from test_oracle_cell import MAT_A, MAT_B, laminate_equation_stiffness

pytestmark = pytest.mark.gpu

SHAPES = [(16, 16, 16), (16, 24, 32), (48, 32, 24), (32, 64, 16)]
TOL = {hom.FP64: 1e-14, hom.FP32: 1e-6}   # measured: 8.2e-16 and 3.3e-7 at most


@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("precision", [hom.FP64, hom.FP32])
@pytest.mark.parametrize("op,C", [(hom.OP_PROJECTOR_ROTATED, 6), (hom.OP_GRAD_PROJECTOR_ROTATED, 3)])
def test_rotated_projectors_match_oracle(shape, precision, op, C):
    rng = np.random.default_rng(hash((shape, op, 7)) % 2**32)
    lengths = (1.0, 1.0, 1.0) if shape[0] == shape[2] else (1.0, 0.8, 1.3)
    f = rng.normal(size=(C,) + shape) + 0.5
    gpu = hom.apply_operator(f, op, precision=precision, lengths=lengths)
    n = fourier.rotated_directions(shape, lengths)
    F = fourier.fft3(f)
    G = green.projector_hermitian(F, n) if C == 6 else green.gradient_projector_hermitian(F, n)
    ref = fourier.ifft3(G)
    err = np.abs(gpu - ref).max() / np.abs(ref).max()
    print(f"rotated shape {shape} C {C} precision {precision}: max rel err {err:.2e}", flush=True)
    assert err <= TOL[precision]


@pytest.mark.parametrize("precision,tol,bound", [(hom.FP64, 1e-9, 1e-5), (hom.FP32, 1e-6, FP32_BOUND)])
def test_rotated_spheres32_matches_oracle(precision, tol, bound):
    wl = W.sphere_composite_workload(32, seed=5)
    ctx = hom.Context(wl.phases, wl.laws, scheme=hom.SCHEME_NEWTON_CG, precision=precision, tol=tol,
                      discretization=hom.DISC_ROTATED)
    ref = solver.Cell(wl.phases, wl.laws, discretization="rotated")
    ms = hom.Context(wl.phases, wl.laws, scheme=hom.SCHEME_NEWTON_CG, precision=precision, tol=tol)
    outs = []
    for st in wl.history[:4]:
        g = ctx.solve_increment(st.strain, st.theta, st.grad, st.dt)
        o = ref.solve_increment(st.strain, st.theta, st.grad, st.dt, tol=1e-10)
        m = ms.solve_increment(st.strain, st.theta, st.grad, st.dt)
        outs.append((g, o, m))
    scale = max(np.abs(o["stress"]).max() for _, o, _ in outs)
    for k, (g, o, m) in enumerate(outs):
        compare(g, o, scale, bound, f"rotated spheres32 inc {k}")
    # a different discretization of the same cell: close to, not equal to, the collocation result
    d = max(np.abs(g["stress"] - m["stress"]).max() for g, _, m in outs) / scale
    print(f"rotated vs collocation: {d:.2e}", flush=True)
    assert 1e-4 < d < 0.05
    # the effective algorithmic tangent with the rotated operator
    t = ctx.algorithmic_tangent(what=0)
    w = np.array([1, 1, 1, np.sqrt(2), np.sqrt(2), np.sqrt(2)])
    to = ref.algorithmic_tangent(tol=1e-12) * w[None, :] / w[:, None]
    err = np.abs(t["dsde"] - to).max() / np.abs(to).max()
    print(f"rotated tangent: {err:.2e}", flush=True)
    assert err <= (1e-6 if precision == hom.FP64 else FP32_BOUND)


def test_rotated_laminate_is_exact():
    img = W.laminate((16, 16, 16), [4, 12], axis=1)
    ctx = hom.Context(img, [MAT_A, MAT_B], scheme=hom.SCHEME_NEWTON_CG, precision=hom.FP64, tol=1e-11,
                      discretization=hom.DISC_ROTATED)
    ctx.solve_increment(np.zeros(6), MAT_A["theta0"], [0, 0, 0], 1.0)
    t = ctx.algorithmic_tangent(what=0)
    cell = solver.Cell(img, [MAT_A, MAT_B])
    la = cell.laws
    lam = 0.5 * min(np.linalg.eigvalsh(la[0].C).min(), np.linalg.eigvalsh(la[1].C).min())
    Cb = laminate_equation_stiffness(la[1].C, la[0].C, img.mean(), [0, 1, 0], lam)
    w = np.array([1, 1, 1, np.sqrt(2), np.sqrt(2), np.sqrt(2)])
    assert np.allclose(t["dsde"], Cb * w[None, :] / w[:, None], rtol=1e-8, atol=1e-8 * np.abs(Cb).max())


def test_rotated_needs_newton_cg():
    img = W.centred_sphere(16, 5.8)
    with pytest.raises(hom.HomError) as e:
        hom.Context(img, [MAT_A, MAT_B], scheme=hom.SCHEME_BASIC, discretization=hom.DISC_ROTATED)
    assert e.value.code == hom.HOM_E_UNSUPPORTED
    with pytest.raises(hom.HomError) as e:
        hom.Context(img, [MAT_A, MAT_B], discretization=2)
    assert e.value.code == hom.HOM_E_ARG
