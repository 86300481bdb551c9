"""Degenerate and ragged cases of the HIP path against the oracle (FP64 mode).

* one phase only (a homogeneous PA66 cell): the effective response is the
  point law of Sec. 4 at the macroscopic strain, the Newton iteration ends at
  once, the heat flux is -kappa grad theta;
* a PA66 / E-glass laminate: MS collocation is exact for layers, and the
  strain field must match the oracle's element by element;
* a non-cubic grid (32 x 24 x 16) with unequal cell lengths;
* a hold increment (macro strain unchanged): viscoelastic relaxation;
* network inference on ragged and empty row counts;
* handles used as context managers are released at the end of the block.
"""
import math

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import solver, tensor  # noqa: E402
from oracle.laws import PA66  # noqa: E402
from paper_2109_14403_amd import hom  # noqa: E402
from paper_2109_14403_amd import workloads as W  # noqa: E402

pytestmark = pytest.mark.gpu

SQ2 = math.sqrt(2.0)
LAWS = [W.pa66(), W.e_glass()]


def to_components(m):
    return np.concatenate([m[:3], m[3:] / SQ2])


def effective_close(g, o, rtol):
    scale = max(np.abs(o["stress"]).max(), 1e-6)
    assert np.abs(g["stress"] - o["stress"]).max() <= rtol * scale
    assert np.allclose(g["heat_flux"], o["heat_flux"], rtol=rtol, atol=1e-12)
    assert g["dissipation"] == pytest.approx(o["dissipation"], rel=rtol, abs=1e-12)
    assert g["coupling"] == pytest.approx(o["coupling"], rel=rtol, abs=1e-12)


def test_homogeneous_pa66_cell_equals_point_law():
    phases = np.zeros((16, 16, 16), np.uint8)
    ctx = hom.Context(phases, LAWS, scheme=hom.SCHEME_NEWTON_CG, precision=hom.FP64, tol=1e-12)
    law = PA66(W.pa66())
    state = law.initial_state(1)
    eps_n = np.zeros((6, 1))
    plastic = False
    for st in W.history_shear_tension()[:6]:
        g = ctx.solve_increment(st.strain, st.theta, st.grad, st.dt)
        E = tensor.components_to_mandel(st.strain)[:, None]
        ref = law.update(E, eps_n, state, st.theta, st.dt)
        sig = to_components(ref["sigma"][:, 0])
        assert np.abs(g["stress"] - sig).max() <= 1e-10 * np.abs(sig).max()
        assert g["dissipation"] == pytest.approx(ref["dissipation"][0], rel=1e-9, abs=1e-14)
        assert g["coupling"] == pytest.approx(ref["coupling"][0], rel=1e-9)
        assert np.allclose(g["heat_flux"], -W.pa66()["kappa0"] * np.asarray(st.grad), rtol=1e-12)
        assert g["newton_iters"] <= 2 and g["krylov_iters"] <= 1
        plastic |= bool(ref["delta"][0] > 0)
        state, eps_n = ref["state"], E
    assert plastic


def test_laminate_fields_match_oracle():
    img = W.laminate((16, 16, 16), [3, 11], axis=2)
    ctx = hom.Context(img, LAWS, scheme=hom.SCHEME_NEWTON_CG, precision=hom.FP64, tol=1e-11)
    ref = solver.Cell(img, LAWS)
    for st in W.history_shear_tension()[:3]:
        g = ctx.solve_increment(st.strain, st.theta, st.grad, st.dt)
        o = ref.solve_increment(st.strain, st.theta, st.grad, st.dt, tol=1e-12)
        effective_close(g, o, 1e-7)
    eps = ctx.field(hom.FIELD_STRAIN)
    assert np.abs(eps - ref.last["eps"]).max() <= 1e-8 * np.abs(ref.last["eps"]).max()
    # piecewise constant in the layer planes
    assert np.abs(eps - eps[:, :, :1, :1]).max() <= 1e-9 * np.abs(eps).max()


def test_non_cubic_grid_with_unequal_lengths():
    rng = np.random.default_rng(8)
    img = (rng.random((16, 24, 32)) < 0.3).astype(np.uint8)      # (nz, ny, nx)
    lengths = (1.0, 0.75, 0.5)                                    # (Lx, Ly, Lz)
    ctx = hom.Context(img, LAWS, lengths=lengths, scheme=hom.SCHEME_NEWTON_CG, precision=hom.FP64, tol=1e-10)
    ref = solver.Cell(img, LAWS, lengths=lengths)
    for st in W.history_shear_tension()[:2]:
        g = ctx.solve_increment(st.strain, st.theta, st.grad, st.dt)
        o = ref.solve_increment(st.strain, st.theta, st.grad, st.dt, tol=1e-12)
        effective_close(g, o, 1e-6)


def test_hold_increment_relaxes():
    wl = W.sphere_composite_workload(16, seed=2)
    ctx = hom.Context(wl.phases, wl.laws, scheme=hom.SCHEME_NEWTON_CG, precision=hom.FP64, tol=1e-11)
    ref = solver.Cell(wl.phases, wl.laws)
    st = wl.history[3]
    outs = []
    for s in list(wl.history[:4]) + [st, st]:                    # two hold increments
        g = ctx.solve_increment(s.strain, s.theta, s.grad, s.dt)
        o = ref.solve_increment(s.strain, s.theta, s.grad, s.dt, tol=1e-12)
        effective_close(g, o, 1e-6)
        outs.append(g)
    s_load, s_hold1, s_hold2 = (np.linalg.norm(r["stress"]) for r in outs[3:])
    assert s_hold2 < s_hold1 < s_load


def test_network_ragged_and_empty_rows():
    rng = np.random.default_rng(12)
    net = hom.MLP(32, 10, seed=3)
    net.set_scaling(np.zeros(32), np.ones(32), np.zeros(10), np.ones(10))
    x = rng.normal(size=(200, 32)).astype(np.float32)
    for precise in (False, True):
        full = net.forward(x, precise=precise)
        for n in (1, 63, 65, 130):
            assert np.array_equal(net.forward(x[:n], precise=precise), full[:n])
    empty = torch.empty((0, 32), dtype=torch.float32, device="cuda")
    out = torch.empty((0, 10), dtype=torch.float32, device="cuda")
    net.forward_device(empty, out)
    y, spread, acc = hom.mlp_ensemble_infer([net, net], empty, 0.1, 1.0)
    assert y.shape == (0, 10) and spread.shape == (0,) and acc.shape == (0,)
    y, spread, acc = hom.mlp_ensemble_infer([net, net, net], empty, 0.1, 1.0)
    assert y.shape == (0, 10) and spread.shape == (0,) and acc.shape == (0,)
    with pytest.raises(hom.HomError) as e:       # an ensemble needs two networks at least
        hom.mlp_ensemble_infer([net], torch.as_tensor(x[:4], device="cuda"), 0.1, 1.0)
    assert e.value.code == hom.HOM_E_ARG


def test_handles_close_at_the_end_of_a_with_block():
    """Context and Dmn used as context managers release their handles on a
    normal exit and when the block raises; close() twice is harmless."""
    wl = W.small_sphere_workload()
    with hom.Context(wl.phases, wl.laws) as ctx:
        st = wl.history[0]
        r = ctx.solve_increment(st.strain, st.theta, st.grad, st.dt)
        assert r["status"] == hom.HOM_OK
    assert ctx._h is None
    ctx.close()
    with pytest.raises(ValueError):
        with hom.Dmn(K=2, seed=0) as net:
            raise ValueError("leave the block")
    assert net._h is None
