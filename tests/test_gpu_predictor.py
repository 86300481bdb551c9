"""The predictor option (start each increment from the committed strain plus
the macro increment plus the last committed strain-fluctuation change, scaled
by the projection of the new macro increment on the last one).

A start value changes the iterations, not the solution: the converged
increments equal those of the uniform start within the solver tolerance,
both for the PA66 / E-glass sphere composite under the shear-tension history
and for the batch path. After a checkpoint restore the predictor has no last
change, so that increment starts as without it (bitwise). Parity of the
uniform start with the oracle is covered by test_gpu_solver.py.
"""
import numpy as np
import pytest

from paper_2109_14403_amd import hom
from test_gpu_solver import FP32_BOUND
from paper_2109_14403_amd import workloads as W

pytestmark = pytest.mark.gpu


def run(wl, predictor, steps, precision=hom.FP64, tol=1e-10):
    ctx = hom.Context(wl.phases, wl.laws, scheme=hom.SCHEME_NEWTON_CG, precision=precision, tol=tol,
                      predictor=predictor)
    out = [ctx.solve_increment(st.strain, st.theta, st.grad, st.dt) for st in wl.history[:steps]]
    return ctx, out


# two solves that each meet the parity bound differ by twice it at most
@pytest.mark.parametrize("precision,tol,bound", [(hom.FP64, 1e-10, 1e-7), (hom.FP32, 1e-6, 2 * FP32_BOUND)])
def test_same_increments_fewer_iterations(precision, tol, bound):
    wl = W.sphere_composite_workload(32, seed=2)
    c0, a = run(wl, 0, 8, precision, tol)
    c1, b = run(wl, 1, 8, precision, tol)
    dmax = max(max(abs(x["dissipation"]) for x in a), 1e-12)
    for k, (x, y) in enumerate(zip(a, b)):
        scale = np.abs(x["stress"]).max()
        ds = np.abs(x["stress"] - y["stress"]).max() / scale
        dd = abs(x["dissipation"] - y["dissipation"]) / dmax
        print(f"precision {precision} inc {k}: stress {ds:.2e} dissipation {dd:.2e}", flush=True)
        assert ds <= bound, k
        assert dd <= bound, k
    na = sum(r["newton_iters"] for r in a[1:])
    nb = sum(r["newton_iters"] for r in b[1:])
    ka = sum(r["krylov_iters"] for r in a[1:])
    kb = sum(r["krylov_iters"] for r in b[1:])
    print(f"precision {precision}: increments 2..8 Newton {na} -> {nb}, CG {ka} -> {kb}", flush=True)
    assert a[0]["newton_iters"] == b[0]["newton_iters"]      # nothing to extrapolate from yet
    assert nb + kb < na + ka
    c0.close()
    c1.close()


def test_no_predictor_after_a_checkpoint_restore():
    wl = W.sphere_composite_workload(32, seed=2)
    ctx, _ = run(wl, 1, 4)
    state = ctx.get_state()
    ref = hom.Context(wl.phases, wl.laws, scheme=hom.SCHEME_NEWTON_CG, precision=hom.FP64, tol=1e-10)
    ref.set_state(state)
    ctx.set_state(state)
    st = wl.history[4]
    x = ctx.solve_increment(st.strain, st.theta, st.grad, st.dt)
    y = ref.solve_increment(st.strain, st.theta, st.grad, st.dt)
    assert np.array_equal(x["stress"], y["stress"])
    assert x["newton_iters"] == y["newton_iters"] and x["krylov_iters"] == y["krylov_iters"]
    # the next increment extrapolates again
    st = wl.history[5]
    x = ctx.solve_increment(st.strain, st.theta, st.grad, st.dt)
    y = ref.solve_increment(st.strain, st.theta, st.grad, st.dt)
    assert np.abs(x["stress"] - y["stress"]).max() <= 1e-7 * np.abs(y["stress"]).max()
    assert x["newton_iters"] + x["krylov_iters"] < y["newton_iters"] + y["krylov_iters"]
    ctx.close()
    ref.close()


def test_batch_with_predictor_equals_single_problems():
    probs = [W.batch_problem(i) for i in (0, 1, 2)]
    img = [p.phases for p in probs]
    hist = [p.history for p in probs]
    laws = probs[0].laws
    b = hom.Batch(img, laws, scheme=hom.SCHEME_NEWTON_CG, precision=hom.FP64, tol=1e-10, predictor=1)
    outs = []
    for k in range(len(hist[0])):
        outs.append(b.solve_increment([h[k].strain for h in hist], [h[k].theta for h in hist],
                                      [h[k].grad for h in hist], [h[k].dt for h in hist]))
    b.close()
    for j in range(3):
        ctx = hom.Context(img[j], laws, scheme=hom.SCHEME_NEWTON_CG, precision=hom.FP64, tol=1e-10, predictor=1)
        for k, st in enumerate(hist[j]):
            r = ctx.solve_increment(st.strain, st.theta, st.grad, st.dt)
            assert np.array_equal(r["stress"], outs[k][j]["stress"]), (j, k)
        ctx.close()


def test_predictor_option_must_be_zero_or_one():
    wl = W.small_sphere_workload()
    with pytest.raises(hom.HomError) as e:
        hom.Context(wl.phases, wl.laws, predictor=2)
    assert e.value.code == hom.HOM_E_ARG


@pytest.mark.parametrize("what", [0, 1])
def test_warm_started_tangents(what):
    """With the predictor option each linearized tangent solve starts from the
    previous call's solution of the same column: the same tangents, fewer
    Krylov iterations from the second call on."""
    wl = W.sphere_composite_workload(32, seed=2)
    ctxs = [hom.Context(wl.phases, wl.laws, scheme=hom.SCHEME_NEWTON_CG, precision=hom.FP64, tol=1e-10,
                        predictor=p, tangent=what) for p in (0, 1)]
    for k, st in enumerate(wl.history[:5]):
        for c in ctxs:
            c.solve_increment(st.strain, st.theta, st.grad, st.dt)
        if k < 2:
            continue
        cold, warm = (c.algorithmic_tangent(what=what) for c in ctxs)
        keys = ("dsde",) + (("dsdt", "dDde", "dDdt") if what else ())
        for key in keys:
            a, b = np.asarray(cold[key]), np.asarray(warm[key])
            assert np.abs(a - b).max() <= 1e-6 * np.abs(a).max(), (k, key)
        print(f"what {what} increment {k}: krylov {cold['krylov_iters']} cold, {warm['krylov_iters']} warm",
              flush=True)
        if k > 2:
            assert warm["krylov_iters"] < cold["krylov_iters"]
    for c in ctxs:
        c.close()


def test_predictor_under_mixed_conditions_and_adiabatic_balance():
    """Uniaxial stress (the lateral components of <sigma> held at zero) with
    the adiabatic heat balance: the same loads with fewer iterations."""
    rng = np.random.default_rng(4)
    img = (rng.random((16, 16, 16)) < 0.3).astype(np.uint8)
    laws = [W.pa66(), W.e_glass()]
    mask = 0b111110
    runs = []
    for p in (0, 1):
        ctx = hom.Context(img, laws, scheme=hom.SCHEME_NEWTON_CG, precision=hom.FP64, tol=1e-10, predictor=p)
        out, theta = [], 300.0
        for k in range(1, 6):
            r = ctx.solve_load([0.004 * k, 0, 0, 0, 0, 0], theta, [0, 0, 0], 2.0, stress=np.zeros(6),
                               stress_mask=mask, adiabatic=True)
            theta = r["theta"]
            out.append(r)
        runs.append(out)
        ctx.close()
    for k, (a, b) in enumerate(zip(*runs)):
        assert np.abs(a["stress"] - b["stress"]).max() <= 1e-7 * np.abs(a["stress"]).max(), k
        assert np.abs(a["strain"] - b["strain"]).max() <= 1e-7 * np.abs(a["strain"]).max(), k
        assert abs(a["theta"] - b["theta"]) <= 1e-6 * max(abs(a["theta"] - 300.0), 1e-3), k
    it = [sum(r["newton_iters"] + r["krylov_iters"] for r in out[1:]) for out in runs]
    print(f"mixed adiabatic increments 2..5: iterations {it[0]} -> {it[1]}", flush=True)
    assert it[1] < it[0]
