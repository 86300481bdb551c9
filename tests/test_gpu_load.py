"""Mixed boundary conditions and the adiabatic heat balance of the HIP solver
(hom_solve_load) against the oracle's solve_load, which reaches the same
state by a different route (an outer chord iteration on the stress-controlled
strain components with the effective algorithmic tangent, every iterate a full
strain-controlled re-solve, and plain fixed-point staggering of theta where
the library takes secant steps).

Bounds: FP64 fields 1e-6 relative (stress to its largest component, strain
to its largest component, theta to its change over the increment); FP32
fields 2e-6 like the increment parity, except theta: 1e-5 of its change
(measured 1.3e-6: the staggering stops at 10 tol of that change).
"""
import numpy as np
import pytest

from oracle import solver
from paper_2109_14403_amd import hom
from paper_2109_14403_amd import workloads as W

from test_oracle_cell import MAT_A, MAT_B

pytestmark = pytest.mark.gpu

LATERAL = [False, True, True, True, True, True]


def errs(g, o, theta_n):
    es = np.abs(g["stress"] - o["stress"]).max() / np.abs(o["stress"]).max()
    ee = np.abs(g["strain"] - o["strain"]).max() / np.abs(o["strain"]).max()
    et = abs(g["theta"] - o["theta"]) / max(abs(o["theta"] - theta_n), 1e-3)
    ec = abs(g["coupling"] - o["coupling"]) / max(abs(o["coupling"]), 1e-9)
    return es, ee, et, ec


def test_laminate_uniaxial_stress_matches_oracle():
    img = W.laminate((16, 16, 16), [4, 12], axis=0)
    ctx = hom.Context(img, [MAT_A, MAT_B], scheme=hom.SCHEME_NEWTON_CG, precision=hom.FP64, tol=1e-11)
    ref = solver.Cell(img, [MAT_A, MAT_B])
    for k, (e11, th) in enumerate([(1e-3, 303.0), (2.5e-3, 318.0)]):
        g = ctx.solve_load([e11, 0, 0, 0, 0, 0], th, [0, 0, 0], 1.0, stress_mask=LATERAL)
        o = ref.solve_load([e11, 0, 0, 0, 0, 0], np.zeros(6), LATERAL, th, [0, 0, 0], 1.0, tol=1e-12)
        es, ee, _, _ = errs(g, o, th)
        print(f"laminate inc {k}: stress {es:.2e} strain {ee:.2e} newton {g['newton_iters']} "
              f"krylov {g['krylov_iters']}", flush=True)
        assert es <= 1e-8 and ee <= 1e-8
        assert np.abs(g["stress"][1:]).max() <= 1e-8 * abs(g["stress"][0])
        assert g["strain"][0] == e11 and g["stagger_iters"] == 1 and g["theta"] == th


def plastic_cell(n, seed=4):
    rng = np.random.default_rng(seed)
    return (rng.random((n, n, n)) < 0.3).astype(np.uint8), [W.pa66(), W.e_glass()]


@pytest.mark.parametrize("precision,steps,bound,theta_bound", [(hom.FP64, 5, 1e-6, 1e-6), (hom.FP32, 3, 2e-6, 1e-5)])
def test_plastic_mixed_adiabatic_matches_oracle(precision, steps, bound, theta_bound):
    n = 16
    img, laws = plastic_cell(n)
    tol = 1e-10 if precision == hom.FP64 else 1e-6
    ctx = hom.Context(img, laws, scheme=hom.SCHEME_NEWTON_CG, precision=precision, tol=tol)
    ref = solver.Cell(img, laws)
    theta_g = theta_o = 293.15
    for k in range(1, steps + 1):
        strain = [0.005 * k, 0, 0, 0, 0, 0]
        g = ctx.solve_load(strain, theta_g, [0, 0, 0], 2.0, stress_mask=LATERAL, adiabatic=True)
        o = ref.solve_load(strain, np.zeros(6), LATERAL, theta_o, [0, 0, 0], 2.0, adiabatic=True, tol=1e-11)
        es, ee, et, ec = errs(g, o, theta_o)
        print(f"n={n} inc {k}: stress {es:.2e} strain {ee:.2e} theta {et:.2e} coupling {ec:.2e} "
              f"theta {g['theta']:.6f} stagger {g['stagger_iters']} newton {g['newton_iters']} "
              f"krylov {g['krylov_iters']}", flush=True)
        assert es <= bound and ee <= bound and et <= theta_bound and ec <= bound
        assert g["stagger_iters"] >= 2
        theta_g, theta_o = g["theta"], o["theta"]
    assert o["dissipation"] > 0.0 and g["dissipation"] > 0.0


def test_strain_controlled_load_equals_increment():
    img, laws = plastic_cell(16, seed=5)
    hist = W.history_shear_tension()
    a = hom.Context(img, laws, scheme=hom.SCHEME_NEWTON_CG, precision=hom.FP64, tol=1e-10)
    b = hom.Context(img, laws, scheme=hom.SCHEME_NEWTON_CG, precision=hom.FP64, tol=1e-10)
    for st in hist[:4]:
        ra = a.solve_increment(st.strain, st.theta, st.grad, st.dt)
        rb = b.solve_load(st.strain, st.theta, st.grad, st.dt)
        assert np.array_equal(ra["stress"], rb["stress"]) and ra["coupling"] == rb["coupling"]
        assert np.array_equal(rb["strain"], np.asarray(st.strain)) and rb["theta"] == st.theta


def test_batch_loads_equal_single_problem_loads():
    probs = [plastic_cell(16, seed=s)[0] for s in (4, 5, 7)]
    laws = plastic_cell(16)[1]
    masks = [LATERAL, [False, True, True, False, False, False], [True, True, False, True, True, True]]
    loads = lambda k: [dict(strain=[0.006 * k, 0, 0.004 * k if j == 2 else 0, 0, 0, 0], theta=300.0,
                            grad=[0, 0, 0], dt=1.0, stress_mask=masks[j], adiabatic=(j != 1))
                       for j in range(3)]
    b = hom.Batch(probs, laws, scheme=hom.SCHEME_NEWTON_CG, precision=hom.FP64, tol=1e-10)
    rb = [b.solve_load(loads(k)) for k in (1, 2)]
    b.close()
    for j, img in enumerate(probs):
        ctx = hom.Context(img, laws, scheme=hom.SCHEME_NEWTON_CG, precision=hom.FP64, tol=1e-10)
        for k in (1, 2):
            L = loads(k)[j]
            g = ctx.solve_load(**L)
            r = rb[k - 1][j]
            assert np.allclose(r["stress"], g["stress"], rtol=1e-8, atol=1e-8 * np.abs(g["stress"]).max())
            assert np.allclose(r["strain"], g["strain"], rtol=1e-8, atol=1e-12)
            assert abs(r["theta"] - g["theta"]) <= 1e-9 * g["theta"]
        ctx.close()


def test_load_argument_errors():
    img, laws = plastic_cell(16)
    ctx = hom.Context(img, laws, scheme=hom.SCHEME_NEWTON_CG, precision=hom.FP64, tol=1e-8)
    for kw, code in ((dict(stress_mask=64), hom.HOM_E_ARG), (dict(stress=[np.nan] * 6), hom.HOM_E_ARG)):
        with pytest.raises(hom.HomError) as e:
            ctx.solve_load([1e-3, 0, 0, 0, 0, 0], 300.0, [0, 0, 0], 1.0, **kw)
        assert e.value.code == code
    L = hom.make_load([1e-3, 0, 0, 0, 0, 0], 300.0, [0, 0, 0], 1.0)
    L.adiabatic = 2
    r = hom.Result()
    assert ctx._lib.hom_solve_load(ctx._h, L, r) == hom.HOM_E_ARG
    ctx.close()
    basic = hom.Context(img, laws, scheme=hom.SCHEME_BASIC, precision=hom.FP64, tol=1e-6)
    with pytest.raises(hom.HomError) as e:
        basic.solve_load([1e-3, 0, 0, 0, 0, 0], 300.0, [0, 0, 0], 1.0, stress_mask=LATERAL)
    assert e.value.code == hom.HOM_E_UNSUPPORTED
    # adiabatic strain control works with the basic scheme
    r = basic.solve_load([1e-3, 0, 0, 0, 0, 0], 300.0, [0, 0, 0], 1.0, adiabatic=True)
    assert r["status"] == hom.HOM_OK and r["theta"] < 300.0
    basic.close()


def test_trial_increments_commit_nothing():
    """Trial solves (a macroscopic Newton method's iterations) leave step n as
    it was: trials then a commit equal the commit alone, bitwise; a trial's
    outputs and tangent are those of the committed solve at the same load."""
    img, laws = plastic_cell(16, seed=5)
    hist = W.history_shear_tension()
    a = hom.Context(img, laws, scheme=hom.SCHEME_NEWTON_CG, precision=hom.FP64, tol=1e-10)
    b = hom.Context(img, laws, scheme=hom.SCHEME_NEWTON_CG, precision=hom.FP64, tol=1e-10)
    for st in hist[:4]:
        a.solve_increment(st.strain, st.theta, st.grad, st.dt)
        b.solve_increment(st.strain, st.theta, st.grad, st.dt)
    st = hist[4]
    kw = dict(stress_mask=[False, True, True, False, False, False], adiabatic=True)
    state_before = a.get_state()
    t1 = a.solve_load(np.asarray(st.strain) * 1.3, st.theta, st.grad, st.dt, trial=True, **kw)
    t2 = a.solve_load(st.strain, st.theta, st.grad, st.dt, trial=True, **kw)
    tan_trial = a.algorithmic_tangent(what=0)["dsde"]
    assert a.get_state() == state_before
    assert not np.allclose(t1["stress"], t2["stress"])
    ra = a.solve_load(st.strain, st.theta, st.grad, st.dt, **kw)
    rb = b.solve_load(st.strain, st.theta, st.grad, st.dt, **kw)
    for k in ("stress", "strain"):
        assert np.array_equal(ra[k], rb[k])
    assert ra["theta"] == rb["theta"] and ra["coupling"] == rb["coupling"]
    assert np.array_equal(t2["stress"], rb["stress"]) and t2["theta"] == rb["theta"]
    assert np.array_equal(tan_trial, b.algorithmic_tangent(what=0)["dsde"])
    assert a.get_state() != state_before
    a.close()
    b.close()
