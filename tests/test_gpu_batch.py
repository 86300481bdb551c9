"""Batched microproblems: every problem of one batched solve must equal its
own single-problem solve, and match the oracle."""
import numpy as np
import pytest

from oracle import solver
from paper_2109_14403_amd import hom
from test_gpu_solver import FP32_BOUND
from paper_2109_14403_amd import workloads as W

pytestmark = pytest.mark.gpu


def problems(idx):
    return [W.batch_problem(i) for i in idx]


def test_batch_equals_single_problem_solves():
    wls = problems([0, 1, 2, 3, 5, 8])
    sizes = sorted({w.record["n"] for w in wls})
    assert len(sizes) >= 2
    laws = [W.pa66(), W.e_glass()]
    opts = dict(scheme=hom.SCHEME_NEWTON_CG, precision=hom.FP64, tol=1e-9)
    b = hom.Batch([w.phases for w in wls], laws, **opts)
    singles = [hom.Context(w.phases, laws, **opts) for w in wls]
    for k in range(3):
        strains = np.array([w.history[k].strain for w in wls])
        thetas = [w.history[k].theta for w in wls]
        grads = [w.history[k].grad for w in wls]
        dts = [w.history[k].dt for w in wls]
        rb = b.solve_increment(strains, thetas, grads, dts)
        for i, (w, ctx) in enumerate(zip(wls, singles)):
            rs = ctx.solve_increment(strains[i], thetas[i], grads[i], dts[i])
            assert rb[i]["status"] == 0
            scale = np.abs(rs["stress"]).max()
            assert np.abs(rb[i]["stress"] - rs["stress"]).max() <= 1e-9 * scale, (k, i)
            assert np.allclose(rb[i]["heat_flux"], rs["heat_flux"], rtol=1e-9)
            assert rb[i]["dissipation"] == pytest.approx(rs["dissipation"], rel=1e-8, abs=1e-14)
            assert rb[i]["coupling"] == pytest.approx(rs["coupling"], rel=1e-8, abs=1e-12)
    stats = b.kernel_stats()
    assert isinstance(stats, dict)


def test_batch_matches_oracle():
    wls = [w for w in problems(range(12)) if w.record["n"] == 24][:2]
    wls += [w for w in problems(range(12)) if w.record["n"] == 32][:1]
    laws = [W.pa66(), W.e_glass()]
    b = hom.Batch([w.phases for w in wls], laws, scheme=hom.SCHEME_NEWTON_CG, precision=hom.FP32, tol=1e-6)
    refs = [solver.Cell(w.phases, laws) for w in wls]
    for k in range(3):
        strains = np.array([w.history[k].strain for w in wls])
        rb = b.solve_increment(strains, [w.history[k].theta for w in wls], [w.history[k].grad for w in wls],
                               [w.history[k].dt for w in wls])
        for i, (w, ref) in enumerate(zip(wls, refs)):
            st = w.history[k]
            o = ref.solve_increment(st.strain, st.theta, st.grad, st.dt, tol=1e-10)
            scale = max(np.abs(o["stress"]).max(), 1e-3)
            err = np.abs(rb[i]["stress"] - o["stress"]).max() / scale
            print(f"batch problem {i} (n={w.record['n']}) inc {k}: stress err {err:.2e}", flush=True)
            assert err <= FP32_BOUND
            assert np.allclose(rb[i]["heat_flux"], o["heat_flux"], rtol=FP32_BOUND)


def test_full_batch_in_bench_configuration_matches_oracle():
    """The 512-problem batch as the benchmark runs it (FP32, autotuned tiles,
    graph chunks, 5 increments): every problem converges, and one problem of
    each grid size matches the oracle (48^3 on its first two increments)."""
    wls = problems(range(512))
    laws = [W.pa66(), W.e_glass()]
    b = hom.Batch([w.phases for w in wls], laws, scheme=hom.SCHEME_NEWTON_CG, precision=hom.FP32, tol=1e-6,
                  autotune=1)
    picks = {}
    for i, w in enumerate(wls):
        picks.setdefault(w.record["n"], i)
    assert sorted(picks) == [24, 32, 48]
    refs = {i: solver.Cell(wls[i].phases, laws) for i in picks.values()}
    for k in range(5):
        strains = np.array([w.history[k].strain for w in wls])
        rb = b.solve_increment(strains, [w.history[k].theta for w in wls], [w.history[k].grad for w in wls],
                               [w.history[k].dt for w in wls])
        assert all(r["status"] == 0 for r in rb)
        for n, i in picks.items():
            if n == 48 and k >= 2:
                continue
            st = wls[i].history[k]
            o = refs[i].solve_increment(st.strain, st.theta, st.grad, st.dt, tol=1e-9)
            scale = max(np.abs(o["stress"]).max(), 1e-3)
            err = np.abs(rb[i]["stress"] - o["stress"]).max() / scale
            print(f"batch of 512, problem {i} (n={n}) inc {k}: stress err {err:.2e}", flush=True)
            assert err <= FP32_BOUND
            assert np.allclose(rb[i]["heat_flux"], o["heat_flux"], rtol=FP32_BOUND)


def test_autotuned_schedules_are_reported_and_solve_alike():
    """The autotuner times every y / z schedule (tile width, FFT plan) per grid
    group and keeps the fastest; whatever it keeps, the batch solves as the
    untuned one does (FP32 bound), and the chosen schedules are valid ones."""
    wls = [w for w in problems(range(12)) if w.record["n"] == 24][:2]
    wls += [w for w in problems(range(12)) if w.record["n"] == 32][:1]
    laws = [W.pa66(), W.e_glass()]
    opts = dict(scheme=hom.SCHEME_NEWTON_CG, precision=hom.FP32, tol=1e-6)
    tuned = hom.Batch([w.phases for w in wls], laws, autotune=1, **opts)
    plain = hom.Batch([w.phases for w in wls], laws, autotune=0, **opts)
    sched = tuned.schedules()
    print(f"autotuned schedules: {sched}", flush=True)
    assert sorted(tuple(s["grid"]) for s in sched) == [(24, 24, 24), (32, 32, 32)]
    for s in sched:
        for k in ("y_mech", "z_mech", "y_thermal", "z_thermal"):
            assert s[k]["tile"] in (2, 4, 8) and s[k]["plan"] in (0, 1)
    for s in plain.schedules():
        assert all(s[k] == {"tile": 4, "plan": 0} for k in ("y_mech", "z_mech", "y_thermal", "z_thermal"))
    st = [w.history[0] for w in wls]
    args = (np.array([h.strain for h in st]), [h.theta for h in st], [h.grad for h in st], [h.dt for h in st])
    rt, rp = tuned.solve_increment(*args), plain.solve_increment(*args)
    for a, b in zip(rt, rp):
        assert a["status"] == 0 and b["status"] == 0
        assert np.abs(a["stress"] - b["stress"]).max() <= 2 * FP32_BOUND * np.abs(b["stress"]).max()
