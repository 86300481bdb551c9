"""The direct DMN (Sec. 3) on the GPU against the oracle.

Offline: the linear homogenization function (the GPU uses the exact
laminate rule with a 3 x 3 solve, the oracle the lambda form of Sec. 3.2),
the loss and its gradients (hand-written reverse mode against torch
autograd), and training that fits a DMN to data of another DMN. Online: the
Newton iteration on the displacement jumps with PA66 and E-glass leaves
(the GPU eliminates the jumps laminate by laminate, the oracle solves the
dense system), stress, coupling term, dissipation and d<sigma>/dE over
several increments.
"""
import numpy as np
import pytest

from oracle import dmn, tensor
from paper_2109_14403_amd import hom
from paper_2109_14403_amd import workloads as W

pytestmark = pytest.mark.gpu

SQ2 = np.sqrt(2.0)
WM = np.array([1, 1, 1, SQ2, SQ2, SQ2])


def samples(n, rng, rank_one=True):
    """Isotropic C1 (fibres) and isotropic-minus-rank-one C2 (matrix), the
    paper's form of the sampled stiffness pairs."""
    C1, C2 = [], []
    for _ in range(n):
        K1, G1 = np.exp(rng.uniform(np.log(5e3), np.log(8e4), 2))
        K2, G2 = np.exp(rng.uniform(np.log(5e2), np.log(8e3), 2))
        C1.append(tensor.isotropic(K1, G1))
        c2 = tensor.isotropic(K2, G2)
        if rank_one:
            N = tensor.deviator(rng.standard_normal(6))
            N /= np.linalg.norm(N)
            c2 = c2 - 2 * G2 * rng.uniform(0, 0.95) * np.outer(N, N)
        C2.append(c2)
    return np.array(C1), np.array(C2)


def random_params(K, rng, negative=0):
    m = rng.standard_normal((2 ** K - 1, 3))
    v = rng.uniform(0.05, 1.0, 2 ** K)
    v /= v.sum()
    if negative:
        v[rng.choice(2 ** K, negative, replace=False)] = -0.01
    return m, v


@pytest.mark.parametrize("K,negative", [(1, 0), (4, 0), (8, 0), (8, 9)])
def test_homogenize_matches_oracle(K, negative):
    rng = np.random.default_rng(K + 10 * negative)
    m, v = random_params(K, rng, negative)
    C1, C2 = samples(64, rng)
    net = hom.Dmn(K)
    net.set_params(m, v)
    got = net.homogenize(C1, C2)
    ref = dmn.homogenize_np(C1, C2, m, v)
    err = np.abs(got - ref).max() / np.abs(ref).max()
    print(f"K={K} negative={negative}: homogenize {err:.2e}", flush=True)
    assert err <= 1e-10
    assert np.allclose(got, got.transpose(0, 2, 1), atol=1e-9 * np.abs(got).max())


@pytest.mark.parametrize("K,negative", [(3, 0), (6, 5)])
def test_loss_and_gradients_match_autograd(K, negative):
    rng = np.random.default_rng(50 + K)
    m, v = random_params(K, rng, negative)
    C1, C2 = samples(16, rng)
    Ceff = dmn.homogenize_np(C1, C2, *random_params(K, rng)) * rng.uniform(0.95, 1.05, (16, 1, 1))
    J, gm, gv = dmn.loss_and_grad(C1, C2, Ceff, m, v * 1.02)
    net = hom.Dmn(K)
    net.set_params(m, v * 1.02)
    Jg, gmg, gvg = net.loss_grad(C1, C2, Ceff)
    em = np.abs(gmg - gm).max() / np.abs(gm).max()
    ev = np.abs(gvg - gv).max() / np.abs(gv).max()
    print(f"K={K}: loss {abs(Jg - J) / J:.2e} grad m {em:.2e} grad v {ev:.2e}", flush=True)
    assert abs(Jg - J) <= 1e-10 * J
    assert em <= 1e-7 and ev <= 1e-7
    assert np.all(gvg[v < 0] == 0.0)


def test_training_fits_a_teacher_network():
    rng = np.random.default_rng(3)
    K = 4
    teacher = random_params(K, rng)
    C1, C2 = samples(320, rng)
    Ceff = dmn.homogenize_np(C1, C2, *teacher)
    net = hom.Dmn(K, seed=11)
    before = np.mean(np.abs(net.homogenize(C1, C2) - Ceff).sum(axis=(1, 2)) / np.abs(Ceff).sum(axis=(1, 2)))
    hist = net.train(C1, C2, Ceff, epochs=1000, batch=32, seed=5)
    after = np.mean(np.abs(net.homogenize(C1, C2) - Ceff).sum(axis=(1, 2)) / np.abs(Ceff).sum(axis=(1, 2)))
    m, v = net.params()
    print(f"mean error {before:.3e} -> {after:.3e}, loss {hist[0]:.3e} -> {hist[-1]:.3e}, sum w {np.maximum(v, 0).sum():.4f}",
          flush=True)
    assert after < 0.2 * before
    assert hist[-1] < hist[0]
    assert abs(np.maximum(v, 0).sum() - 1.0) < 0.02


def oracle_online(m, v, law1, law2, npts, tol):
    return [dmn.OnlineDMN(m, v, law1, law2, tol=tol) for _ in range(npts)]


@pytest.mark.parametrize("K", [1, 2, 3, 6, 7, 8])
def test_online_matches_oracle(K):
    rng = np.random.default_rng(70 + K)
    m, v = random_params(K, rng)
    law1, law2 = W.e_glass(), W.pa66()
    npts = 3
    tol = 1e-10
    gpu = hom.DmnOnline(_net(K, m, v), law1, law2, npts, tol=tol)
    ref = oracle_online(m, v, law1, law2, npts, tol)
    dirs = np.array([[1, 0, 0, 0, 0, 0.4], [0.3, -0.2, 1, 0, 0.5, 0], [0, 0, 0, 1, 0, 0]], dtype=float)
    plastic = False
    for k in range(1, 5):
        strains = dirs * 0.008 * k
        theta = 293.15 + 10 * k
        what = k % 2                               # all four tangents on every other increment
        out = gpu.step(strains, theta, 2.0, what=what)
        for i in range(npts):
            o = ref[i].step(strains[i], theta, 2.0, all_tangents=bool(what))
            g = out[i]
            if what:
                et2 = max(np.abs(g["dsdt"] - o["dsdt"] / WM).max() / np.abs(o["dsdt"]).max(),
                          np.abs(g["dDde"] - o["dDde"] * WM).max() / np.abs(o["dDde"]).max(),
                          abs(g["dDdt"] - o["dDdt"]) / abs(o["dDdt"]))
                print(f"K={K} inc {k} point {i}: temperature / coupling tangents {et2:.2e}", flush=True)
                assert et2 <= 1e-6
            else:
                assert np.isnan(g["dsdt"]).all() and np.isnan(g["dDdt"])
            es = np.abs(g["stress"] - o["stress"]).max() / np.abs(o["stress"]).max()
            dsde_o = o["dsde"] * WM[None, :] / WM[:, None]
            et = np.abs(g["dsde"] - dsde_o).max() / np.abs(dsde_o).max()
            ec = abs(g["coupling"] - o["coupling"]) / max(abs(o["coupling"]), 1e-9)
            ed = abs(g["dissipation"] - o["dissipation"]) / max(abs(o["dissipation"]), 1e-12)
            print(f"K={K} inc {k} point {i}: stress {es:.2e} dsde {et:.2e} coupling {ec:.2e} dissipation {ed:.2e}"
                  f" newton {g['newton_iters']}/{o['newton_iters']}", flush=True)
            assert g["status"] == hom.HOM_OK
            assert es <= 1e-8 and et <= 1e-7 and ec <= 1e-7 and ed <= 1e-6
            plastic = plastic or o["dissipation"] > 0.0
    assert plastic


def _net(K, m, v):
    net = hom.Dmn(K)
    net.set_params(m, v)
    return net


def test_online_linear_phases_equal_offline():
    rng = np.random.default_rng(9)
    K = 8
    m, v = random_params(K, rng)
    l1 = dict(kind="thermoelastic", E=70e3, nu=0.22, alpha0=5e-6, kappa0=1.0, c0=2.0, theta0=293.15)
    l2 = dict(l1, E=3e3, nu=0.35)
    net = _net(K, m, v)
    C1 = tensor.isotropic(*tensor.bulk_shear(l1["E"], l1["nu"]))
    C2 = tensor.isotropic(*tensor.bulk_shear(l2["E"], l2["nu"]))
    D = net.homogenize(C1[None], C2[None])[0]
    on = hom.DmnOnline(net, l1, l2, 2, tol=1e-12)
    strains = np.array([[2e-3, -1e-3, 5e-4, 3e-4, 0, -2e-4], [0, 0, 1e-3, 0, 2e-3, 0]])
    out = on.step(strains, 293.15, 1.0)
    for i in range(2):
        expect = tensor.mandel_to_components(D @ tensor.components_to_mandel(strains[i]))
        assert np.allclose(out[i]["stress"], expect, rtol=1e-9, atol=1e-9 * np.abs(expect).max())
        assert np.allclose(out[i]["dsde"], D * WM[None, :] / WM[:, None], rtol=1e-8, atol=1e-8 * np.abs(D).max())


def test_dmn_argument_errors():
    with pytest.raises(hom.HomError):
        hom.Dmn(11)
    net = hom.Dmn(9)
    with pytest.raises(hom.HomError) as e:
        hom.DmnOnline(net, W.e_glass(), W.pa66(), 4)
    assert e.value.code == hom.HOM_E_UNSUPPORTED
    net = hom.Dmn(3)
    with pytest.raises(hom.HomError):
        net.set_params(np.zeros((7, 3)), np.ones(8))
    with pytest.raises(hom.HomError):
        hom.DmnOnline(net, W.pa66(), W.pa66(), 4)      # at most one PA66 law


def test_online_trial_steps_commit_nothing():
    rng = np.random.default_rng(31)
    K = 5
    m, v = random_params(K, rng)
    net = _net(K, m, v)
    a = hom.DmnOnline(net, W.e_glass(), W.pa66(), 2, tol=1e-12)
    b = hom.DmnOnline(net, W.e_glass(), W.pa66(), 2, tol=1e-12)
    d = np.array([[1, 0, 0, 0, 0, 0.4], [0, 0.5, -0.2, 0.3, 0, 0]], dtype=float)
    for k in (1, 2):
        a.step(d * 0.01 * k, 300.0, 2.0)
        b.step(d * 0.01 * k, 300.0, 2.0)
    a.step(d * 0.045, 300.0, 2.0, trial=True)
    t = a.step(d * 0.03, 300.0, 2.0, trial=True, what=1)
    ra = a.step(d * 0.03, 300.0, 2.0)
    rb = b.step(d * 0.03, 300.0, 2.0, what=1)
    for i in range(2):
        for r in (ra[i], t[i]):
            assert np.allclose(r["stress"], rb[i]["stress"], rtol=1e-10, atol=1e-10 * np.abs(rb[i]["stress"]).max())
            assert abs(r["dissipation"] - rb[i]["dissipation"]) <= 1e-9 * abs(rb[i]["dissipation"])
        assert np.allclose(t[i]["dDde"], rb[i]["dDde"], rtol=1e-8, atol=1e-8 * np.abs(rb[i]["dDde"]).max())
    # the next increment after the commit agrees too
    ra = a.step(d * 0.04, 300.0, 2.0)
    rb = b.step(d * 0.04, 300.0, 2.0)
    for i in range(2):
        assert np.allclose(ra[i]["stress"], rb[i]["stress"], rtol=1e-10, atol=1e-10 * np.abs(rb[i]["stress"]).max())


def test_online_points_with_their_own_temperature_and_step():
    """Per-point theta and dt (some repeated, some not) give each point the
    result of a one-point evaluation with its own history."""
    rng = np.random.default_rng(44)
    K = 7
    m, v = random_params(K, rng)
    net = _net(K, m, v)
    thetas = np.array([300.0, 310.0, 300.0, 325.0, 310.0])
    dts = np.array([2.0, 2.0, 0.5, 2.0, 2.0])
    d = rng.standard_normal((5, 6))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    many = hom.DmnOnline(net, W.e_glass(), W.pa66(), 5, tol=1e-11)
    ones = [hom.DmnOnline(net, W.e_glass(), W.pa66(), 1, tol=1e-11) for _ in range(5)]
    for k in (1, 2, 3):
        th = thetas + 2.0 * k
        out = many.step(d * 0.006 * k, th, dts, what=k % 2)
        for i in range(5):
            r = ones[i].step(d[i:i + 1] * 0.006 * k, th[i], dts[i], what=k % 2)[0]
            assert out[i]["status"] == hom.HOM_OK and r["status"] == hom.HOM_OK
            assert out[i]["newton_iters"] == r["newton_iters"]
            for key in ("stress", "dsde", "coupling", "dissipation") + (("dsdt", "dDde", "dDdt") if k % 2 else ()):
                a, b = np.asarray(out[i][key]), np.asarray(r[key])
                assert np.allclose(a, b, rtol=1e-12, atol=1e-12 * max(np.abs(b).max(), 1e-30)), (k, i, key)
    assert out["dissipation"].max() > 0.0
    many.close()
    for o in ones:
        o.close()
    net.close()


@pytest.mark.parametrize("K", [6, 8])
def test_online_predictor_same_solutions_fewer_newton_steps(K):
    rng = np.random.default_rng(80 + K)
    m, v = random_params(K, rng)
    net = _net(K, m, v)
    npts = 4
    d = rng.standard_normal((npts, 6))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    runs = []
    for pred in (False, True):
        # both runs converged far below the comparison bound (the stop test
        # bounds the traction residual, not the stress)
        on = hom.DmnOnline(net, W.e_glass(), W.pa66(), npts, tol=1e-12, predictor=pred)
        runs.append([on.step(d * 0.006 * k, 293.15 + 5 * k, 2.0) for k in range(1, 7)])
        on.close()
    for k, (a, b) in enumerate(zip(*runs)):
        assert (a["status"] == hom.HOM_OK).all() and (b["status"] == hom.HOM_OK).all()
        for key, bound in (("stress", 1e-8), ("dsde", 1e-6), ("dissipation", 1e-6)):
            x, y = np.asarray(a[key]), np.asarray(b[key])
            assert np.abs(x - y).max() <= bound * np.abs(x).max(), (k, key)
    na = sum(int(r["newton_iters"].sum()) for r in runs[0][2:])
    nb = sum(int(r["newton_iters"].sum()) for r in runs[1][2:])
    print(f"K={K}: Newton steps of increments 3..6: {na} -> {nb}", flush=True)
    assert nb < na
    net.close()


def test_online_predictor_with_trial_steps():
    """Trials in between: no shift after a trial, the commit equals the plain run."""
    rng = np.random.default_rng(33)
    K = 5
    m, v = random_params(K, rng)
    net = _net(K, m, v)
    d = np.array([[1, 0, 0, 0, 0, 0.4], [0, 0.5, -0.2, 0.3, 0, 0]], dtype=float)
    a = hom.DmnOnline(net, W.e_glass(), W.pa66(), 2, tol=1e-12, predictor=True)
    b = hom.DmnOnline(net, W.e_glass(), W.pa66(), 2, tol=1e-12)
    for k in (1, 2, 3):
        a.step(d * 0.008 * k, 300.0, 2.0)
        b.step(d * 0.008 * k, 300.0, 2.0)
    a.step(d * 0.036, 300.0, 2.0, trial=True)
    ra = a.step(d * 0.032, 300.0, 2.0)
    rb = b.step(d * 0.032, 300.0, 2.0)
    ra2 = a.step(d * 0.040, 300.0, 2.0)
    rb2 = b.step(d * 0.040, 300.0, 2.0)
    for x, y in ((ra, rb), (ra2, rb2)):
        assert np.allclose(x["stress"], y["stress"], rtol=1e-9, atol=1e-9 * np.abs(y["stress"]).max())
        assert np.allclose(x["dissipation"], y["dissipation"], rtol=1e-8)
    assert a._lib.hom_dmn_online_set_predictor(a._h, 2) == hom.HOM_E_ARG
    assert a._lib.hom_dmn_online_set_predictor(None, 1) == hom.HOM_E_ARG
    a.close()
    b.close()
    net.close()


def test_online_predictor_switched_off_and_on_again_starts_over():
    """An increment solved with the predictor off records no jump change: the
    first call after switching it on again starts from the current jumps
    (bitwise the run that stays off), the next one extrapolates again."""
    rng = np.random.default_rng(34)
    K = 5
    m, v = random_params(K, rng)
    net = _net(K, m, v)
    d = rng.standard_normal((4, 6))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    a = hom.DmnOnline(net, W.e_glass(), W.pa66(), 4, tol=1e-12, predictor=True)
    b = hom.DmnOnline(net, W.e_glass(), W.pa66(), 4, tol=1e-12, predictor=True)
    for k in (1, 2, 3):
        a.step(d * 0.006 * k, 300.0, 2.0)
        b.step(d * 0.006 * k, 300.0, 2.0)
    a.set_predictor(False)
    b.set_predictor(False)
    a.step(d * 0.024, 300.0, 2.0)
    b.step(d * 0.024, 300.0, 2.0)
    a.set_predictor(True)
    ra = a.step(d * 0.030, 300.0, 2.0)
    rb = b.step(d * 0.030, 300.0, 2.0)
    assert (ra["status"] == hom.HOM_OK).all() and (rb["status"] == hom.HOM_OK).all()
    assert np.array_equal(ra["stress"], rb["stress"])
    assert np.array_equal(ra["newton_iters"], rb["newton_iters"])
    ra = a.step(d * 0.036, 300.0, 2.0)
    rb = b.step(d * 0.036, 300.0, 2.0)
    assert np.abs(ra["stress"] - rb["stress"]).max() <= 1e-8 * np.abs(rb["stress"]).max()
    assert int(ra["newton_iters"].sum()) <= int(rb["newton_iters"].sum())
    a.close()
    b.close()
    net.close()
