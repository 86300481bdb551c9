"""Parity at full size, in the configuration the benchmark times.

256^3 short-fibre composite, FP32 fields with FP64 reductions and return
mapping, Newton-CG at tolerance 1e-6, autotuned tiles, the first three
increments of its load history. The oracle cannot solve this grid, so the
checks are ones it can make one voxel at a time, plus properties that hold at
any size:

* sampled voxels (random matrix voxels, the most plastic ones, random fibre
  voxels): the stress and the committed internal variables of the HIP solver
  against the oracle's point laws (Sec. 4), fed with the solver's own strain
  and the internal variables of step n;
* the effective stress is the volume average of the stress field (Sec. 2);
* the converged stress field is in equilibrium: the projection P(n) of its
  spectrum (Sec. 3.2 projector) is below the Newton tolerance;
* the strain fluctuation is compatible: P(n) leaves its spectrum unchanged.

The 64^3 sphere composite is small enough for the oracle itself: its first
two increments are compared on the effective quantities.
"""
import math

import numpy as np
import pytest
import scipy.fft

from oracle import fourier, green, solver
from oracle.laws import PA66, Thermoelastic
from paper_2109_14403_amd import hom
from test_gpu_solver import FP32_BOUND
from paper_2109_14403_amd import workloads as W

pytestmark = pytest.mark.gpu

TOL = 1e-6
SQ2 = math.sqrt(2.0)


def spectrum(field):
    """Full complex spectra of the components (c, nz, ny, nx)."""
    return scipy.fft.fftn(field, axes=(-3, -2, -1), workers=16)


def projected_ratio(spec, n_dir, slab=16):
    """|P(n) spec| / |spec| over all frequencies (Parseval), in kz slabs."""
    num = den = 0.0
    for z0 in range(0, spec.shape[1], slab):
        s = spec[:, z0:z0 + slab]
        p = green.projector(s, n_dir[:, z0:z0 + slab])
        num += float((np.abs(p) ** 2).sum())
        den += float((np.abs(s) ** 2).sum())
    return math.sqrt(num / den)


@pytest.fixture(scope="module")
def fibres256():
    wl = W.fibre_composite_workload(256, seed=3)
    ctx = hom.Context(wl.phases, wl.laws, scheme=hom.SCHEME_NEWTON_CG, precision=hom.FP32, tol=TOL, autotune=1)
    steps = wl.history[:3]
    for st in steps[:2]:
        r = ctx.solve_increment(st.strain, st.theta, st.grad, st.dt)
        print(f"256^3 increment: newton {r['newton_iters']} krylov {r['krylov_iters']}", flush=True)
    rng = np.random.default_rng(11)
    phase = wl.phases.reshape(-1)
    matrix = np.flatnonzero(phase == 0)
    fibre = np.flatnonzero(phase == 1)
    eps_n = ctx.field(hom.FIELD_STRAIN).reshape(6, -1)
    state_n = ctx.field(hom.FIELD_STATE).reshape(-1, phase.size)
    st = steps[2]
    res = ctx.solve_increment(st.strain, st.theta, st.grad, st.dt)
    print(f"256^3 increment: newton {res['newton_iters']} krylov {res['krylov_iters']}", flush=True)
    state1 = ctx.field(hom.FIELD_STATE).reshape(-1, phase.size)
    plastic = matrix[np.argsort(state1[0, matrix])[-1000:]]     # largest eps_p after the increment
    samples_m = np.concatenate([rng.choice(matrix, 2000, replace=False), plastic])
    samples_f = rng.choice(fibre, 500, replace=False)
    sm = dict(eps_n=eps_n[:, samples_m].copy(), state_n=state_n[:, samples_m].copy(),
              state1=state1[:, samples_m].copy())
    del state_n, state1
    eps = ctx.field(hom.FIELD_STRAIN)
    sig = ctx.field(hom.FIELD_STRESS)
    ctx.close()
    return dict(wl=wl, step=st, res=res, eps=eps, sig=sig, samples_m=samples_m, samples_f=samples_f,
                eps_n_f=eps_n[:, samples_f].copy(), **sm)


def test_fibres256_sampled_voxels_match_point_laws(fibres256):
    d = fibres256
    st = d["step"]
    law = PA66(W.pa66())
    m = d["samples_m"]
    eps = d["eps"].reshape(6, -1)[:, m]
    sig = d["sig"].reshape(6, -1)[:, m]
    sn = d["state_n"]
    state = {"ep": sn[0], "evp": sn[1:7], "ev": sn[7:].reshape(law.N, 6, -1)}
    ref = law.update(eps, d["eps_n"], state, st.theta, st.dt)
    scale = np.abs(ref["sigma"]).max(axis=0) + 1e-3
    err = (np.abs(sig - ref["sigma"]).max(axis=0) / scale).max()
    print(f"matrix voxels: max stress error {err:.2e}, plastic {np.count_nonzero(ref['delta'] > 0)} of {m.size}")
    assert np.count_nonzero(ref["delta"] > 0) >= 500
    assert err <= 1e-6                       # the field is stored in FP32
    s1 = d["state1"]
    rs = ref["state"]
    ref_flat = np.concatenate([rs["ep"][None], rs["evp"], rs["ev"].reshape(-1, m.size)])
    assert np.allclose(s1, ref_flat, rtol=1e-8, atol=1e-13)
    f = d["samples_f"]
    glass = Thermoelastic(W.e_glass())
    eps_f = d["eps"].reshape(6, -1)[:, f]
    sig_f = d["sig"].reshape(6, -1)[:, f]
    ref_f = glass.stress(eps_f, st.theta)
    assert (np.abs(sig_f - ref_f).max(axis=0) <= 1e-6 * (np.abs(ref_f).max(axis=0) + 1e-3)).all()


def test_fibres256_effective_stress_is_volume_average(fibres256):
    d = fibres256
    mean = d["sig"].reshape(6, -1).mean(axis=1)
    mean_tensor = np.concatenate([mean[:3], mean[3:] / SQ2])       # Mandel -> tensor components
    got = np.asarray(d["res"]["stress"])
    assert np.abs(got - mean_tensor).max() <= 1e-6 * np.abs(got).max()
    assert np.abs(d["eps"].reshape(6, -1).mean(axis=1)[0] - d["step"].strain[0]) <= 1e-6 * abs(d["step"].strain[0])


def test_fibres256_equilibrium_and_compatibility(fibres256):
    d = fibres256
    n_dir = fourier.directions(d["sig"].shape[1:])
    ratio = projected_ratio(spectrum(d["sig"]), n_dir)
    print(f"|P sigma| / |sigma| = {ratio:.2e}")
    assert ratio <= 2 * TOL
    fluct = d["eps"] - d["eps"].reshape(6, -1).mean(axis=1)[:, None, None, None]
    spec = spectrum(fluct)
    comp = projected_ratio(spec, n_dir)
    print(f"|P eps~| / |eps~| = {comp:.8f}")
    assert abs(comp - 1.0) <= 1e-5


def test_spheres64_matches_oracle():
    wl = W.sphere_composite_workload(64, seed=2)
    ctx = hom.Context(wl.phases, wl.laws, scheme=hom.SCHEME_NEWTON_CG, precision=hom.FP32, tol=TOL, autotune=1)
    ref = solver.Cell(wl.phases, wl.laws)
    outs = []
    for st in wl.history[:2]:
        g = ctx.solve_increment(st.strain, st.theta, st.grad, st.dt)
        o = ref.solve_increment(st.strain, st.theta, st.grad, st.dt, tol=1e-8)
        outs.append((g, o))
    scale = max(np.abs(o["stress"]).max() for _, o in outs)
    for k, (g, o) in enumerate(outs):
        err_s = np.abs(g["stress"] - o["stress"]).max() / scale
        err_q = np.abs(g["heat_flux"] - o["heat_flux"]).max() / np.abs(o["heat_flux"]).max()
        err_c = abs(g["coupling"] - o["coupling"]) / abs(o["coupling"])
        print(f"spheres64 inc {k}: stress {err_s:.2e} flux {err_q:.2e} coupling {err_c:.2e}", flush=True)
        assert err_s <= FP32_BOUND and err_q <= FP32_BOUND and err_c <= FP32_BOUND
