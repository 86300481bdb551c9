"""The whole 20-increment history of the 64^3-recipe sphere composite, at
32^3, against the oracle: mixed shear/tension to 2 % under the cyclic
temperature 293.15-373.15 K (Sec. 4 WLF shift and softening over both
heating and both cooling halves). The oracle's outputs are stored in
tests/golden/spheres32_history.json by tests/golden/make_spheres32_history.py."""
import json
import os

import numpy as np
import pytest

from paper_2109_14403_amd import hom
from paper_2109_14403_amd import workloads as W
from test_gpu_solver import FP32_BOUND

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "spheres32_history.json")


@pytest.fixture(scope="module")
def history():
    with open(GOLDEN) as f:
        doc = json.load(f)
    wl = W.sphere_composite_workload(32, seed=2)
    rows = doc["increments"]
    assert len(rows) == len(wl.history) == 20
    for r, st in zip(rows, wl.history):
        assert np.allclose(r["strain"], st.strain, rtol=0, atol=1e-15) and r["theta"] == st.theta
    return wl, rows


@pytest.mark.parametrize("precision,tol,bound", [(hom.FP64, 1e-10, 1e-5), (hom.FP32, 1e-6, FP32_BOUND)])
def test_spheres32_full_cyclic_history(history, precision, tol, bound):
    wl, rows = history
    ctx = hom.Context(wl.phases, wl.laws, scheme=hom.SCHEME_NEWTON_CG, precision=precision, tol=tol)
    scale = max(np.abs(r["stress"]).max() for r in rows)
    dscale = max(abs(r["dissipation"]) for r in rows)
    cscale = max(abs(r["coupling"]) for r in rows)
    worst = dict(stress=0.0, flux=0.0, coupling=0.0, dissipation=0.0)
    for st, r in zip(wl.history, rows):
        g = ctx.solve_increment(st.strain, st.theta, st.grad, st.dt)
        assert g["status"] == 0
        e = dict(stress=np.abs(g["stress"] - r["stress"]).max() / scale,
                 flux=np.abs(g["heat_flux"] - r["heat_flux"]).max() / np.abs(r["heat_flux"]).max(),
                 coupling=abs(g["coupling"] - r["coupling"]) / cscale,
                 dissipation=abs(g["dissipation"] - r["dissipation"]) / dscale)
        print(f"spheres32 history prec {precision} inc {r['increment']} theta {st.theta:.2f}: "
              + " ".join(f"{k} {v:.2e}" for k, v in e.items())
              + f" newton {g['newton_iters']} krylov {g['krylov_iters']}", flush=True)
        for k, v in e.items():
            worst[k] = max(worst[k], v)
        assert g["heat_capacity"] == pytest.approx(r["heat_capacity"], rel=1e-12)
    print(f"spheres32 history prec {precision} worst: " + " ".join(f"{k} {v:.2e}" for k, v in worst.items()))
    for k, v in worst.items():
        assert v <= bound, (k, v)
    ctx.close()
