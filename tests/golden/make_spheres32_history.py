"""Writes spheres32_history.json: the oracle's effective outputs over the
whole 20-increment shear/tension history with the cyclic temperature
(293.15-373.15 K, two heating and two cooling halves) on the 32^3 RSA sphere
composite (PA66 matrix, E-glass spheres, seed 2).

Test infrastructure: calls only the oracle and the seeded input generator.
Run from the repository root:  python tests/golden/make_spheres32_history.py
"""
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import solver  # noqa: E402
from paper_2109_14403_amd import workloads as W  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "spheres32_history.json")


def main():
    wl = W.sphere_composite_workload(32, seed=2)
    ref = solver.Cell(wl.phases, wl.laws)
    rows = []
    for k, st in enumerate(wl.history):
        o = ref.solve_increment(st.strain, st.theta, st.grad, st.dt, tol=1e-10)
        rows.append(dict(increment=k + 1, strain=list(map(float, st.strain)), theta=float(st.theta),
                         grad=list(map(float, st.grad)), dt=float(st.dt),
                         stress=list(map(float, o["stress"])), heat_flux=list(map(float, o["heat_flux"])),
                         dissipation=o["dissipation"], coupling=o["coupling"], heat_capacity=o["heat_capacity"]))
        print(f"increment {k + 1}: theta {st.theta:.2f} stress11 {o['stress'][0]:.6f}", flush=True)
    doc = dict(source="oracle/solver.py Cell.solve_increment, Newton-CG, tol 1e-10 (FP64); "
                      "workload paper_2109_14403_amd.workloads.sphere_composite_workload(32, seed=2)",
               voxels=int(wl.phases.size), inclusion_fraction=float((wl.phases == 1).mean()), increments=rows)
    with open(OUT, "w") as f:
        json.dump(doc, f, indent=1)


if __name__ == "__main__":
    main()
