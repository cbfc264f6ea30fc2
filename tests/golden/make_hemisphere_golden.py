"""Writes hemisphere_ss_1088.json: the FP64 oracle's quasi-static equilibrium of the pinched hemisphere
(Sec. 6: R = 10, 18 degree hole, four radial loads of 200 on the equator, E = 6.825e7, nu = 0.3, h = 0.04;
x held on the plane x = 0, y on y = 0, z of the hole-rim vertices on x = 0; 17 rings x 64 vertices),
smoothed shell with its membrane, Newton-Raphson with eps_f = 1e-3 and eps_u = 0.1, PCG rtol 1e-10.
Calls the oracle only.  Run from the repository root: python tests/golden/make_hemisphere_golden.py"""

import json
import os
import sys

import numpy as np

sys.path.insert(0, os.path.join(os.path.dirname(os.path.abspath(__file__)), "..", ".."))

import oracle as O  # noqa: E402
from paper_2502_10872_amd import inputs as I  # noqa: E402


def main():
    mesh, held, F, (ia, ib) = I.hemisphere_problem(17, 64, model="SS")
    mat = I.HEMISPHERE_MATERIAL
    st = O.Stencils("SS", mesh.X, mesh.tris, mat["young"], mat["poisson"], mat["thickness"])
    x, _, stats = O.solve_static_membrane(st, np.zeros(mesh.nv), F, eps_f=1e-3, eps_u=0.1, max_newton=250,
                                          pcg_rtol=1e-10, held=held)
    u = x - mesh.X
    sample = list(range(0, mesh.nv, 17)) + [int(ia), int(ib)]
    out = dict(source="oracle.solve_static_membrane, SS, 17 x 64 hemisphere, eps_f 1e-3, eps_u 0.1, rtol 1e-10",
               newton_iters=stats["newton_iters"], pcg_total=stats["pcg_total"], resid=stats["resid"],
               u_min=float(u[:, 0].min()), v_max=float(u[:, 1].max()),
               load_point_x=[float(c) for c in u[ia]], load_point_y=[float(c) for c in u[ib]],
               sample_vertices=sample, sample_displacements=[[float(c) for c in u[k]] for k in sample])
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "hemisphere_ss_1088.json")
    with open(path, "w") as fh:
        json.dump(out, fh, indent=1)
    print(f"wrote {path}: newton {stats['newton_iters']}, u_min {out['u_min']:.5f}, v_max {out['v_max']:.5f}")


if __name__ == "__main__":
    main()
