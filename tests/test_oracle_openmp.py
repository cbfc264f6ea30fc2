"""The oracle's OpenMP timing build (the all-cores CPU baseline) against its plain build: the same
arithmetic up to summation order, and the switch back to the plain build that every check uses."""

import os

import numpy as np

import oracle as O
from paper_2502_10872_amd import inputs as I


def test_openmp_build_matches_the_plain_build():
    mesh = I.sphere_cap_mesh(48, 0.8, 0.9, 0.2, 7, "SS", "ring")
    m = I.MATERIAL
    x = mesh.X + 1e-3 * np.sin(3.0 * mesh.X[:, [1, 2, 0]])
    res = {}
    try:
        for omp in (False, True):
            threads = O.use_openmp(omp, 4 if omp else 0)
            assert threads == (min(4, threads) if omp else 1)
            st = O.Stencils("SS", mesh.X, mesh.tris, m["young"], m["poisson"], m["thickness"])
            f, e = st.forces(x)
            sim = O.Sim(st, m, mesh.pinned)
            counts, stats = sim.step(1 / 30, max_newton=2, replay=np.array([[25, 25, 25], [25, 25, 25]], np.int32))
            res[omp] = (f, e, sim.x.copy(), stats["grad_norm"])
    finally:
        assert O.use_openmp(False) == 1
    (f0, e0, x0, g0), (f1, e1, x1, g1) = res[False], res[True]
    assert np.linalg.norm(f1 - f0) <= 1e-12 * np.linalg.norm(f0)
    assert abs(e1 - e0) <= 1e-12 * abs(e0)
    u0 = x0 - mesh.X
    assert np.linalg.norm(x1 - x0) <= 1e-10 * np.linalg.norm(u0)
    assert abs(g1 - g0) <= 1e-8 * g0


def test_openmp_build_uses_the_requested_threads():
    try:
        n = O.use_openmp(True, 2)
        assert n == 2 or (os.cpu_count() or 1) < 2
    finally:
        O.use_openmp(False)
