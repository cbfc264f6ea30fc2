"""ctypes wrapper of the plain FP64 CPU oracle (shell_oracle.c).

TEST INFRASTRUCTURE ONLY: imported by tests/, by the smoke check and by the
CPU-baseline leg of the benchmark.  The product path (the HIP library and its
Python binding) never imports it, and it imports nothing from the product.

Each function cites the passage of the paper it follows in shell_oracle.c.
"""

from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "shell_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
WORLD_FRAME = 1  # orc_build flag: the world-frame (App. D) edge operator

MODELS = ("EP", "ES", "FP", "FS", "SP", "SS")
ERRORS = {-1: "invalid argument", -2: "non-manifold mesh", -3: "inconsistent orientation",
          -4: "degenerate stencil", -5: "iteration budget exhausted"}


class OracleError(RuntimeError):
    def __init__(self, code: int, what: str):
        super().__init__(f"{what}: {ERRORS.get(code, code)}")
        self.code = code


_LIB_OMP = os.path.join(_HERE, "liboracle_omp.so")


def build(openmp: bool = False) -> str:
    """Compile the oracle with gcc (plain -O2, no fast-math, no FMA contraction).  openmp: the timing
    build of the same source, whose stencil loop, sparse product and vector loops run on all cores."""
    out = _LIB_OMP if openmp else _LIB
    cmd = ["gcc", "-O2", "-std=c99", "-ffp-contract=off", "-fPIC", "-shared"] + (["-fopenmp"] if openmp else []) + \
        ["-o", out, _SRC, "-lm"]
    subprocess.run(cmd, check=True)
    return out


_lib = None
_variant = False  # True: the OpenMP timing build is the one loaded


def use_openmp(enable: bool, threads: int = 0) -> int:
    """Switch later oracle calls to the OpenMP timing build (or back to the plain build) and return the
    thread count in use.  Only the benchmark's CPU-baseline leg uses the timing build; every check uses
    the plain build, whose summation order is fixed."""
    global _lib, _variant
    if enable != _variant:
        _lib, _variant = None, enable
    return int(lib().orc_threads(int(threads)))


def lib():
    global _lib
    if _lib is None:
        path = _LIB_OMP if _variant else _LIB
        if not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(_SRC):
            build(_variant)
        L = ctypes.CDLL(path)
        P = ctypes.c_void_p
        i64 = ctypes.c_int64
        d = ctypes.c_double
        i = ctypes.c_int
        L.orc_topology.argtypes = [i, i64, i64, P, i64, P, P, P, P]
        L.orc_build.argtypes = [i, i64, P, i64, P, P, d, d, d, i, P, P, P, P]
        L.orc_forces.argtypes = [i, i64, P, i64, P, P, P, P, P, P, P]
        L.orc_hessian.argtypes = [i, i64, i64, P, P, P, P, P, P, P]
        L.orc_mass.argtypes = [i64, P, i64, P, d, d, P]
        L.orc_apply.argtypes = [i64, P, P, P, P, d, P, P]
        L.orc_step.argtypes = [i, i64, i64, P, P, P, P, P, P, P, P, P, P, P, P, d, P, i, d, d, i, P, P, P]
        L.orc_static.argtypes = [i, i64, i64, P, P, P, P, P, P, P, P, P, P, P, d, d, i, d, i, P, P, P]
        L.orc_membrane.argtypes = [i64, P, i64, P, P, d, d, d, P, P]
        L.orc_membrane_rest_hessian.argtypes = [i64, P, P, d, d, d, P]
        L.orc_membrane_gn_hessian.argtypes = [i64, P, P, P, d, d, d, P]
        L.orc_membrane_tangent.argtypes = [i64, P, P, P, d, d, d, P]
        L.orc_static_membrane.argtypes = [i, i64, i64, P, P, P, P, P, P, P, P, i64, P, P, d, d, d, P, P, P, d, d, i,
                                          d, i, P, P, P]
        L.orc_step_membrane.argtypes = [i, i64, i64, P, P, P, P, P, P, P, P, i64, P, P, d, d, d, P, P, P, P, d, P,
                                        i, d, d, i, P, P, P, P, P]
        L.orc_edge_normal_literal.argtypes = [P, P, P, P, P]
        L.orc_threads.argtypes = [i]
        _lib = L
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def held_mask(pinned, held=None):
    """The solvers' per-vertex mask of held coordinates: every coordinate of a vertex whose `pinned`
    entry is nonzero, plus the coordinates that `held` names (bit d holds coordinate d of the vertex)."""
    m = np.where(np.asarray(pinned) != 0, 7, 0).astype(np.uint8)
    if held is not None:
        m |= np.asarray(held, dtype=np.uint8) & 7
    return np.ascontiguousarray(m)


def _check(rc, what):
    if rc != 0:
        raise OracleError(rc, what)


def model_id(model) -> int:
    return MODELS.index(model) if isinstance(model, str) else int(model)


def stencil_size(model) -> int:
    return 4 if model_id(model) < 2 else 6


def curv_size(model) -> int:
    return 1 if model_id(model) < 2 else 3


class Stencils:
    """Rest-precomputed stencils of one mesh for one model.  world_frame (edge models): the quadratic
    thin plate/shell operator of App. D (eq 79) instead of the projected one.  clamped: [n][2] vertex
    pairs of boundary edges with the clamped condition (eqs 30-31, 59); other boundary edges are free."""

    def __init__(self, model, X, tris, young, poisson, thickness, world_frame=False, clamped=None):
        self.model = model_id(model)
        self.X = np.ascontiguousarray(X, dtype=np.float64)
        self.tris = np.ascontiguousarray(tris, dtype=np.int32)
        self.nv = self.X.shape[0]
        self.nt = self.tris.shape[0]
        self.k = stencil_size(self.model)
        self.r = curv_size(self.model)
        cl = np.zeros((0, 2), dtype=np.int32) if clamped is None else \
            np.ascontiguousarray(clamped, dtype=np.int32).reshape(-1, 2)
        self.clamped = cl
        ns = ctypes.c_int64(0)
        _check(lib().orc_topology(self.model, self.nv, self.nt, _p(self.tris), cl.shape[0], _p(cl),
                                  ctypes.byref(ns), None, None), "topology")
        self.ns = ns.value
        self.idx = np.zeros((self.ns, self.k), dtype=np.int32)
        self.bc = np.zeros(self.ns, dtype=np.uint8)
        _check(lib().orc_topology(self.model, self.nv, self.nt, _p(self.tris), cl.shape[0], _p(cl),
                                  ctypes.byref(ns), _p(self.idx), _p(self.bc)), "topology")
        self.B = np.zeros((self.ns, self.r, self.k))
        self.kappa0 = np.zeros((self.ns, self.r))
        self.D = np.zeros((self.ns, self.r, self.r))
        self.Crest = np.zeros((self.ns, self.r, 3))
        self.world_frame = bool(world_frame)
        self.young, self.poisson, self.thickness = float(young), float(poisson), float(thickness)
        _check(lib().orc_build(self.model, self.nv, _p(self.X), self.ns, _p(self.idx), _p(self.bc), young, poisson,
                               thickness, WORLD_FRAME if world_frame else 0, _p(self.B), _p(self.kappa0),
                               _p(self.D), _p(self.Crest)), "build")

    def forces(self, x):
        x = np.ascontiguousarray(x, dtype=np.float64)
        f = np.zeros((self.nv, 3))
        e = ctypes.c_double(0.0)
        _check(lib().orc_forces(self.model, self.nv, _p(x), self.ns, _p(self.idx), _p(self.B), _p(self.kappa0),
                                _p(self.Crest), _p(self.D), _p(f), ctypes.byref(e)), "forces")
        return f, e.value

    def energy(self, x):
        return self.forces(x)[1]

    def hessian(self):
        """Scalar CSR (rowptr int64, col int32, val float64) of K_s."""
        nnz = ctypes.c_int64(0)
        rowptr = np.zeros(self.nv + 1, dtype=np.int64)
        _check(lib().orc_hessian(self.model, self.nv, self.ns, _p(self.idx), _p(self.B), _p(self.D),
                                 ctypes.byref(nnz), _p(rowptr), None, None), "hessian")
        col = np.zeros(nnz.value, dtype=np.int32)
        val = np.zeros(nnz.value)
        _check(lib().orc_hessian(self.model, self.nv, self.ns, _p(self.idx), _p(self.B), _p(self.D),
                                 ctypes.byref(nnz), _p(rowptr), _p(col), _p(val)), "hessian")
        return rowptr, col, val


def hessian_dense(st: Stencils) -> np.ndarray:
    rowptr, col, val = st.hessian()
    K = np.zeros((st.nv, st.nv))
    for i in range(st.nv):
        K[i, col[rowptr[i]:rowptr[i + 1]]] = val[rowptr[i]:rowptr[i + 1]]
    return K


def mass(X, tris, density, thickness):
    X = np.ascontiguousarray(X, dtype=np.float64)
    tris = np.ascontiguousarray(tris, dtype=np.int32)
    m = np.zeros(X.shape[0])
    _check(lib().orc_mass(X.shape[0], _p(X), tris.shape[0], _p(tris), density, thickness, _p(m)), "mass")
    return m


def apply(csr, mass_v, dt2, p):
    rowptr, col, val = csr
    p = np.ascontiguousarray(p, dtype=np.float64)
    q = np.zeros_like(p)
    _check(lib().orc_apply(p.shape[0], _p(rowptr), _p(col), _p(val), _p(mass_v), dt2, _p(p), _p(q)), "apply")
    return q


def membrane_forces(st: Stencils, x):
    """Membrane force and energy (Sec. 3, eq 1; constant strain triangles, Saint Venant-Kirchhoff)."""
    x = np.ascontiguousarray(x, dtype=np.float64)
    f = np.zeros((st.nv, 3))
    e = ctypes.c_double(0.0)
    _check(lib().orc_membrane(st.nv, _p(x), st.nt, _p(st.tris), _p(st.X), st.young, st.poisson, st.thickness,
                              _p(f), ctypes.byref(e)), "membrane")
    return f, e.value


def membrane_rest_hessian(st: Stencils):
    """Per-triangle membrane Hessian at rest, [nt][9][9] (vertex-major, coordinate-minor)."""
    K9 = np.zeros((st.nt, 9, 9))
    _check(lib().orc_membrane_rest_hessian(st.nt, _p(st.tris), _p(st.X), st.young, st.poisson, st.thickness,
                                           _p(K9)), "membrane hessian")
    return K9


def membrane_gn_hessian(st: Stencils, x):
    """Per-triangle Gauss-Newton membrane tangent at x, [nt][9][9]."""
    x = np.ascontiguousarray(x, dtype=np.float64)
    K9 = np.zeros((st.nt, 9, 9))
    _check(lib().orc_membrane_gn_hessian(st.nt, _p(st.tris), _p(st.X), _p(x), st.young, st.poisson, st.thickness,
                                         _p(K9)), "membrane gn hessian")
    return K9


def membrane_tangent(st: Stencils, x):
    """Per-triangle membrane tangent of the solvers at x (Gauss-Newton plus the stress part with the
    stress's positive semi-definite part), [nt][9][9]."""
    x = np.ascontiguousarray(x, dtype=np.float64)
    K9 = np.zeros((st.nt, 9, 9))
    _check(lib().orc_membrane_tangent(st.nt, _p(st.tris), _p(st.X), _p(x), st.young, st.poisson, st.thickness,
                                      _p(K9)), "membrane tangent")
    return K9


class MembraneSim:
    """Implicit-Euler state of the shell with its membrane (Sec. 3 and Sec. 5): the membrane tangent, one
    coupled Jacobi-PCG per Newton solve, Armijo backtracking on the incremental potential."""

    def __init__(self, st: Stencils, material: dict, pinned, x0=None, v0=None, held=None):
        self.st = st
        self.csr = st.hessian()
        self.mass = mass(st.X, st.tris, material["density"], material["thickness"])
        self.pinned = held_mask(pinned, held)
        self.x = np.array(st.X if x0 is None else x0, dtype=np.float64, copy=True)
        self.v = np.zeros_like(self.x) if v0 is None else np.array(v0, dtype=np.float64, copy=True)

    def step(self, dt, gravity=(0.0, 0.0, -9.81), max_newton=4, newton_rtol=1e-8, pcg_rtol=1e-10, max_pcg=200000,
             replay_pcg=None, replay_halvings=None):
        """Returns (counts [max_newton], halvings [max_newton], stats dict)."""
        g = np.ascontiguousarray(gravity, dtype=np.float64)
        n = max(max_newton, 1)
        counts = np.zeros(n, dtype=np.int32)
        halv = np.zeros(n, dtype=np.int32)
        stats = np.zeros(4)
        rp = None if replay_pcg is None else np.ascontiguousarray(replay_pcg, dtype=np.int32)
        rh = None if replay_halvings is None else np.ascontiguousarray(replay_halvings, dtype=np.int32)
        rowptr, col, val = self.csr
        st = self.st
        rc = lib().orc_step_membrane(st.model, st.nv, st.ns, _p(st.idx), _p(st.B), _p(st.kappa0), _p(st.Crest),
                                     _p(st.D), _p(rowptr), _p(col), _p(val), st.nt, _p(st.tris), _p(st.X), st.young,
                                     st.poisson, st.thickness, _p(self.mass), _p(self.pinned), _p(self.x),
                                     _p(self.v), dt, _p(g), max_newton, newton_rtol, pcg_rtol, max_pcg, _p(rp),
                                     _p(rh), _p(counts), _p(halv), _p(stats))
        if rc not in (0, -5):
            _check(rc, "membrane step")
        return counts, halv, dict(newton_iters=int(stats[0]), pcg_total=int(stats[1]), grad_norm0=stats[2],
                                  grad_norm=stats[3], budget_hit=(rc == -5))


class Sim:
    """Implicit-Euler state advanced by the oracle (Sec. 5, eqs 62-63 without contact)."""

    def __init__(self, st: Stencils, material: dict, pinned, x0=None, v0=None, held=None):
        self.st = st
        self.csr = st.hessian()
        self.mass = mass(st.X, st.tris, material["density"], material["thickness"])
        self.pinned = held_mask(pinned, held)
        self.x = np.array(st.X if x0 is None else x0, dtype=np.float64, copy=True)
        self.v = np.zeros_like(self.x) if v0 is None else np.array(v0, dtype=np.float64, copy=True)

    def step(self, dt, gravity=(0.0, 0.0, -9.81), max_newton=1, newton_rtol=1e-8, pcg_rtol=1e-10,
             max_pcg=200000, replay=None):
        """Advance one step; returns (counts [max_newton,3], stats dict).  replay: counts to re-run."""
        g = np.ascontiguousarray(gravity, dtype=np.float64)
        counts = np.zeros((max(max_newton, 1), 3), dtype=np.int32)
        stats = np.zeros(4)
        rep = None if replay is None else np.ascontiguousarray(replay, dtype=np.int32).reshape(-1, 3)
        if rep is not None and rep.shape[0] < max_newton:
            raise ValueError("replay needs one row per Newton iteration")
        rowptr, col, val = self.csr
        st = self.st
        rc = lib().orc_step(st.model, st.nv, st.ns, _p(st.idx), _p(st.B), _p(st.kappa0), _p(st.Crest), _p(st.D),
                            _p(rowptr), _p(col), _p(val), _p(self.mass), _p(self.pinned), _p(self.x), _p(self.v), dt,
                            _p(g),
                            max_newton, newton_rtol, pcg_rtol, max_pcg, _p(rep), _p(counts), _p(stats))
        if rc not in (0, -5):
            _check(rc, "step")
        return counts, dict(newton_iters=int(stats[0]), pcg_total=int(stats[1]), grad_norm0=stats[2],
                            grad_norm=stats[3], budget_hit=(rc == -5))


def solve_static(st: Stencils, pinned, load=None, x0=None, eps_f=1e-3, eps_u=0.0, max_newton=20, pcg_rtol=1e-10,
                 max_pcg=200000, replay=None, held=None):
    """Quasi-static equilibrium under the applied load (Sec. 5, eq 64); returns (x, counts, stats)."""
    rowptr, col, val = st.hessian()
    x = np.array(st.X if x0 is None else x0, dtype=np.float64, copy=True)
    pin = held_mask(pinned, held)
    F = None if load is None else np.ascontiguousarray(load, dtype=np.float64)
    counts = np.zeros((max(max_newton, 1), 3), dtype=np.int32)
    stats = np.zeros(4)
    rep = None if replay is None else np.ascontiguousarray(replay, dtype=np.int32).reshape(-1, 3)
    if rep is not None and rep.shape[0] < max_newton:
        raise ValueError("replay needs one row per Newton iteration")
    rc = lib().orc_static(st.model, st.nv, st.ns, _p(st.idx), _p(st.B), _p(st.kappa0), _p(st.Crest), _p(st.D),
                          _p(rowptr), _p(col), _p(val), _p(pin), _p(F), _p(x), eps_f, eps_u, max_newton, pcg_rtol,
                          max_pcg, _p(rep), _p(counts), _p(stats))
    if rc not in (0, -5):
        _check(rc, "static")
    return x, counts, dict(newton_iters=int(stats[0]), pcg_total=int(stats[1]), resid0=stats[2], resid=stats[3],
                           budget_hit=(rc == -5))


def solve_static_membrane(st: Stencils, pinned, load=None, x0=None, eps_f=1e-3, eps_u=0.1, max_newton=200,
                          pcg_rtol=1e-10, max_pcg=200000, replay=None, held=None):
    """Quasi-static equilibrium of the shell with its membrane (eq 64); returns (x, counts, stats)."""
    rowptr, col, val = st.hessian()
    x = np.array(st.X if x0 is None else x0, dtype=np.float64, copy=True)
    pin = held_mask(pinned, held)
    F = None if load is None else np.ascontiguousarray(load, dtype=np.float64)
    counts = np.zeros(max(max_newton, 1), dtype=np.int32)
    stats = np.zeros(4)
    rep = None if replay is None else np.ascontiguousarray(replay, dtype=np.int32)
    rc = lib().orc_static_membrane(st.model, st.nv, st.ns, _p(st.idx), _p(st.B), _p(st.kappa0), _p(st.Crest),
                                   _p(st.D), _p(rowptr), _p(col), _p(val), st.nt, _p(st.tris), _p(st.X), st.young,
                                   st.poisson, st.thickness, _p(pin), _p(F), _p(x), eps_f, eps_u, max_newton,
                                   pcg_rtol, max_pcg, _p(rep), _p(counts), _p(stats))
    if rc not in (0, -5):
        _check(rc, "static membrane")
    return x, counts, dict(newton_iters=int(stats[0]), pcg_total=int(stats[1]), resid0=stats[2], resid=stats[3],
                           budget_hit=(rc == -5))


def edge_normal_literal(x1, x2, x3, x4):
    a = [np.ascontiguousarray(v, dtype=np.float64) for v in (x1, x2, x3, x4)]
    n = np.zeros(3)
    _check(lib().orc_edge_normal_literal(*[_p(v) for v in a], _p(n)), "edge normal")
    return n
