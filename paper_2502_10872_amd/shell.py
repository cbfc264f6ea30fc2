"""Thin ctypes binding of the HIP library (include/shell.h); argument marshalling only.

Every entry point keeps the C name.  Device arrays are torch tensors on a HIP device (torch is used
for device memory and streams only); host arrays are numpy.  A non-OK status raises ShellError.  The
library must be built (`python -m paper_2502_10872_amd.build`); there is no fallback path.
"""

from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIBRARY = os.path.join(_HERE, "libshell_hip.so")

SHELL_OK, SHELL_E_BUDGET, SHELL_E_NONFINITE = 0, 6, 5
SHELL_E_INVALID_ARG, SHELL_E_UNSUPPORTED = 1, 9
SHELL_PREC_FP64, SHELL_PREC_MIXED = 0, 1
SHELL_PCG_TOLERANCE, SHELL_PCG_REPLAY = 0, 1
SHELL_MAX_NEWTON = 256
MODELS = ("EP", "ES", "FP", "FS", "SP", "SS")
STATUS = {0: "SHELL_OK", 1: "SHELL_E_INVALID_ARG", 2: "SHELL_E_NONMANIFOLD", 3: "SHELL_E_ORIENTATION",
          4: "SHELL_E_DEGENERATE", 5: "SHELL_E_NONFINITE", 6: "SHELL_E_BUDGET", 7: "SHELL_E_OOM", 8: "SHELL_E_HIP",
          9: "SHELL_E_UNSUPPORTED"}


class ShellError(RuntimeError):
    def __init__(self, status: int, where: str, detail: str):
        super().__init__(f"{where}: {STATUS.get(status, status)}: {detail}")
        self.status = status


class shell_material_t(ctypes.Structure):
    _fields_ = [("young", ctypes.c_double), ("poisson", ctypes.c_double), ("thickness", ctypes.c_double),
                ("density", ctypes.c_double)]


class shell_config_t(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int32), ("block_vertices", ctypes.c_int32), ("reorder", ctypes.c_int32),
                ("flags", ctypes.c_int32)]


SHELL_FLAG_DIRECT_PRODUCT = 1
SHELL_FLAG_WORLD_FRAME = 2  # edge models: the quadratic thin plate/shell operator (App. D, eq 79)
SHELL_FLAG_MEMBRANE = 4  # adds the membrane of Sec. 3 (eq 1): forces (both precisions), step and static solve (FP64)


class shell_stencils_info_t(ctypes.Structure):
    _fields_ = [("nv", ctypes.c_int64), ("nt", ctypes.c_int64), ("ns", ctypes.c_int64),
                ("ns_tiled", ctypes.c_int64), ("nblocks", ctypes.c_int64), ("model", ctypes.c_int32),
                ("k", ctypes.c_int32), ("r", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("block_vertices", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class shell_step_params_t(ctypes.Structure):
    _fields_ = [("dt", ctypes.c_double), ("gravity", ctypes.c_double * 3), ("max_newton", ctypes.c_int32),
                ("max_pcg", ctypes.c_int32), ("newton_rtol", ctypes.c_double), ("pcg_rtol", ctypes.c_double),
                ("mode", ctypes.c_int32), ("chunk", ctypes.c_int32), ("pcg_workgroups", ctypes.c_int32),
                ("flags", ctypes.c_int32), ("replay_counts", ctypes.c_void_p)]


SHELL_STEP_NO_GRAPHS = 1


class shell_static_params_t(ctypes.Structure):
    _fields_ = [("load", ctypes.c_void_p), ("eps_f", ctypes.c_double), ("eps_u", ctypes.c_double),
                ("max_newton", ctypes.c_int32), ("max_pcg", ctypes.c_int32), ("pcg_rtol", ctypes.c_double),
                ("mode", ctypes.c_int32), ("chunk", ctypes.c_int32), ("pcg_workgroups", ctypes.c_int32),
                ("flags", ctypes.c_int32), ("replay_counts", ctypes.c_void_p)]


class shell_step_stats_t(ctypes.Structure):
    _fields_ = [("newton_iters", ctypes.c_int32), ("pcg_total", ctypes.c_int32), ("status", ctypes.c_int32),
                ("newton_capped", ctypes.c_int32), ("grad_norm0", ctypes.c_double), ("grad_norm", ctypes.c_double),
                ("counts", (ctypes.c_int32 * 3) * SHELL_MAX_NEWTON)]


class shell_kernel_times_t(ctypes.Structure):
    _fields_ = [("force_ms", ctypes.c_double), ("spmv_ms", ctypes.c_double), ("update_ms", ctypes.c_double),
                ("direction_ms", ctypes.c_double), ("reps", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class shell_hessian_info_t(ctypes.Structure):
    _fields_ = [("nv", ctypes.c_int64), ("nnz", ctypes.c_int64), ("slots", ctypes.c_int64),
                ("nslices", ctypes.c_int64), ("group_cols", ctypes.c_int64), ("max_group_cols", ctypes.c_int32),
                ("staged", ctypes.c_int32)]


SHELL_NUM_PHASES = 3
PHASES = ("forces", "product", "update")  # SHELL_PHASE_* order


class shell_profile_t(ctypes.Structure):
    _fields_ = [("ms", ctypes.c_double * SHELL_NUM_PHASES), ("count", ctypes.c_int64 * SHELL_NUM_PHASES)]


EXPORTS = ("shell_build_stencils", "shell_stencils_info", "shell_stencils_export", "shell_eval_forces",
           "shell_assemble_constant_hessian", "shell_hessian_export_csr", "shell_hessian_info",
           "shell_hessian_apply", "shell_sim_create",
           "shell_step_implicit", "shell_solve_static", "shell_sim_get_stats", "shell_sim_get_state", "shell_sim_set_state",
           "shell_sim_set_held",
           "shell_sim_device_state", "shell_sim_time_kernels", "shell_batch_create", "shell_batch_step",
           "shell_batch_reset", "shell_sim_device_bytes", "shell_batch_profile", "shell_batch_profile_read",
           "shell_sim_profile", "shell_sim_profile_read",
           "shell_destroy_stencils", "shell_destroy_hessian", "shell_destroy_sim", "shell_destroy_batch",
           "shell_status_string", "shell_last_error", "shell_eval_forces_noalloc")

_lib = None


def lib() -> ctypes.CDLL:
    """Load libshell_hip.so; raises if it has not been built (there is no other implementation)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIBRARY):
            raise RuntimeError(f"{LIBRARY} is missing: build it with `python -m paper_2502_10872_amd.build`")
        L = ctypes.CDLL(LIBRARY)
        P, i64, i32, d = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_double
        L.shell_build_stencils.argtypes = [P, i64, P, i64, i32, P, P, i64, P, P, P]
        L.shell_stencils_info.argtypes = [P, P]
        L.shell_stencils_export.argtypes = [P, P, P, P]
        L.shell_eval_forces.argtypes = [P, P, P, P, P]
        L.shell_eval_forces_noalloc.argtypes = [P, P, P, P, P]
        L.shell_assemble_constant_hessian.argtypes = [P, P, P]
        L.shell_hessian_export_csr.argtypes = [P, P, P, P, P]
        L.shell_hessian_info.argtypes = [P, P]
        L.shell_hessian_apply.argtypes = [P, P, d, P, P, P]
        L.shell_sim_create.argtypes = [P, P, P, P, P, P]
        L.shell_step_implicit.argtypes = [P, P, P, P]
        L.shell_solve_static.argtypes = [P, P, P, P]
        L.shell_sim_get_stats.argtypes = [P, P]
        L.shell_sim_get_state.argtypes = [P, P, P, P]
        L.shell_sim_set_state.argtypes = [P, P, P, i64]
        L.shell_sim_set_held.argtypes = [P, P]
        L.shell_sim_device_state.argtypes = [P, P, P]
        L.shell_sim_time_kernels.argtypes = [P, d, i32, P, P]
        L.shell_batch_create.argtypes = [P, i32, P]
        L.shell_batch_step.argtypes = [P, P, i32, P, P]
        L.shell_batch_reset.argtypes = [P, P, i32]
        L.shell_sim_device_bytes.argtypes = [P, P, P, P]
        L.shell_batch_profile.argtypes = [P, i32]
        L.shell_batch_profile_read.argtypes = [P, P]
        L.shell_sim_profile.argtypes = [P, i32]
        L.shell_sim_profile_read.argtypes = [P, P]
        for name in ("shell_destroy_stencils", "shell_destroy_hessian", "shell_destroy_sim", "shell_destroy_batch"):
            getattr(L, name).argtypes = [P]
            getattr(L, name).restype = None
        L.shell_status_string.argtypes = [ctypes.c_int]
        L.shell_status_string.restype = ctypes.c_char_p
        L.shell_last_error.argtypes = []
        L.shell_last_error.restype = ctypes.c_char_p
        for name in EXPORTS:
            if name not in ("shell_status_string", "shell_last_error") and not name.startswith("shell_destroy"):
                getattr(L, name).restype = ctypes.c_int
        _lib = L
    return _lib


def _check(rc: int, where: str, allow=(SHELL_OK,)):
    if rc not in allow:
        raise ShellError(rc, where, lib().shell_last_error().decode())
    return rc


def _np_ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _dev_ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(stream):
    if stream is None:
        import torch

        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, int):
        return ctypes.c_void_p(stream)
    return ctypes.c_void_p(stream.cuda_stream)


def _model(m) -> int:
    return MODELS.index(m) if isinstance(m, str) else int(m)


# ------------------------------------------------------------------------------------ entry points


def shell_build_stencils(X, tris, model, material: dict, precision=SHELL_PREC_FP64, block_vertices=0, reorder=1,
                         stream=None, flags=0, clamped_edges=None):
    X = np.ascontiguousarray(X, dtype=np.float64)
    tris = np.ascontiguousarray(tris, dtype=np.int32)
    mat = shell_material_t(material["young"], material["poisson"], material["thickness"],
                           material.get("density", 0.0))
    cfg = shell_config_t(int(precision), int(block_vertices), int(reorder), int(flags))
    ce = None if clamped_edges is None else np.ascontiguousarray(clamped_edges, dtype=np.int32).reshape(-1, 2)
    out = ctypes.c_void_p()
    _check(lib().shell_build_stencils(_np_ptr(X), X.shape[0], _np_ptr(tris), tris.shape[0], _model(model),
                                      ctypes.byref(mat), None if ce is None else _np_ptr(ce),
                                      0 if ce is None else ce.shape[0], ctypes.byref(cfg), _stream(stream),
                                      ctypes.byref(out)),
           "shell_build_stencils")
    return out.value


def shell_stencils_info(st) -> dict:
    info = shell_stencils_info_t()
    _check(lib().shell_stencils_info(st, ctypes.byref(info)), "shell_stencils_info")
    return {name: getattr(info, name) for name, _ in shell_stencils_info_t._fields_ if name != "reserved"}


def shell_stencils_export(st):
    info = shell_stencils_info(st)
    ns, k, r = info["ns"], info["k"], info["r"]
    idx = np.zeros((ns, k), np.int32)
    B = np.zeros((ns, r, k))
    k0 = np.zeros((ns, r))
    _check(lib().shell_stencils_export(st, _np_ptr(idx), _np_ptr(B), _np_ptr(k0)), "shell_stencils_export")
    return idx, B, k0


def shell_eval_forces(st, x, f, energy=None, stream=None):
    _check(lib().shell_eval_forces(st, _dev_ptr(x), _dev_ptr(f), _dev_ptr(energy), _stream(stream)),
           "shell_eval_forces")


def shell_eval_forces_noalloc(st, x, f, energy=None, stream=None):
    """shell_eval_forces with its scratch in the library's fixed device array (allocates nothing)."""
    _check(lib().shell_eval_forces_noalloc(st, _dev_ptr(x), _dev_ptr(f), _dev_ptr(energy), _stream(stream)),
           "shell_eval_forces_noalloc")


def shell_assemble_constant_hessian(st, stream=None):
    out = ctypes.c_void_p()
    _check(lib().shell_assemble_constant_hessian(st, _stream(stream), ctypes.byref(out)),
           "shell_assemble_constant_hessian")
    return out.value


def shell_hessian_export_csr(h, nv: int):
    nnz = ctypes.c_int64(0)
    _check(lib().shell_hessian_export_csr(h, ctypes.byref(nnz), None, None, None), "shell_hessian_export_csr")
    rowptr = np.zeros(nv + 1, np.int64)
    col = np.zeros(nnz.value, np.int32)
    val = np.zeros(nnz.value)
    _check(lib().shell_hessian_export_csr(h, ctypes.byref(nnz), _np_ptr(rowptr), _np_ptr(col), _np_ptr(val)),
           "shell_hessian_export_csr")
    return rowptr, col, val


def shell_hessian_apply(h, mass, dt2, p, q, stream=None):
    _check(lib().shell_hessian_apply(h, _dev_ptr(mass), float(dt2), _dev_ptr(p), _dev_ptr(q), _stream(stream)),
           "shell_hessian_apply")


def shell_sim_create(st, h, x0, v0=None, pinned=None):
    x0 = np.ascontiguousarray(x0, dtype=np.float64)
    v0 = None if v0 is None else np.ascontiguousarray(v0, dtype=np.float64)
    pinned = None if pinned is None else np.ascontiguousarray(pinned, dtype=np.uint8)
    out = ctypes.c_void_p()
    _check(lib().shell_sim_create(st, h, _np_ptr(x0), _np_ptr(v0), _np_ptr(pinned), ctypes.byref(out)),
           "shell_sim_create")
    return out.value


def step_params(dt, gravity=(0.0, 0.0, -9.81), max_newton=1, max_pcg=200000, newton_rtol=1e-8, pcg_rtol=1e-10,
                replay=None, chunk=0, pcg_workgroups=0, flags=0):
    p = shell_step_params_t()
    p.dt = dt
    p.gravity[:] = list(gravity)
    p.max_newton = max_newton
    p.max_pcg = max_pcg
    p.newton_rtol = newton_rtol
    p.pcg_rtol = pcg_rtol
    p.chunk = chunk
    p.pcg_workgroups = pcg_workgroups
    p.flags = flags
    keep = None
    if replay is not None:
        keep = np.ascontiguousarray(replay, dtype=np.int32).reshape(-1, 3)
        if keep.shape[0] < max_newton:
            raise ValueError("replay needs one row of counts per Newton iteration")
        p.mode = SHELL_PCG_REPLAY
        p.replay_counts = keep.ctypes.data
    else:
        p.mode = SHELL_PCG_TOLERANCE
    return p, keep


def stats_dict(s: shell_step_stats_t) -> dict:
    n = max(s.newton_iters, 0)
    counts = np.array([[s.counts[k][d] for d in range(3)] for k in range(n)], np.int32).reshape(n, 3)
    return dict(newton_iters=s.newton_iters, pcg_total=s.pcg_total, status=s.status, grad_norm0=s.grad_norm0,
                grad_norm=s.grad_norm, counts=counts, newton_capped=bool(s.newton_capped))


def shell_step_implicit(sim, params: shell_step_params_t, with_stats=True, stream=None):
    """Returns (status, stats dict or None); SHELL_E_BUDGET is returned, not raised."""
    stats = shell_step_stats_t()
    rc = lib().shell_step_implicit(sim, ctypes.byref(params), ctypes.byref(stats) if with_stats else None,
                                   _stream(stream))
    _check(rc, "shell_step_implicit", allow=(SHELL_OK, SHELL_E_BUDGET))
    return rc, (stats_dict(stats) if with_stats else None)


def shell_solve_static(sim, load=None, eps_f=0.0, eps_u=0.0, max_newton=1, pcg_rtol=1e-10, max_pcg=200000,
                       replay=None, chunk=0, pcg_workgroups=0, flags=0, stream=None):
    """Quasi-static Newton-Raphson from the simulation's current state (eq 64).  load: host [nv][3] applied
    force in caller order, or None.  Returns (status, stats dict); SHELL_E_BUDGET is returned, not raised."""
    p = shell_static_params_t()
    F = None if load is None else np.ascontiguousarray(load, dtype=np.float64)
    p.load = None if F is None else F.ctypes.data
    p.eps_f = eps_f
    p.eps_u = eps_u
    p.max_newton = max_newton
    p.max_pcg = max_pcg
    p.pcg_rtol = pcg_rtol
    p.chunk = chunk
    p.pcg_workgroups = pcg_workgroups
    p.flags = flags
    keep = None
    if replay is not None:
        keep = np.ascontiguousarray(replay, dtype=np.int32).reshape(-1, 3)
        if keep.shape[0] < max_newton:
            raise ValueError("replay needs one row of counts per Newton iteration")
        p.mode = SHELL_PCG_REPLAY
        p.replay_counts = keep.ctypes.data
    else:
        p.mode = SHELL_PCG_TOLERANCE
    stats = shell_step_stats_t()
    rc = lib().shell_solve_static(sim, ctypes.byref(p), ctypes.byref(stats), _stream(stream))
    _check(rc, "shell_solve_static", allow=(SHELL_OK, SHELL_E_BUDGET))
    return rc, stats_dict(stats)


def shell_sim_get_stats(sim) -> dict:
    stats = shell_step_stats_t()
    _check(lib().shell_sim_get_stats(sim, ctypes.byref(stats)), "shell_sim_get_stats")
    return stats_dict(stats)


def shell_sim_get_state(sim, nv: int):
    x = np.zeros((nv, 3))
    v = np.zeros((nv, 3))
    step = ctypes.c_int64(0)
    _check(lib().shell_sim_get_state(sim, _np_ptr(x), _np_ptr(v), ctypes.byref(step)), "shell_sim_get_state")
    return x, v, step.value


def shell_sim_set_state(sim, x, v, step: int):
    """x, v: host [nv][3] in caller order, or None to keep the current one."""
    x = None if x is None else np.ascontiguousarray(x, dtype=np.float64)
    v = None if v is None else np.ascontiguousarray(v, dtype=np.float64)
    _check(lib().shell_sim_set_state(sim, _np_ptr(x), _np_ptr(v), int(step)), "shell_sim_set_state")


def shell_sim_set_held(sim, held):
    """held: host [nv] in caller order, bit c holding coordinate c (7 the vertex), or None (nothing held)."""
    held = None if held is None else np.ascontiguousarray(held, dtype=np.uint8)
    _check(lib().shell_sim_set_held(sim, _np_ptr(held)), "shell_sim_set_held")


def shell_sim_device_state(sim):
    x = ctypes.c_void_p()
    v = ctypes.c_void_p()
    _check(lib().shell_sim_device_state(sim, ctypes.byref(x), ctypes.byref(v)), "shell_sim_device_state")
    return x.value, v.value


def shell_sim_time_kernels(sim, dt, reps=20, stream=None) -> dict:
    out = shell_kernel_times_t()
    _check(lib().shell_sim_time_kernels(sim, float(dt), int(reps), ctypes.byref(out), _stream(stream)),
           "shell_sim_time_kernels")
    return {name: getattr(out, name) for name, _ in shell_kernel_times_t._fields_ if name != "reserved"}


# member count of each live batch handle: the stats buffer of a step must hold one record per member
_batch_members = {}


def shell_batch_create(sims):
    arr = (ctypes.c_void_p * len(sims))(*sims)
    out = ctypes.c_void_p()
    _check(lib().shell_batch_create(arr, len(sims), ctypes.byref(out)), "shell_batch_create")
    _batch_members[out.value] = len(sims)
    return out.value


def shell_batch_step(batch, params, n, with_stats=True, stream=None, allow_nonfinite=False):
    """params: one shell_step_params_t (shared) or a list of n.  Returns (status, [stats dict] or None).
    SHELL_E_BUDGET is returned, not raised; so is SHELL_E_NONFINITE with allow_nonfinite (the per-mesh
    statuses in the stats then say which meshes went non-finite)."""
    if batch in _batch_members and n != _batch_members[batch]:
        raise ValueError(f"shell_batch_step: n = {n}, but the batch has {_batch_members[batch]} members")
    plist = params if isinstance(params, (list, tuple)) else [params]
    parr = (shell_step_params_t * len(plist))(*plist)
    stats = (shell_step_stats_t * n)()
    rc = lib().shell_batch_step(batch, parr, len(plist), stats if with_stats else None, _stream(stream))
    _check(rc, "shell_batch_step",
           allow=(SHELL_OK, SHELL_E_BUDGET, SHELL_E_NONFINITE) if allow_nonfinite else (SHELL_OK, SHELL_E_BUDGET))
    return rc, ([stats_dict(stats[m]) for m in range(n)] if with_stats else None)


def shell_batch_reset(batch, sims):
    arr = (ctypes.c_void_p * len(sims))(*sims)
    _check(lib().shell_batch_reset(batch, arr, len(sims)), "shell_batch_reset")
    _batch_members[batch] = len(sims)


def shell_sim_device_bytes(sim) -> int:
    a, b, c = ctypes.c_int64(0), ctypes.c_int64(0), ctypes.c_int64(0)
    _check(lib().shell_sim_device_bytes(sim, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)),
           "shell_sim_device_bytes")
    return a.value + b.value + c.value


def _profile_dict(out) -> dict:
    return {name: {"ms": out.ms[k], "count": out.count[k],
                   "avg_ms": out.ms[k] / out.count[k] if out.count[k] else None}
            for k, name in enumerate(PHASES)}


def shell_hessian_info(h) -> dict:
    out = shell_hessian_info_t()
    _check(lib().shell_hessian_info(h, ctypes.byref(out)), "shell_hessian_info")
    return {name: getattr(out, name) for name, _ in shell_hessian_info_t._fields_}


def shell_batch_profile(batch, every):
    _check(lib().shell_batch_profile(batch, int(every)), "shell_batch_profile")


def shell_batch_profile_read(batch) -> dict:
    out = shell_profile_t()
    _check(lib().shell_batch_profile_read(batch, ctypes.byref(out)), "shell_batch_profile_read")
    return _profile_dict(out)


def shell_sim_profile(sim, every):
    _check(lib().shell_sim_profile(sim, int(every)), "shell_sim_profile")


def shell_sim_profile_read(sim) -> dict:
    """Per phase: summed sampled duration (ms), number of sampled launches and their average."""
    out = shell_profile_t()
    _check(lib().shell_sim_profile_read(sim, ctypes.byref(out)), "shell_sim_profile_read")
    return _profile_dict(out)


def shell_destroy_batch(batch):
    _batch_members.pop(batch, None)
    lib().shell_destroy_batch(batch)


def shell_destroy_stencils(st):
    lib().shell_destroy_stencils(st)


def shell_destroy_hessian(h):
    lib().shell_destroy_hessian(h)


def shell_destroy_sim(sim):
    lib().shell_destroy_sim(sim)


def shell_status_string(status: int) -> str:
    return lib().shell_status_string(int(status)).decode()


# ------------------------------------------------------------------------------------ convenience


class Problem:
    """One mesh with its stencils, constant Hessian and (optionally) a simulation, freed together."""

    def __init__(self, mesh, material: dict, model=None, precision=SHELL_PREC_FP64, block_vertices=0, reorder=1,
                 sim=True, flags=0, clamped_edges=None, held=None):
        self.mesh = mesh
        self.nv = mesh.nv
        self.model = mesh.model if model is None else model
        self.st = shell_build_stencils(mesh.X, mesh.tris, self.model, material, precision, block_vertices, reorder,
                                       flags=flags, clamped_edges=clamped_edges)
        self.info = shell_stencils_info(self.st)
        self.h = shell_assemble_constant_hessian(self.st)
        self.sim = shell_sim_create(self.st, self.h, mesh.X, None, mesh.pinned) if sim else None
        if self.sim and held is not None:
            # the mesh's pinned vertices hold every coordinate, `held` adds single coordinates
            shell_sim_set_held(self.sim, np.where(np.asarray(mesh.pinned) != 0, 7, 0).astype(np.uint8)
                               | (np.asarray(held, dtype=np.uint8) & 7))

    def close(self):
        if self.sim:
            shell_destroy_sim(self.sim)
            self.sim = None
        if self.h:
            shell_destroy_hessian(self.h)
            self.h = None
        if self.st:
            shell_destroy_stencils(self.st)
            self.st = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
