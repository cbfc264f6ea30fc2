"""GPU parity: the HIP library (through its C ABI) against the FP64 CPU oracle on the same seeded
inputs.  FP64 results must agree to 1e-10 (norm-wise relative); the mixed path to the stated bounds.

Meshes span several force tiles with a ragged last tile (block sizes 64..4096 vertices)."""

import numpy as np
import pytest

import oracle as O
from paper_2502_10872_amd import inputs as I
from paper_2502_10872_amd import shell as S

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

MAT = I.MATERIAL
TOL64 = 1e-10
# Mixed-precision forces against the FP64 oracle.  Float32 operators and curvatures (relative rounding
# 6e-8) in sums that cancel by about an order of magnitude leave some 1e-7 to 1e-6 norm-wise (observed
# 2e-8 to 1.3e-6 over the six models, the membrane, clamped and world-frame forms); per vertex (the
# largest entry error over the largest reference entry) a vertex's own rounding shows up to a few times
# that (observed up to 6.5e-6, ES).
TOL_MIXED_FORCE = 5e-6
TOL_MIXED_FORCE_VERTEX = 2e-5


def dev():
    return torch.device("cuda:0")


def rel(a, b):
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


def relmax(a, b):
    """Largest per-entry error over the largest entry of the reference: an error confined to a few
    vertices (the boundary stencils, one tile's halo) that a norm-wise comparison would dilute."""
    nb = np.abs(b).max()
    return np.abs(a - b).max() / (nb if nb > 0 else 1.0)


def mesh_for(model, n=37, seed=3):
    if model.endswith("P"):
        return I.plate_mesh(n, 1.0, 0.2, seed, model, "clamp_x0")
    return I.cylinder_mesh(n, 0.5, 0.9, 0.8, 0.2, seed, model, "ends")


def oracle_stencils(model, mesh):
    return O.Stencils(model, mesh.X, mesh.tris, MAT["young"], MAT["poisson"], MAT["thickness"])


def gpu_forces(st, x, f32=False):
    xd = torch.tensor(x, device=dev())
    fd = torch.zeros(x.shape, dtype=torch.float32 if f32 else torch.float64, device=dev())
    ed = torch.zeros(1, dtype=torch.float64, device=dev())
    S.shell_eval_forces(st, xd, fd, ed)
    torch.cuda.synchronize()
    return fd.double().cpu().numpy(), ed.item()


@pytest.mark.parametrize("model", I.MODELS)
def test_stencil_operators_match_oracle(model):
    mesh = mesh_for(model, 20)
    ost = oracle_stencils(model, mesh)
    st = S.shell_build_stencils(mesh.X, mesh.tris, model, MAT, block_vertices=64)
    try:
        idx, B, k0 = S.shell_stencils_export(st)
        assert idx.shape == ost.idx.shape
        # the library folds sqrt(stiffness) into the operator: k_b A_E (edge) or A (triangle)
        if model in ("EP", "ES"):
            scale = np.sqrt(ost.D[:, 0, 0])
        else:
            scale = np.sqrt(ost.D[:, 0, 0] / (MAT["young"] * MAT["thickness"] ** 3 / (12 * (1 - MAT["poisson"] ** 2))))
        ref_B = ost.B * scale[:, None, None]
        ref_k = ost.kappa0 * scale[:, None]
        where = {tuple(r): i for i, r in enumerate(ost.idx.tolist())}
        order = np.array([where[tuple(r)] for r in idx.tolist()])
        assert rel(B, ref_B[order]) <= 1e-12
        if model in ("ES", "FS", "SS"):
            assert rel(k0, ref_k[order]) <= 1e-12
        else:
            assert np.abs(k0).max() == 0.0
    finally:
        S.shell_destroy_stencils(st)


@pytest.mark.parametrize("model", I.MODELS)
@pytest.mark.parametrize("block,reorder", [(64, 1), (256, 1), (4096, 1), (256, 0), (256, 2)])
def test_forces_and_energy_match_oracle(model, block, reorder):
    mesh = mesh_for(model)
    ost = oracle_stencils(model, mesh)
    x = mesh.X + 3e-3 * I.rng(11).standard_normal(mesh.X.shape)
    f_ref, e_ref = ost.forces(x)
    st = S.shell_build_stencils(mesh.X, mesh.tris, model, MAT, block_vertices=block, reorder=reorder)
    try:
        info = S.shell_stencils_info(st)
        assert info["ns"] == ost.ns and info["nblocks"] == -(-mesh.nv // block)
        f, e = gpu_forces(st, x)
        assert rel(f, f_ref) <= TOL64 and relmax(f, f_ref) <= TOL64
        assert abs(e - e_ref) <= TOL64 * abs(e_ref)
        # rest state: zero force up to rounding of the operator's scale
        f0, e0 = gpu_forces(st, mesh.X)
        assert np.abs(f0).max() <= 1e-10 * np.abs(f_ref).max()
    finally:
        S.shell_destroy_stencils(st)


@pytest.mark.parametrize("model", I.MODELS)
def test_mixed_precision_forces_within_bound(model):
    mesh = mesh_for(model)
    ost = oracle_stencils(model, mesh)
    x = mesh.X + 3e-3 * I.rng(12).standard_normal(mesh.X.shape)
    f_ref, e_ref = ost.forces(x)
    st = S.shell_build_stencils(mesh.X, mesh.tris, model, MAT, precision=S.SHELL_PREC_MIXED, block_vertices=256)
    try:
        f, e = gpu_forces(st, x, f32=True)
        err, emax = rel(f, f_ref), relmax(f, f_ref)
        print(f"{model} mixed force rel err {err:.2e} norm-wise, {emax:.2e} per vertex")
        assert err <= TOL_MIXED_FORCE and emax <= TOL_MIXED_FORCE_VERTEX
        assert abs(e - e_ref) <= 1e-4 * abs(e_ref)
    finally:
        S.shell_destroy_stencils(st)


@pytest.mark.parametrize("model", I.MODELS)
def test_mixed_forces_of_a_small_smooth_deformation(model):
    """Mixed precision on a 128 x 128 mesh deformed from rest by a smooth field of amplitude side/10^4.
    The net force is a cancelling sum over stencils of forces far larger than it; the float kernels form
    the curvature relative to the rest shape (from the float64 positions), which keeps the error near
    1e-7 to 6e-7 norm-wise and per vertex (observed).  Float position differences gave 2e-2 here."""
    if model.endswith("S"):
        mesh = I.workload_sphere_cap(128, model)
    else:
        mesh = I.plate_mesh(128, 1.0, 0.2, 5, model, "ring")
    X = mesh.X
    side = float(X[:, 0].max() - X[:, 0].min())
    k, a = 2.0 * np.pi / side, 1e-4 * side
    u = np.stack([np.sin(k * X[:, 0]) * np.cos(k * X[:, 1]), np.cos(k * X[:, 0]) * np.sin(k * X[:, 1]),
                  np.sin(k * X[:, 0]) * np.sin(k * X[:, 1])], axis=1)
    x = X + a * u
    f_ref, _ = oracle_stencils(model, mesh).forces(x)
    st = S.shell_build_stencils(mesh.X, mesh.tris, model, MAT, precision=S.SHELL_PREC_MIXED)
    try:
        f, _ = gpu_forces(st, x, f32=True)
        err, emax = rel(f, f_ref), relmax(f, f_ref)
        print(f"{model} mixed force rel err at a smooth deformation of amplitude side/1e4: {err:.2e} norm-wise, "
              f"{emax:.2e} per vertex")
        assert err <= 2e-6 and emax <= 2e-6
    finally:
        S.shell_destroy_stencils(st)


@pytest.mark.parametrize("model", ["ES", "FS", "SS"])
def test_mixed_shell_forces_vanish_at_rest(model):
    """At the rest shape the float shell kernels' bending strain n.C - kappa0 (C = C0 + B u^e with u = 0)
    cancels to the rounding of the float C0 and kappa0: the rest force stays below 1e-3 of the force of a
    smooth deformation of amplitude side/10^4 (observed 3e-5 to 8e-5)."""
    mesh = mesh_for(model)
    X = mesh.X
    side = float(X[:, 0].max() - X[:, 0].min())
    k = 2.0 * np.pi / side
    u = np.stack([np.sin(k * X[:, 0]) * np.cos(k * X[:, 1]), np.cos(k * X[:, 0]) * np.sin(k * X[:, 1]),
                  np.sin(k * X[:, 0]) * np.sin(k * X[:, 1])], axis=1)
    st = S.shell_build_stencils(mesh.X, mesh.tris, model, MAT, precision=S.SHELL_PREC_MIXED, block_vertices=256)
    try:
        f0, e0 = gpu_forces(st, X, f32=True)
        f1, e1 = gpu_forces(st, X + 1e-4 * side * u, f32=True)
        ratio = np.linalg.norm(f0) / np.linalg.norm(f1)
        print(f"{model} mixed rest force / force of a side/1e4 deformation: {ratio:.2e}")
        assert ratio <= 1e-3
        assert abs(e0) <= 1e-4 * abs(e1)
    finally:
        S.shell_destroy_stencils(st)


@pytest.mark.parametrize("model,flags", [(m, 0) for m in I.MODELS] + [("SS", 1), ("EP", 1)])
def test_hessian_and_apply_match_oracle(model, flags):
    """flags = 1: the product without LDS staging (32-bit column ids, direct gathers)."""
    mesh = mesh_for(model, 29)
    ost = oracle_stencils(model, mesh)
    rp, col, val = ost.hessian()
    with S.Problem(mesh, MAT, block_vertices=128, sim=False, flags=flags) as pb:
        assert S.shell_hessian_info(pb.h)["staged"] == (0 if flags else 1)
        grp, gcol, gval = S.shell_hessian_export_csr(pb.h, mesh.nv)
        assert np.array_equal(grp, rp) and np.array_equal(gcol, col)
        assert rel(gval, val) <= 1e-12
        g = I.rng(13)
        p = g.standard_normal((mesh.nv, 3))
        mass = O.mass(mesh.X, mesh.tris, MAT["density"], MAT["thickness"])
        dt2 = (1 / 60) ** 2
        q_ref = O.apply((rp, col, val), mass, dt2, p)
        pd = torch.tensor(p, device=dev())
        qd = torch.zeros_like(pd)
        S.shell_hessian_apply(pb.h, torch.tensor(mass, device=dev()), dt2, pd, qd)
        torch.cuda.synchronize()
        assert rel(qd.cpu().numpy(), q_ref) <= 1e-12
        S.shell_hessian_apply(pb.h, None, 1.0, pd, qd)
        torch.cuda.synchronize()
        assert rel(qd.cpu().numpy(), O.apply((rp, col, val), None, 1.0, p)) <= 1e-12


def _replay_run(mesh, model, steps, dt, max_newton, pcg_rtol, block=256, flags=0, reorder=1, wg=0):
    ost = oracle_stencils(model, mesh)
    osim = O.Sim(ost, MAT, mesh.pinned)
    with S.Problem(mesh, MAT, model=model, block_vertices=block, flags=flags, reorder=reorder) as pb:
        assert S.shell_hessian_info(pb.h)["staged"] == (0 if flags & S.SHELL_FLAG_DIRECT_PRODUCT else 1)
        for _ in range(steps):
            counts, ostats = osim.step(dt, max_newton=max_newton, pcg_rtol=pcg_rtol)
            params, _keep = S.step_params(dt, max_newton=max_newton, pcg_rtol=pcg_rtol, replay=counts,
                                          pcg_workgroups=wg)
            rc, gstats = S.shell_step_implicit(pb.sim, params)
            assert gstats["newton_iters"] == ostats["newton_iters"]
            assert np.array_equal(gstats["counts"], counts[: gstats["newton_iters"]])
        x, v, step = S.shell_sim_get_state(pb.sim, mesh.nv)
        assert step == steps
        return x, v, osim


def test_plate_steps_replay_match_oracle():
    """Clamped 32 x 32 edge-hinge plate, 10 steps of dt = 1/60 at PCG rtol 1e-10."""
    mesh = I.workload_plate32()
    x, v, osim = _replay_run(mesh, "EP", 10, 1 / 60, 1, 1e-10)
    assert rel(x - mesh.X, osim.x - mesh.X) <= TOL64 and relmax(x - mesh.X, osim.x - mesh.X) <= TOL64
    assert rel(v, osim.v) <= TOL64 and relmax(v, osim.v) <= TOL64
    assert abs(x[:, 2].min() - (-0.16517)) < 2e-4


@pytest.mark.parametrize("model", ["ES", "FS", "SS", "FP", "SP"])
def test_shell_steps_replay_match_oracle(model):
    mesh = I.workload_cylinder(24, model) if model.endswith("S") else I.plate_mesh(24, 0.6, 0.2, 4, model)
    x, v, osim = _replay_run(mesh, model, 3, 1 / 30, 3, 1e-8, block=128)
    assert rel(x - mesh.X, osim.x - mesh.X) <= TOL64 and relmax(x - mesh.X, osim.x - mesh.X) <= TOL64
    assert rel(v, osim.v) <= TOL64 and relmax(v, osim.v) <= TOL64


# ------------------------------------------------------------------ quadratic thin plate/shell (App. D)


def _qt_mesh(model, n=25):
    """A curved rest for both edge models (on a flat rest the variant equals EP/ES)."""
    return I.cylinder_mesh(n, 0.5, 0.9, 0.8, 0.2, 9, model, "ends")


@pytest.mark.parametrize("model", ["EP", "ES"])
def test_world_frame_variant_matches_oracle(model):
    """SHELL_FLAG_WORLD_FRAME (QTP/QTS, eq 79) on a cylinder rest: operators, K_s, forces and energy
    against the oracle's world-frame build, FP64, and mixed forces within the mixed bound."""
    mesh = _qt_mesh(model)
    ost = O.Stencils(model, mesh.X, mesh.tris, MAT["young"], MAT["poisson"], MAT["thickness"], world_frame=True)
    plain = oracle_stencils(model, mesh)
    assert np.abs(ost.B - plain.B).max() > 1e-3 * np.abs(plain.B).max()  # the variant differs here
    x = mesh.X + 2e-3 * I.rng(41).standard_normal(mesh.X.shape)
    f_ref, e_ref = ost.forces(x)
    with S.Problem(mesh, MAT, model=model, block_vertices=128, sim=False, flags=S.SHELL_FLAG_WORLD_FRAME) as pb:
        idx, B, k0 = S.shell_stencils_export(pb.st)
        scale = np.sqrt(ost.D[:, 0, 0])
        where = {tuple(r): i for i, r in enumerate(ost.idx.tolist())}
        order = np.array([where[tuple(r)] for r in idx.tolist()])
        assert rel(B, (ost.B * scale[:, None, None])[order]) <= 1e-12
        if model == "ES":
            assert rel(k0, (ost.kappa0 * scale[:, None])[order]) <= 1e-12
        rp, col, val = ost.hessian()
        grp, gcol, gval = S.shell_hessian_export_csr(pb.h, mesh.nv)
        assert np.array_equal(grp, rp) and np.array_equal(gcol, col)
        assert rel(gval, val) <= 1e-12
        f, e = gpu_forces(pb.st, x)
        assert rel(f, f_ref) <= TOL64
        assert abs(e - e_ref) <= TOL64 * abs(e_ref)
    st32 = S.shell_build_stencils(mesh.X, mesh.tris, model, MAT, precision=S.SHELL_PREC_MIXED,
                                  flags=S.SHELL_FLAG_WORLD_FRAME)
    try:
        f32, _ = gpu_forces(st32, x, f32=True)
        err, emax = rel(f32, f_ref), relmax(f32, f_ref)
        print(f"{model} mixed force (world frame or clamped) rel err {err:.2e} norm-wise, {emax:.2e} per vertex")
        assert err <= TOL_MIXED_FORCE and emax <= TOL_MIXED_FORCE_VERTEX
    finally:
        S.shell_destroy_stencils(st32)


def test_world_frame_shell_steps_replay_match_oracle():
    """QTS steps on the cylinder rest: three steps of two Newton solves, counts replayed, against the
    oracle's world-frame simulation."""
    mesh = _qt_mesh("ES", 24)
    ost = O.Stencils("ES", mesh.X, mesh.tris, MAT["young"], MAT["poisson"], MAT["thickness"], world_frame=True)
    osim = O.Sim(ost, MAT, mesh.pinned)
    with S.Problem(mesh, MAT, model="ES", block_vertices=128, flags=S.SHELL_FLAG_WORLD_FRAME) as pb:
        for _ in range(3):
            counts, ostats = osim.step(1 / 30, max_newton=2, pcg_rtol=1e-8)
            params, _keep = S.step_params(1 / 30, max_newton=2, pcg_rtol=1e-8, replay=counts)
            rc, gstats = S.shell_step_implicit(pb.sim, params)
            assert gstats["newton_iters"] == ostats["newton_iters"]
        x, v, _ = S.shell_sim_get_state(pb.sim, mesh.nv)
    assert rel(x - mesh.X, osim.x - mesh.X) <= TOL64
    assert rel(v, osim.v) <= TOL64


def test_world_frame_flag_is_rejected_for_triangle_models():
    mesh = _qt_mesh("SS", 9)
    with pytest.raises(S.ShellError) as ei:
        S.shell_build_stencils(mesh.X, mesh.tris, "SS", MAT, flags=S.SHELL_FLAG_WORLD_FRAME)
    assert ei.value.status == S.SHELL_E_INVALID_ARG


# ------------------------------------------------------------------ clamped boundary operators


def _clamp_mesh(model, n=23):
    """Plates: a flat jittered square; shells: a cylinder patch.  Clamped: the edges on the sides
    x = 0 and y = 0 (so stencils carry clamped and free flaps, and corners both)."""
    mesh = I.plate_mesh(n, 1.0, 0.2, 6, model, "clamp_x0") if model.endswith("P") else \
        I.cylinder_mesh(n, 0.5, 0.9, 0.8, 0.2, 6, model, "ends")
    be = I.boundary_edges(mesh.tris)
    i, j = be % n, be // n
    side = ((i[:, 0] == 0) & (i[:, 1] == 0)) | ((j[:, 0] == 0) & (j[:, 1] == 0))
    return mesh, be[side]


@pytest.mark.parametrize("model", I.MODELS)
def test_clamped_operators_forces_and_hessian_match_oracle(model):
    """Clamped folds (eqs 30-31, 59): operators, rest curvatures, K_s, forces and energy at a deformed
    state against the oracle, FP64 (plates rest-relative through the constant clamp force), and mixed
    forces within the mixed bound."""
    mesh, cl = _clamp_mesh(model)
    ost = O.Stencils(model, mesh.X, mesh.tris, MAT["young"], MAT["poisson"], MAT["thickness"], clamped=cl)
    assert (ost.bc != 0).any() or model == "ES"
    x = mesh.X + 2e-3 * I.rng(44).standard_normal(mesh.X.shape)
    f_ref, e_ref = ost.forces(x)
    with S.Problem(mesh, MAT, model=model, block_vertices=128, sim=False, clamped_edges=cl) as pb:
        idx, B, k0 = S.shell_stencils_export(pb.st)
        assert idx.shape == ost.idx.shape
        kb = MAT["young"] * MAT["thickness"] ** 3 / (12 * (1 - MAT["poisson"] ** 2))
        scale = np.sqrt(ost.D[:, 0, 0] if model in ("EP", "ES") else ost.D[:, 0, 0] / kb)
        where = {tuple(r): i for i, r in enumerate(ost.idx.tolist())}
        order = np.array([where[tuple(r)] for r in idx.tolist()])
        assert rel(B, (ost.B * scale[:, None, None])[order]) <= 1e-12
        if model.endswith("S"):
            assert rel(k0, (ost.kappa0 * scale[:, None])[order]) <= 1e-12
        rp, col, val = ost.hessian()
        grp, gcol, gval = S.shell_hessian_export_csr(pb.h, mesh.nv)
        assert np.array_equal(grp, rp) and np.array_equal(gcol, col)
        assert rel(gval, val) <= 1e-12
        f, e = gpu_forces(pb.st, x)
        assert rel(f, f_ref) <= TOL64
        assert abs(e - e_ref) <= TOL64 * abs(e_ref)
        f0, e0 = gpu_forces(pb.st, mesh.X)  # rest: no force, no energy
        assert np.abs(f0).max() <= 1e-12 * np.abs(f_ref).max() and abs(e0) <= 1e-12 * abs(e_ref)
    st32 = S.shell_build_stencils(mesh.X, mesh.tris, model, MAT, precision=S.SHELL_PREC_MIXED, clamped_edges=cl)
    try:
        f32, _ = gpu_forces(st32, x, f32=True)
        err, emax = rel(f32, f_ref), relmax(f32, f_ref)
        print(f"{model} mixed force (world frame or clamped) rel err {err:.2e} norm-wise, {emax:.2e} per vertex")
        assert err <= TOL_MIXED_FORCE and emax <= TOL_MIXED_FORCE_VERTEX
    finally:
        S.shell_destroy_stencils(st32)


@pytest.mark.parametrize("model", ["EP", "SP", "FS"])
def test_clamped_steps_replay_match_oracle(model):
    """Three steps of the clamped meshes under gravity, counts replayed, against the oracle (the
    plates rest-relative, FS keeping its twist on clamped edges)."""
    mesh, cl = _clamp_mesh(model, 24)
    ost = O.Stencils(model, mesh.X, mesh.tris, MAT["young"], MAT["poisson"], MAT["thickness"], clamped=cl)
    osim = O.Sim(ost, MAT, mesh.pinned)
    with S.Problem(mesh, MAT, model=model, block_vertices=128, clamped_edges=cl) as pb:
        for _ in range(3):
            counts, ostats = osim.step(1 / 30, max_newton=2, pcg_rtol=1e-8)
            params, _keep = S.step_params(1 / 30, max_newton=2, pcg_rtol=1e-8, replay=counts)
            rc, gstats = S.shell_step_implicit(pb.sim, params)
            assert gstats["newton_iters"] == ostats["newton_iters"]
        x, v, _ = S.shell_sim_get_state(pb.sim, mesh.nv)
    assert rel(x - mesh.X, osim.x - mesh.X) <= TOL64
    assert rel(v, osim.v) <= TOL64


# ------------------------------------------------------------------ membrane (Sec. 3, eq 1)


@pytest.mark.parametrize("model", ["SS", "EP", "FS"])
def test_membrane_forces_match_oracle(model):
    """SHELL_FLAG_MEMBRANE: bending plus membrane force and energy at a deformed state against the oracle
    (FP64 to 1e-10, mixed within its bound), on a curved rest for shells and a flat one for the plate."""
    mesh = mesh_for(model, 23) if model != "EP" else I.plate_mesh(23, 1.0, 0.2, 3, "EP", "none")
    ost = oracle_stencils(model, mesh)
    x = mesh.X + 2e-3 * I.rng(71).standard_normal(mesh.X.shape)
    fb, eb = ost.forces(x)
    fm, em = O.membrane_forces(ost, x)
    f_ref, e_ref = fb + fm, eb + em
    assert np.abs(fm).max() > np.abs(fb).max()  # the membrane matters at this state
    st = S.shell_build_stencils(mesh.X, mesh.tris, model, MAT, block_vertices=128, flags=S.SHELL_FLAG_MEMBRANE)
    try:
        f, e = gpu_forces(st, x)
        assert rel(f, f_ref) <= TOL64 and relmax(f, f_ref) <= TOL64
        assert abs(e - e_ref) <= TOL64 * abs(e_ref)
        f0, e0 = gpu_forces(st, mesh.X)
        assert np.abs(f0).max() <= 1e-11 * np.abs(f_ref).max() and abs(e0) <= 1e-12 * abs(e_ref)
    finally:
        S.shell_destroy_stencils(st)
    st32 = S.shell_build_stencils(mesh.X, mesh.tris, model, MAT, precision=S.SHELL_PREC_MIXED,
                                  flags=S.SHELL_FLAG_MEMBRANE)
    try:
        f32, e32 = gpu_forces(st32, x, f32=True)
        err, emax = rel(f32, f_ref), relmax(f32, f_ref)
        print(f"{model} membrane mixed force rel err {err:.2e} norm-wise, {emax:.2e} per vertex")
        assert err <= TOL_MIXED_FORCE and emax <= TOL_MIXED_FORCE_VERTEX
        assert abs(e32 - e_ref) <= 1e-4 * abs(e_ref)
    finally:
        S.shell_destroy_stencils(st32)


@pytest.mark.parametrize("model", ["SS", "FS", "ES"])
def test_membrane_step_replay_matches_oracle(model):
    """The implicit step with the membrane (membrane tangent, coupled PCG, Armijo backtracking) on a
    cylinder patch held at its ends: two steps with the oracle's PCG counts and halvings replayed give the
    oracle's positions and velocities to 1e-10.  The membrane makes the system stiff, so two solvers
    stopped at the same count agree only to about the condition number times the residual they reached
    (at dt = 1/30 and rtol 1e-8 the gap is 4e-7, at rtol 1e-13 it is 3e-10): here the solves run to
    rtol 1e-13 at dt = 1/120."""
    mesh = I.cylinder_mesh(17, 0.5, 0.9, 0.8, 0.2, 3, model, "ends")
    ost = oracle_stencils(model, mesh)
    osim = O.MembraneSim(ost, MAT, mesh.pinned)
    with S.Problem(mesh, MAT, model=model, block_vertices=128, flags=S.SHELL_FLAG_MEMBRANE) as pb:
        for _ in range(2):
            counts, halv, ostats = osim.step(1 / 120, max_newton=3, newton_rtol=1e-6, pcg_rtol=1e-13)
            n = ostats["newton_iters"]
            rep = np.zeros((max(n, 1), 3), np.int32)
            rep[:n, 0] = counts[:n]
            rep[:n, 1] = halv[:n]
            params, _keep = S.step_params(1 / 120, max_newton=n, newton_rtol=1e-6, pcg_rtol=1e-13, replay=rep)
            rc, gs = S.shell_step_implicit(pb.sim, params)
            assert gs["newton_iters"] == n
            assert [list(c[:2]) for c in gs["counts"][:n]] == [[int(a), int(b)] for a, b in zip(counts[:n], halv[:n])]
        x, v, step = S.shell_sim_get_state(pb.sim, mesh.nv)
    assert step == 2
    err = (rel(x - mesh.X, osim.x - mesh.X), rel(v, osim.v), relmax(x - mesh.X, osim.x - mesh.X), relmax(v, osim.v))
    print(f"{model} membrane replay: norm-wise {err[0]:.2e} {err[1]:.2e}, per vertex {err[2]:.2e} {err[3]:.2e}")
    assert max(err) <= TOL64, err


@pytest.mark.parametrize("n", [7, 11, 15])
def test_membrane_step_small_meshes_match_oracle(n):
    """Small meshes take the one-work-group PCG (up to 512 vertices): 7 x 7, 11 x 11 and 15 x 15 cylinder
    patches (49, 121 and 225 vertices) give it 16, 8 and 4 lanes per row.  Two steps replaying the
    oracle's counts and halvings reach the oracle's positions and velocities to 1e-10."""
    mesh = I.cylinder_mesh(n, 0.5, 0.9, 0.8, 0.2, 3, "SS", "ends")
    osim = O.MembraneSim(oracle_stencils("SS", mesh), MAT, mesh.pinned)
    with S.Problem(mesh, MAT, model="SS", block_vertices=128, flags=S.SHELL_FLAG_MEMBRANE) as pb:
        for _ in range(2):
            counts, halv, ostats = osim.step(1 / 120, max_newton=3, newton_rtol=1e-6, pcg_rtol=1e-13)
            k = ostats["newton_iters"]
            rep = np.zeros((max(k, 1), 3), np.int32)
            rep[:k, 0] = counts[:k]
            rep[:k, 1] = halv[:k]
            params, _keep = S.step_params(1 / 120, max_newton=k, newton_rtol=1e-6, pcg_rtol=1e-13, replay=rep)
            rc, gs = S.shell_step_implicit(pb.sim, params)
            assert gs["newton_iters"] == k
        x, v, _ = S.shell_sim_get_state(pb.sim, mesh.nv)
    err = (rel(x - mesh.X, osim.x - mesh.X), rel(v, osim.v))
    assert err[0] <= TOL64 and err[1] <= TOL64, err


def test_membrane_pcg_graphs_match_direct_launches():
    """The membrane's PCG chunks replayed from captured graphs run the same kernels as launching them one by
    one (SHELL_STEP_NO_GRAPHS).  The direct launches replay the graph run's counts and halvings and must
    give its positions and velocities to 1e-10, over several chunks per solve and two steps that reuse the
    captured graphs.  (Every sum of the step has a fixed order, so the two agree to the bit in practice;
    the bound stays at the parity tolerance.)"""
    mesh = I.cylinder_mesh(17, 0.5, 0.9, 0.8, 0.2, 3, "SS", "ends")
    states, reps = [], []
    for flags in (0, S.SHELL_STEP_NO_GRAPHS):
        with S.Problem(mesh, MAT, model="SS", block_vertices=128, flags=S.SHELL_FLAG_MEMBRANE) as pb:
            for k in range(2):
                if flags == 0:
                    params, _keep = S.step_params(1 / 120, max_newton=3, newton_rtol=1e-6, pcg_rtol=1e-13)
                    rc, gs = S.shell_step_implicit(pb.sim, params)
                    n = gs["newton_iters"]
                    rep = np.zeros((max(n, 1), 3), np.int32)
                    rep[:n, :2] = np.asarray(gs["counts"][:n])[:, :2]
                    reps.append((n, rep))
                else:
                    n, rep = reps[k]
                    params, _keep = S.step_params(1 / 120, max_newton=n, newton_rtol=1e-6, pcg_rtol=1e-13,
                                                  replay=rep, flags=flags)
                    rc, gs = S.shell_step_implicit(pb.sim, params)
                    assert gs["newton_iters"] == n
                    assert np.array_equal(np.asarray(gs["counts"][:n])[:, :2], rep[:n, :2])
            x, v, _ = S.shell_sim_get_state(pb.sim, mesh.nv)
            states.append((x, v))
    assert max(int(c) for _, rep in reps for c in rep[:, 0]) > 48  # several chunks per solve
    # the same kernels on the same data in the same order: the same bits
    assert np.array_equal(states[1][0], states[0][0]) and np.array_equal(states[1][1], states[0][1])


def test_membrane_step_tolerance_mode_descends_and_refusals():
    """Tolerance mode: the residual falls within the Newton budget, in both precisions.  A batch does not
    mix simulations with and without the membrane, and sampled timing refuses a membrane batch."""
    mesh = I.cylinder_mesh(17, 0.5, 0.9, 0.8, 0.2, 3, "SS", "ends")
    for prec in (S.SHELL_PREC_FP64, S.SHELL_PREC_MIXED):
        with S.Problem(mesh, MAT, model="SS", precision=prec, block_vertices=128, flags=S.SHELL_FLAG_MEMBRANE) as pb, \
                S.Problem(mesh, MAT, model="SS", precision=prec, block_vertices=128) as plain:
            params, _ = S.step_params(1 / 30, max_newton=6, newton_rtol=1e-6, pcg_rtol=1e-6)
            rc, gs = S.shell_step_implicit(pb.sim, params)
            assert gs["newton_iters"] >= 1 and gs["grad_norm"] < 0.1 * gs["grad_norm0"]
            with pytest.raises(S.ShellError) as ei:
                S.shell_batch_create([pb.sim, plain.sim])
            assert ei.value.status == S.SHELL_E_INVALID_ARG
            batch = S.shell_batch_create([pb.sim])
            try:
                with pytest.raises(S.ShellError) as ei:
                    S.shell_batch_profile(batch, 4)
                assert ei.value.status == S.SHELL_E_UNSUPPORTED
            finally:
                S.shell_destroy_batch(batch)


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_membrane_batch_equals_each_simulation_alone(prec):
    """A batch of simulations with the membrane (models, sizes and per-member parameters differing) steps
    every member exactly as stepping it alone does, bit for bit; the
    first member replays the oracle's counts through the batch and matches the oracle (FP64 bound, or
    the mixed bound).  Resetting the batch to a subset, and to simulations without the membrane, works."""
    precision = S.SHELL_PREC_MIXED if prec == "mixed" else S.SHELL_PREC_FP64
    models = ["SS", "FS", "ES", "SS", "FS", "ES", "SS", "FS", "ES", "SS"]
    meshes = [I.cylinder_mesh(17 + 3 * k, 0.5, 0.9, 0.8, 0.2, 3, mdl, "ends") for k, mdl in enumerate(models)]
    ost = oracle_stencils(models[0], meshes[0])
    osim = O.MembraneSim(ost, MAT, meshes[0].pinned)
    tol_params = [S.step_params(1 / 60, max_newton=3, newton_rtol=1e-8, pcg_rtol=1e-6 * (1 + k))
                  for k in range(len(meshes))]
    flags = S.SHELL_FLAG_MEMBRANE

    def problems():
        return [S.Problem(m, MAT, model=mdl, precision=precision, block_vertices=128, flags=flags)
                for m, mdl in zip(meshes, models)]

    batched, alone = problems(), problems()
    keep = []
    try:
        batch = S.shell_batch_create([pb.sim for pb in batched])
        try:
            for step in range(2):
                counts, halv, ostats = osim.step(1 / 120, max_newton=3, newton_rtol=1e-6, pcg_rtol=1e-13)
                n = ostats["newton_iters"]
                rep = np.zeros((max(n, 1), 3), np.int32)
                rep[:n, 0] = counts[:n]
                rep[:n, 1] = halv[:n]
                p0, k0 = S.step_params(1 / 120, max_newton=n, newton_rtol=1e-6, pcg_rtol=1e-13, replay=rep)
                keep.append(k0)
                plist = [p0] + [tp[0] for tp in tol_params[1:]]
                rc, stats = S.shell_batch_step(batch, plist, len(plist))
                assert stats[0]["newton_iters"] == n
                for k, pb in enumerate(alone):
                    rc1, st1 = S.shell_step_implicit(pb.sim, plist[k])
                    assert st1["pcg_total"] == stats[k]["pcg_total"] and st1["newton_iters"] == stats[k]["newton_iters"]
            for pa, pb in zip(batched, alone):
                xa, va, sa = S.shell_sim_get_state(pa.sim, pa.nv)
                xb, vb, sb = S.shell_sim_get_state(pb.sim, pb.nv)
                assert sa == sb == 2
                assert np.array_equal(xa, xb) and np.array_equal(va, vb)
            x0, v0, _ = S.shell_sim_get_state(batched[0].sim, meshes[0].nv)
            err = (rel(x0 - meshes[0].X, osim.x - meshes[0].X), rel(v0, osim.v))
            bound = TOL64 if prec == "fp64" else 1e-6
            assert err[0] <= bound and err[1] <= bound, err
            # a subset, then simulations without the membrane, through the same batch
            sub = [batched[k].sim for k in (1, 4, 7)]
            S.shell_batch_reset(batch, sub)
            rc, stats = S.shell_batch_step(batch, tol_params[1][0], len(sub))
            assert all(st["newton_iters"] >= 1 for st in stats)
            with S.Problem(meshes[1], MAT, model=models[1], precision=precision, block_vertices=128) as plain:
                S.shell_batch_reset(batch, [plain.sim])
                rc, stats = S.shell_batch_step(batch, tol_params[1][0], 1)
                assert stats[0]["newton_iters"] >= 1
        finally:
            S.shell_destroy_batch(batch)
    finally:
        for pb in batched + alone:
            pb.close()


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_membrane_batch_members_sharing_stencils_step_as_alone(prec):
    """Simulations made from one stencils handle and its Hessian, with different initial velocities,
    stepped together in a batch (their steps in flight at once on their own streams) reach bit for bit
    the states that stepping each alone reaches: nothing a step writes lives in the shared handles.
    Sizes below and above the one-work-group solver's limit."""
    precision = S.SHELL_PREC_MIXED if prec == "mixed" else S.SHELL_PREC_FP64
    params, _keep = S.step_params(1 / 60, max_newton=3, newton_rtol=1e-8, pcg_rtol=1e-6)
    rng = np.random.default_rng(7)
    handles = []  # (destroy, handle), destroyed in reverse
    members, twins, nvs = [], [], []
    try:
        for n, model, count in ((26, "SS", 3), (17, "FS", 2)):
            m = I.cylinder_mesh(n, 0.5, 0.9, 0.8, 0.2, 3, model, "ends")
            st = S.shell_build_stencils(m.X, m.tris, model, MAT, precision, 128, flags=S.SHELL_FLAG_MEMBRANE)
            handles.append((S.shell_destroy_stencils, st))
            h = S.shell_assemble_constant_hessian(st)
            handles.append((S.shell_destroy_hessian, h))
            for k in range(count):
                v0 = 0.05 * (k + 1) * rng.standard_normal((m.nv, 3))
                for out in (members, twins):
                    sim = S.shell_sim_create(st, h, m.X, v0, m.pinned)
                    handles.append((S.shell_destroy_sim, sim))
                    out.append(sim)
                nvs.append(m.nv)
        batch = S.shell_batch_create(members)
        try:
            for _ in range(2):
                rc, stats = S.shell_batch_step(batch, params, len(members))
                for k, t in enumerate(twins):
                    rc1, st1 = S.shell_step_implicit(t, params)
                    assert st1["pcg_total"] == stats[k]["pcg_total"] and st1["newton_iters"] == stats[k]["newton_iters"]
        finally:
            S.shell_destroy_batch(batch)
        for sim, t, nv in zip(members, twins, nvs):
            xa, va, sa = S.shell_sim_get_state(sim, nv)
            xb, vb, sb = S.shell_sim_get_state(t, nv)
            assert sa == sb == 2
            assert np.isfinite(xa).all() and np.array_equal(xa, xb) and np.array_equal(va, vb)
    finally:
        for destroy, hnd in reversed(handles):
            destroy(hnd)


@pytest.mark.parametrize("model", ["SS", "ES"])
def test_mixed_membrane_step_replay_matches_oracle(model):
    """The step with the membrane in mixed precision (float32 forces, float32 K_s and tangent blocks in
    difference form, float64 vectors and Newton loop) against the FP64 oracle, the oracle's PCG counts and
    halvings replayed as in the FP64 test: two steps at dt = 1/120 to 1e-6 relative displacement
    (float32 rounding of the forces and of the matrix entries, 6e-8 relative each, through a
    mass-dominated system)."""
    mesh = I.cylinder_mesh(17, 0.5, 0.9, 0.8, 0.2, 3, model, "ends")
    ost = oracle_stencils(model, mesh)
    osim = O.MembraneSim(ost, MAT, mesh.pinned)
    with S.Problem(mesh, MAT, model=model, precision=S.SHELL_PREC_MIXED, block_vertices=128,
                   flags=S.SHELL_FLAG_MEMBRANE) as pb:
        for _ in range(2):
            counts, halv, ostats = osim.step(1 / 120, max_newton=3, newton_rtol=1e-6, pcg_rtol=1e-13)
            n = ostats["newton_iters"]
            rep = np.zeros((max(n, 1), 3), np.int32)
            rep[:n, 0] = counts[:n]
            rep[:n, 1] = halv[:n]
            params, _keep = S.step_params(1 / 120, max_newton=n, newton_rtol=1e-6, pcg_rtol=1e-13, replay=rep)
            rc, gs = S.shell_step_implicit(pb.sim, params)
            assert gs["newton_iters"] == n
        x, v, step = S.shell_sim_get_state(pb.sim, mesh.nv)
    err = (rel(x - mesh.X, osim.x - mesh.X), rel(v, osim.v))
    print(f"{model} mixed membrane step: displacement {err[0]:.2e}, velocity {err[1]:.2e}")
    assert err[0] <= 1e-6 and err[1] <= 1e-6, err


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_membrane_step_multi_block_matches_oracle(prec):
    """The membrane step's multi-kernel CSR product chain (meshes above the one-work-group solver's 2048
    vertices and below the staged layout's size) over many work-groups with a partial last one (a 48 x 48
    cylinder patch, 2304 vertices): two steps replaying the oracle's counts reach the oracle to the FP64
    bound, or to the mixed bound of the small-mesh test."""
    mesh = I.cylinder_mesh(48, 0.5, 0.9, 0.8, 0.2, 3, "SS", "ends")
    assert mesh.nv == 2304
    ost = oracle_stencils("SS", mesh)
    osim = O.MembraneSim(ost, MAT, mesh.pinned)
    precision = S.SHELL_PREC_MIXED if prec == "mixed" else S.SHELL_PREC_FP64
    with S.Problem(mesh, MAT, model="SS", precision=precision, flags=S.SHELL_FLAG_MEMBRANE) as pb:
        for _ in range(2):
            counts, halv, ostats = osim.step(1 / 120, max_newton=3, newton_rtol=1e-6, pcg_rtol=1e-13)
            n = ostats["newton_iters"]
            rep = np.zeros((max(n, 1), 3), np.int32)
            rep[:n, 0] = counts[:n]
            rep[:n, 1] = halv[:n]
            params, _keep = S.step_params(1 / 120, max_newton=n, newton_rtol=1e-6, pcg_rtol=1e-13, replay=rep)
            rc, gs = S.shell_step_implicit(pb.sim, params)
            assert gs["newton_iters"] == n
        x, v, step = S.shell_sim_get_state(pb.sim, mesh.nv)
    err = (rel(x - mesh.X, osim.x - mesh.X), rel(v, osim.v))
    print(f"{prec} multi-block membrane step: {err[0]:.2e} {err[1]:.2e}")
    bound = TOL64 if prec == "fp64" else 1e-6
    assert err[0] <= bound and err[1] <= bound, err


_STAGED_N = 223  # 49729 vertices: 98 row groups of 512, the last with 65 rows, a last slice of one row
_staged_oracle_cache = {}


def _staged_oracle():
    if not _staged_oracle_cache:
        mesh = I.cylinder_mesh(_STAGED_N, 0.5, 0.9, 0.8, 0.2, 3, "SS", "ends")
        osim = O.MembraneSim(oracle_stencils("SS", mesh), MAT, mesh.pinned)
        osim.step(1 / 60, max_newton=2, newton_rtol=1e-12, pcg_rtol=1e-13, replay_pcg=[150, 150],
                  replay_halvings=[0, 0])
        _staged_oracle_cache["v"] = (mesh, osim.x.copy(), osim.v.copy())
    return _staged_oracle_cache["v"]


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_membrane_step_staged_product_matches_oracle(prec):
    """The staged SELL product (rows in groups, 128 rows at this size, the group's directions in LDS, K_s
    from the bending Hessian's slots, the blocks in SELL-64 component arrays), taken from 32768 vertices up, against the
    CSR product forced by SHELL_FLAG_DIRECT_PRODUCT and against the oracle, on a 49729-vertex cylinder
    patch whose last row group and last slice are partial: one step of two Newton iterations with 150 PCG
    iterations each, replayed on every side.  At a fixed count this far from convergence (the residual
    has fallen by about 1e-3) the iterates carry the sides' rounding differences amplified by the Krylov
    recurrence, so the FP64 bound against the oracle is 1e-9 (measured 1.1e-10 for either layout, against
    the 1e-10 of converged replays); the two layouts differ only in the product's summation order and
    must agree to 1e-12 (measured 7e-14).  Mixed precision: 1e-6 against the oracle, as in the converged
    mixed tests, and 1e-9 between the layouts (the same float32 entries summed in another order in
    float64; measured 6e-11)."""
    mesh, ox, ov = _staged_oracle()
    precision = S.SHELL_PREC_MIXED if prec == "mixed" else S.SHELL_PREC_FP64
    res = {}
    for direct in (False, True):
        flags = S.SHELL_FLAG_MEMBRANE | (S.SHELL_FLAG_DIRECT_PRODUCT if direct else 0)
        with S.Problem(mesh, MAT, model="SS", precision=precision, flags=flags) as pb:
            rep = np.array([[150, 0, 0], [150, 0, 0]], np.int32)
            params, _keep = S.step_params(1 / 60, max_newton=2, newton_rtol=1e-12, pcg_rtol=1e-13, replay=rep)
            rc, gs = S.shell_step_implicit(pb.sim, params)
            assert gs["newton_iters"] == 2 and gs["pcg_total"] == 300
            res[direct] = S.shell_sim_get_state(pb.sim, mesh.nv)[:2]
    errs = {d: (rel(x - mesh.X, ox - mesh.X), rel(v, ov)) for d, (x, v) in res.items()}
    mutual = (rel(res[False][0] - mesh.X, res[True][0] - mesh.X), rel(res[False][1], res[True][1]))
    print(f"{prec} membrane step at {mesh.nv} vertices: staged {errs[False][0]:.2e} {errs[False][1]:.2e}, "
          f"direct {errs[True][0]:.2e} {errs[True][1]:.2e}, staged vs direct {mutual[0]:.2e} {mutual[1]:.2e}")
    bound = 1e-9 if prec == "fp64" else 1e-6
    for d in (False, True):
        assert errs[d][0] <= bound and errs[d][1] <= bound, (d, errs[d])
    mbound = 1e-12 if prec == "fp64" else 1e-9
    assert mutual[0] <= mbound and mutual[1] <= mbound, mutual


@pytest.mark.parametrize("n", [257, 363])
def test_membrane_staged_product_group_sizes_agree_with_the_direct_product(n):
    """The staged product's larger row groups: 256 rows at 66,049 vertices and 512 rows at 131,769 (the
    group size follows the mesh size; the last group holds 1 and 185 rows).  One step of two Newton
    iterations with 150 PCG iterations each, replayed, against the CSR product forced by
    SHELL_FLAG_DIRECT_PRODUCT on the same mesh: the two differ only in the product's summation order
    (bounds as in the 49,729-vertex test: 1e-12 FP64, 1e-9 mixed)."""
    mesh = I.cylinder_mesh(n, 0.5, 0.9, 0.8, 0.2, 3, "SS", "ends")
    for precision, mbound in ((S.SHELL_PREC_FP64, 1e-12), (S.SHELL_PREC_MIXED, 1e-9)):
        res = {}
        for direct in (False, True):
            flags = S.SHELL_FLAG_MEMBRANE | (S.SHELL_FLAG_DIRECT_PRODUCT if direct else 0)
            with S.Problem(mesh, MAT, model="SS", precision=precision, flags=flags) as pb:
                rep = np.array([[150, 0, 0], [150, 0, 0]], np.int32)
                params, _keep = S.step_params(1 / 60, max_newton=2, newton_rtol=1e-12, pcg_rtol=1e-13, replay=rep)
                rc, gs = S.shell_step_implicit(pb.sim, params)
                assert gs["newton_iters"] == 2 and gs["pcg_total"] == 300
                res[direct] = S.shell_sim_get_state(pb.sim, mesh.nv)[:2]
        x, v = res[False]
        assert np.isfinite(x).all() and np.abs(x - mesh.X).max() > 0  # the step moved the mesh
        mutual = (rel(x - mesh.X, res[True][0] - mesh.X), rel(v, res[True][1]))
        print(f"{mesh.nv} vertices, precision {precision}: staged vs direct {mutual[0]:.2e} {mutual[1]:.2e}")
        assert mutual[0] <= mbound and mutual[1] <= mbound, mutual


def test_membrane_step_staged_product_with_held_coordinates_matches_oracle():
    """The staged product's held rows: on the 49729-vertex cylinder patch, besides its pinned ends, every
    7th vertex has z held and every 11th x held (bit c holds coordinate c), so rows mix free and held
    coordinates across the row groups.  One step of two Newton iterations with 40 replayed PCG iterations
    each: the staged and the CSR layouts reach the oracle to 1e-10, agree with each other to 1e-12, and
    leave every held coordinate at its rest value bit for bit.  The count stays at 40: the held points,
    kept at rest while their neighbours fall, stretch the membrane (the first gradient is 23 times that
    of the unconstrained patch), and on that stiffer system unconverged CG iterates lose their agreement
    once orthogonality is lost.  At 150 iterations (1793 are needed to converge) even the two GPU layouts,
    which differ only in the product's summation order, are 5e-7 apart, against 1e-14 at 40."""
    mesh = I.cylinder_mesh(_STAGED_N, 0.5, 0.9, 0.8, 0.2, 3, "SS", "ends")
    held = np.zeros(mesh.nv, np.uint8)
    held[::7] |= 4
    held[::11] |= 1
    osim = O.MembraneSim(oracle_stencils("SS", mesh), MAT, mesh.pinned, held=held)
    osim.step(1 / 60, max_newton=2, newton_rtol=1e-12, pcg_rtol=1e-13, replay_pcg=[40, 40], replay_halvings=[0, 0])
    mask = O.held_mask(mesh.pinned, held)
    res = {}
    for direct in (False, True):
        flags = S.SHELL_FLAG_MEMBRANE | (S.SHELL_FLAG_DIRECT_PRODUCT if direct else 0)
        with S.Problem(mesh, MAT, model="SS", flags=flags, held=held) as pb:
            rep = np.array([[40, 0, 0], [40, 0, 0]], np.int32)
            params, _keep = S.step_params(1 / 60, max_newton=2, newton_rtol=1e-12, pcg_rtol=1e-13, replay=rep)
            rc, gs = S.shell_step_implicit(pb.sim, params)
            assert gs["newton_iters"] == 2 and gs["pcg_total"] == 80
            res[direct] = S.shell_sim_get_state(pb.sim, mesh.nv)[:2]
    for direct, (x, v) in res.items():
        err = (rel(x - mesh.X, osim.x - mesh.X), rel(v, osim.v))
        print(f"held coordinates, {'direct' if direct else 'staged'}: {err[0]:.2e} {err[1]:.2e}")
        assert err[0] <= TOL64 and err[1] <= TOL64, (direct, err)
        for c in range(3):
            rows = (mask >> c) & 1 == 1
            assert np.array_equal(x[rows, c], mesh.X[rows, c]) and not v[rows, c].any()
    assert rel(res[False][0] - mesh.X, res[True][0] - mesh.X) <= 1e-12


def _cantilever(model, scale=1.0, nx=17, ny=3):
    """The Sec. 6 cantilever: a 10 x 1 strip of nx x ny vertices, E = 1.2e6, nu = 0.1, h = 0.1, its two
    left vertex columns held, an end shear of total 4 * scale along Z on the right-end vertices."""
    X = np.zeros((nx * ny, 3))
    for j in range(ny):
        for i in range(nx):
            X[j * nx + i] = (10.0 * i / (nx - 1), 1.0 * j / (ny - 1), 0.0)
    col = np.arange(nx * ny) % nx
    load = np.zeros((nx * ny, 3))
    load[col == nx - 1, 2] = 4.0 * scale / ny
    mesh = I.Mesh("cantilever", X, I.grid_tris(nx, ny), (col <= 1).astype(np.uint8), model, 10.0 / (nx - 1), {})
    return mesh, load, col, dict(young=1.2e6, poisson=0.1, thickness=0.1, density=1.0)


@pytest.mark.parametrize("model", ["FS", "SP"])
def test_static_membrane_cantilever_matches_oracle(model):
    """Quasi-static Newton-Raphson with the membrane on the Sec. 6 cantilever.  With no mass the matrix
    K_s (x) I3 + K_m spans the membrane's in-plane stiffness down to the softest bending mode, and
    finite-precision CG iterates part after a few iterations (against the exact recurrence: 7e-12 after
    one, 9e-5 after five, 0.8 after twenty), so replayed counts prove nothing here: every solve runs to
    rtol 1e-13.  The first solve equals a dense solve of the oracle's system; 12 solves under eps_u = 0.1
    give the oracle's state to 1e-8; a run to eps_f = 1e-3 lands on the oracle's tip deflection."""
    import scipy.sparse as sp
    mesh, load, col, mat = _cantilever(model)
    ost = O.Stencils(model, mesh.X, mesh.tris, mat["young"], mat["poisson"], mat["thickness"])
    nv = mesh.nv
    rp, c, v = ost.hessian()
    K = np.kron(sp.csr_matrix((v, c, rp), shape=(nv, nv)).toarray(), np.eye(3))
    for t, tv in enumerate(ost.tris):
        ii = np.array([3 * tv[j] + d for j in range(3) for d in range(3)])
        K[np.ix_(ii, ii)] += O.membrane_rest_hessian(ost)[t]
    free = np.repeat(mesh.pinned == 0, 3)
    y = np.zeros(3 * nv)
    y[free] = np.linalg.solve(K[np.ix_(free, free)], load.ravel()[free])
    with S.Problem(mesh, mat, model=model, block_vertices=64, flags=S.SHELL_FLAG_MEMBRANE) as pb:
        S.shell_solve_static(pb.sim, load, eps_f=0.0, eps_u=0.0, max_newton=1, pcg_rtol=1e-13)
        x, _, _ = S.shell_sim_get_state(pb.sim, nv)
        assert rel((x - mesh.X).ravel(), y) <= 1e-9
        xo, _, _ = O.solve_static_membrane(ost, mesh.pinned, load, eps_f=0.0, eps_u=0.1, max_newton=12,
                                           pcg_rtol=1e-13)
        S.shell_sim_set_state(pb.sim, mesh.X, None, 0)
        rc, gs = S.shell_solve_static(pb.sim, load, eps_f=0.0, eps_u=0.1, max_newton=12, pcg_rtol=1e-13)
        x, _, _ = S.shell_sim_get_state(pb.sim, nv)
        assert gs["newton_iters"] == 12
        err = rel(x - mesh.X, xo - mesh.X)
        assert err <= 1e-8, err
        xf, _, fst = O.solve_static_membrane(ost, mesh.pinned, load, eps_f=1e-3, eps_u=0.1, max_newton=200,
                                             pcg_rtol=1e-10)
        S.shell_sim_set_state(pb.sim, mesh.X, None, 0)
        rc, gs = S.shell_solve_static(pb.sim, load, eps_f=1e-3, eps_u=0.1, max_newton=200, pcg_rtol=1e-10)
        x, _, _ = S.shell_sim_get_state(pb.sim, nv)
        assert fst["newton_iters"] < 200 and gs["grad_norm"] < 1e-3
        tip, tip_o = x[col == 16][:, 2].mean(), xf[col == 16][:, 2].mean()
        assert abs(tip - tip_o) <= 1e-3 * abs(tip_o), (tip, tip_o)


# ------------------------------------------------------------------ quasi-static Newton-Raphson (eq 64)


def _static_plate(model, n, clamp, q=9.81):
    """Square plate of side 8 (the linear benchmark's), jittered, boundary held, uniform transverse load
    per unit area; clamp: every boundary edge clamped, else simply supported."""
    m = I.plate_mesh(n, 8.0, 0.2, 5, model, "ring")
    cl = I.boundary_edges(m.tris) if clamp else None
    load = np.zeros((m.nv, 3))
    load[:, 2] = -q * O.mass(m.X, m.tris, 1.0, 1.0)
    return m, cl, load


@pytest.mark.parametrize("model,clamp", [("SP", False), ("FP", True), ("EP", True), ("SS", False)])
def test_static_linear_plate_matches_oracle(model, clamp):
    """The linear plate benchmark as one Newton-Raphson solve: replayed PCG counts give the oracle's
    deflection to 1e-10 (the flat-rest shell SS too: its first iterate is the plate's); in tolerance mode
    one solve meets eps_f for the plates, which are linear."""
    m, cl, load = _static_plate(model, 33, clamp)
    mat = dict(MAT, young=2e11, poisson=0.3, thickness=0.01)
    ost = O.Stencils(model, m.X, m.tris, mat["young"], mat["poisson"], mat["thickness"], clamped=cl)
    xo, counts, ostats = O.solve_static(ost, m.pinned, load, eps_f=0.0, max_newton=1, pcg_rtol=1e-12)
    with S.Problem(m, mat, model=model, block_vertices=128, clamped_edges=cl) as pb:
        rc, gs = S.shell_solve_static(pb.sim, load, eps_f=0.0, max_newton=1, replay=counts)
        x, v, step = S.shell_sim_get_state(pb.sim, m.nv)
        assert gs["newton_iters"] == 1 and step == 0 and np.abs(v).max() == 0.0
        assert rel(x - m.X, xo - m.X) <= TOL64
        if model == "SS":
            return
        S.shell_sim_set_state(pb.sim, m.X, None, 0)
        eps_f = 1e-6 * np.linalg.norm(load)
        rc, gs = S.shell_solve_static(pb.sim, load, eps_f=eps_f, max_newton=4, pcg_rtol=1e-12)
        x2, _, _ = S.shell_sim_get_state(pb.sim, m.nv)
        assert rc == S.SHELL_OK and gs["newton_iters"] == 1 and gs["grad_norm"] < eps_f
        assert rel(x2 - m.X, xo - m.X) <= 1e-9


def test_static_increment_limit_and_shell_iterations_match_oracle():
    """eps_u active for three Newton-Raphson iterations, counts replayed: the smoothed plate and the
    smoothed shell on a flat rest (whose iterations carry the geometric terms) against the oracle."""
    for model in ("SP", "SS"):
        m, cl, load = _static_plate(model, 25, False)
        mat = dict(MAT, young=2e11, poisson=0.3, thickness=0.01)
        ost = O.Stencils(model, m.X, m.tris, mat["young"], mat["poisson"], mat["thickness"])
        full, _, _ = O.solve_static(ost, m.pinned, load, eps_f=0.0, max_newton=1, pcg_rtol=1e-12)
        lim = 0.4 * np.abs(full - m.X).max()
        xo, counts, ostats = O.solve_static(ost, m.pinned, load, eps_f=0.0, eps_u=lim, max_newton=3,
                                            pcg_rtol=1e-12)
        if model == "SP":  # linear: steps of 0.4, 0.4 and 0.2 of the solution land on it
            assert np.abs(xo - full).max() <= 1e-9 * lim
        with S.Problem(m, mat, model=model, block_vertices=128) as pb:
            rc, gs = S.shell_solve_static(pb.sim, load, eps_f=0.0, eps_u=lim, max_newton=3, replay=counts)
            x, _, _ = S.shell_sim_get_state(pb.sim, m.nv)
            assert gs["newton_iters"] == 3
            assert rel(x - m.X, xo - m.X) <= TOL64
            assert abs(gs["grad_norm"] - ostats["resid"]) <= 1e-8 * ostats["resid0"]


def test_static_mixed_precision_refines_to_the_oracle():
    """Mixed precision: float PCG solves refined by the float64 residual until eps_f, against the
    oracle's FP64 solution of the clamped FVM plate.  The float force carries a rounding error of order
    1e-7 |B||u| against a curvature of order u / a^2, about 1e-4 relative on this 33 x 33 mesh, which
    bounds what the refinement can reach."""
    m, cl, load = _static_plate("FP", 33, True)
    mat = dict(MAT, young=2e11, poisson=0.3, thickness=0.01)
    ost = O.Stencils("FP", m.X, m.tris, mat["young"], mat["poisson"], mat["thickness"], clamped=cl)
    xo, _, _ = O.solve_static(ost, m.pinned, load, eps_f=0.0, max_newton=1, pcg_rtol=1e-13)
    with S.Problem(m, mat, model="FP", precision=S.SHELL_PREC_MIXED, block_vertices=128, clamped_edges=cl) as pb:
        eps_f = 2e-4 * np.linalg.norm(load)
        rc, gs = S.shell_solve_static(pb.sim, load, eps_f=eps_f, max_newton=12, pcg_rtol=1e-4)
        x, _, _ = S.shell_sim_get_state(pb.sim, m.nv)
        err = rel(x - m.X, xo - m.X)
        assert rc == S.SHELL_OK and gs["grad_norm"] < eps_f and gs["newton_iters"] > 1, (gs, err)
        assert err <= 1e-4, (gs, err)


@pytest.mark.parametrize("model,n,wg", [("SS", 40, 1), ("FS", 36, 1), ("SS", 46, 2), ("EP", 32, 1)])
def test_several_row_groups_per_pcg_workgroup(model, n, wg):
    """Few PCG work-groups, each walking several consecutive row groups (the large-mesh launch shape).
    The plate case is the clamped 32 x 32 plate configuration (dt = 1/60, one Newton solve, which is
    exact for a plate)."""
    if model.endswith("S"):
        mesh = I.workload_cylinder(n, model)
        x, v, osim = _replay_run(mesh, model, 2, 1 / 30, 2, 1e-8, block=128, wg=wg)
    else:
        mesh = I.workload_plate32()
        x, v, osim = _replay_run(mesh, model, 3, 1 / 60, 1, 1e-10, block=128, wg=wg)
    assert rel(x - mesh.X, osim.x - mesh.X) <= TOL64
    assert rel(v, osim.v) <= TOL64


@pytest.mark.parametrize("model,reorder", [("SS", 1), ("EP", 0), ("FS", 2)])
def test_direct_product_replay_matches_oracle(model, reorder):
    """The product without LDS staging (each neighbour gathered from memory) gives the same steps."""
    mesh = I.workload_cylinder(24, model) if model.endswith("S") else I.plate_mesh(24, 0.6, 0.2, 4, model)
    x, v, osim = _replay_run(mesh, model, 2, 1 / 30, 2, 1e-8, block=128, flags=S.SHELL_FLAG_DIRECT_PRODUCT,
                             reorder=reorder)
    assert rel(x - mesh.X, osim.x - mesh.X) <= TOL64
    assert rel(v, osim.v) <= TOL64


@pytest.mark.parametrize("model", ["SS", "EP"])
def test_graph_replays_equal_direct_launches(model):
    """PCG chunks replayed from captured HIP graphs against the same chunks launched kernel by kernel:
    several steps, so each graph is replayed many times with eager work and host synchronisation in
    between; both runs replay the oracle's counts (not powers of two, so graph pieces and direct
    remainders mix) and each must match the oracle."""
    mesh = I.workload_cylinder(28, model) if model.endswith("S") else I.workload_plate32()
    dt, newton = (1 / 30, 2) if model.endswith("S") else (1 / 60, 1)
    ost = oracle_stencils(model, mesh)
    osim = O.Sim(ost, MAT, mesh.pinned)
    runs = []
    with S.Problem(mesh, MAT, model=model, block_vertices=128) as pa, \
            S.Problem(mesh, MAT, model=model, block_vertices=128) as pb:
        for _ in range(4):
            counts, _ = osim.step(dt, max_newton=newton, pcg_rtol=1e-9)
            for pb_, flags in ((pa, 0), (pb, S.SHELL_STEP_NO_GRAPHS)):
                prm, _keep = S.step_params(dt, max_newton=newton, pcg_rtol=1e-9, replay=counts, flags=flags)
                rc, st = S.shell_step_implicit(pb_.sim, prm)
                assert np.array_equal(st["counts"], counts[: st["newton_iters"]])
        for pb_ in (pa, pb):
            x, v, _ = S.shell_sim_get_state(pb_.sim, mesh.nv)
            runs.append((x, v))
    for x, v in runs:
        assert rel(x - mesh.X, osim.x - mesh.X) <= TOL64
        assert rel(v, osim.v) <= TOL64
    # the same kernels on the same data in the same order: the same bits
    assert np.array_equal(runs[0][0], runs[1][0]) and np.array_equal(runs[0][1], runs[1][1])


def test_graphs_in_tolerance_mode_match_direct_launches():
    """Tolerance mode launches chunks of 8, 16, ..., 128 iterations, all from graphs after the first."""
    mesh = I.workload_cylinder(32, "SS")
    out = []
    for flags in (0, S.SHELL_STEP_NO_GRAPHS):
        with S.Problem(mesh, MAT) as pb:
            prm, _ = S.step_params(1 / 30, max_newton=2, pcg_rtol=1e-8, flags=flags)
            tot = 0
            for _ in range(3):
                rc, st = S.shell_step_implicit(pb.sim, prm)
                tot += st["pcg_total"]
            x, v, _ = S.shell_sim_get_state(pb.sim, mesh.nv)
            out.append((x, v, tot))
    (xa, va, ta), (xb, vb, tb) = out
    assert ta == tb
    assert np.array_equal(xa, xb) and np.array_equal(va, vb)


def test_hessian_info_counts():
    """Storage figures against the pattern itself (caller order kept, so slices and groups are known)."""
    mesh = mesh_for("SS", 29)
    rp, col, _ = oracle_stencils("SS", mesh).hessian()
    with S.Problem(mesh, MAT, block_vertices=128, reorder=0, sim=False) as pb:
        hi = S.shell_hessian_info(pb.h)
    assert hi["nv"] == mesh.nv and hi["nnz"] == len(col)
    assert hi["nslices"] == (mesh.nv + 63) // 64
    lens = np.diff(rp)
    # every 64-row slice is padded to its longest row
    assert hi["slots"] == sum(64 * int(lens[a:a + 64].max()) for a in range(0, mesh.nv, 64))
    groups = [np.unique(col[rp[a]:rp[min(a + 512, mesh.nv)]]) for a in range(0, mesh.nv, 512)]
    assert hi["staged"] == 1
    assert hi["group_cols"] == sum(len(g) for g in groups)
    assert hi["max_group_cols"] == max(len(g) for g in groups)


def test_in_step_profiling_changes_nothing():
    """Event sampling inside the steps changes no result (the same kernels in the same order, launched
    directly with events around them: the same bits) and counts its samples."""
    mesh = I.workload_cylinder(24, "SS")
    params, _ = S.step_params(1 / 30, max_newton=2, pcg_rtol=1e-6)
    out = []
    for every in (0, 3):
        with S.Problem(mesh, MAT) as pb:
            S.shell_sim_profile(pb.sim, every)
            for _ in range(2):
                rc, st = S.shell_step_implicit(pb.sim, params)
            prof = S.shell_sim_profile_read(pb.sim)
            x, v, _ = S.shell_sim_get_state(pb.sim, mesh.nv)
            out.append((x, v, st, prof))
    (xa, va, sa, pa), (xb, vb, sb, pb_) = out
    assert np.array_equal(xa, xb) and np.array_equal(va, vb)
    assert all(pa[k]["count"] == 0 for k in pa)
    iters = max(int(sb["counts"][k].max()) for k in range(sb["newton_iters"]))
    # every solve's first product is sampled, then one (update, product) pair in every 3
    assert pb_["product"]["count"] >= 2 and pb_["product"]["count"] >= pb_["update"]["count"]
    assert pb_["forces"]["count"] >= 2 and iters > 0
    for k in pb_:
        assert pb_[k]["ms"] > 0 and pb_[k]["avg_ms"] < 100.0


def test_cylinder_256_fvm_shell_replay_matches_oracle():
    """The FVM shell cylinder at its benchmark size (256 x 256 vertices, jitter 0.2, ends pinned,
    dt = 1/30): three steps of one Newton solve of up to 150 iterations per column, the GPU replaying
    the oracle's counts (observed 2e-12).

    Why not longer: the two implementations differ only in summation order (1e-14 after one solve),
    but on this mesh that difference grows 10-30x per step along the trajectory (3.5e-11 after four
    steps, 6e-9 with two solves per step), and within one solve it grows exponentially beyond ~200
    iterations (1e-8 after 400, 1e-5 after 800): the usual finite-precision behaviour of long CG runs
    and of an inexact Newton iteration, not of the kernels (forces agree to 4e-14)."""
    mesh = I.workload_cylinder(256, "FS")
    ost = oracle_stencils("FS", mesh)
    osim = O.Sim(ost, MAT, mesh.pinned)
    with S.Problem(mesh, MAT, model="FS", block_vertices=2048) as pb:
        for _ in range(3):
            counts, _ = osim.step(1 / 30, max_newton=1, pcg_rtol=1e-2, max_pcg=150)
            params, _keep = S.step_params(1 / 30, max_newton=1, replay=counts)
            rc, st = S.shell_step_implicit(pb.sim, params)
            assert np.array_equal(st["counts"], counts[: st["newton_iters"]])
        x, v, _ = S.shell_sim_get_state(pb.sim, mesh.nv)
    assert rel(x - mesh.X, osim.x - mesh.X) <= TOL64
    assert rel(v, osim.v) <= TOL64


def test_tolerance_mode_counts_close_to_oracle():
    mesh = I.workload_plate32()
    ost = oracle_stencils("EP", mesh)
    osim = O.Sim(ost, MAT, mesh.pinned)
    counts, _ = osim.step(1 / 60, max_newton=1, pcg_rtol=1e-10)
    with S.Problem(mesh, MAT) as pb:
        params, _ = S.step_params(1 / 60, max_newton=1, pcg_rtol=1e-10)
        rc, st = S.shell_step_implicit(pb.sim, params)
        assert rc == S.SHELL_OK
        assert abs(int(st["counts"][0, 2]) - int(counts[0, 2])) <= 1
        x, _, _ = S.shell_sim_get_state(pb.sim, mesh.nv)
        assert rel(x - mesh.X, osim.x - mesh.X) <= 1e-8


def test_budget_status_is_returned():
    mesh = I.workload_plate32()
    with S.Problem(mesh, MAT) as pb:
        params, _ = S.step_params(1 / 60, max_newton=1, pcg_rtol=1e-12, max_pcg=3)
        rc, st = S.shell_step_implicit(pb.sim, params)
        assert rc == S.SHELL_E_BUDGET and st["counts"][0, 2] == 3


def test_state_roundtrip_and_resume():
    """N + M steps equal N steps, save, restore into a fresh simulation, M steps (two independently built
    problems; bitwise, since every sum on the path has a fixed order)."""
    mesh = I.workload_cylinder(20, "SS")
    params, _ = S.step_params(1 / 30, max_newton=2, pcg_rtol=1e-6)
    with S.Problem(mesh, MAT) as a, S.Problem(mesh, MAT) as b:
        for _ in range(3):
            S.shell_step_implicit(a.sim, params)
        x, v, step = S.shell_sim_get_state(a.sim, mesh.nv)
        S.shell_sim_set_state(b.sim, x, v, step)
        for _ in range(2):
            S.shell_step_implicit(a.sim, params)
            S.shell_step_implicit(b.sim, params)
        xa, va, sa = S.shell_sim_get_state(a.sim, mesh.nv)
        xb, vb, sb = S.shell_sim_get_state(b.sim, mesh.nv)
        assert sa == sb == 5
        assert np.array_equal(xa, xb) and np.array_equal(va, vb)


# ------------------------------------------------------------------ edge cases


def test_empty_mesh():
    st = S.shell_build_stencils(np.zeros((0, 3)), np.zeros((0, 3), np.int32), "SS", MAT)
    try:
        assert S.shell_stencils_info(st)["ns"] == 0
        x = torch.zeros((0, 3), dtype=torch.float64, device=dev())
        S.shell_eval_forces(st, x, torch.zeros_like(x))
    finally:
        S.shell_destroy_stencils(st)


@pytest.mark.parametrize("model", I.MODELS)
def test_single_and_two_triangle_meshes(model):
    kb = MAT["young"] * MAT["thickness"] ** 3 / (12 * (1 - MAT["poisson"] ** 2))
    X = np.array([[0, 0, 0], [1, 0, 0.1], [0, 1, 0], [1, 1, 0.3]], float)
    for tris in (np.array([[0, 1, 2]], np.int32), np.array([[0, 1, 2], [1, 3, 2]], np.int32)):
        ost = oracle_stencils(model, type("M", (), dict(X=X, tris=tris))())
        x = X + 0.05 * I.rng(2).standard_normal(X.shape)
        f_ref, e_ref = ost.forces(x)
        st = S.shell_build_stencils(X, tris, model, MAT)
        try:
            f, e = gpu_forces(st, x)
            # a lone triangle has every edge free: its folded operator vanishes and only rounding
            # noise remains, so the scale is the bending rigidity times the deformation
            atol = 1e-12 * kb * np.abs(x - X).max()
            assert np.abs(f - f_ref).max() <= TOL64 * np.abs(f_ref).max() + atol
            assert abs(e - e_ref) <= TOL64 * abs(e_ref) + atol * 1e-3
        finally:
            S.shell_destroy_stencils(st)


def test_clamped_edge_that_is_not_a_boundary_edge_is_rejected():
    mesh = I.plate_mesh(8, 1.0, 0.0, 1, "FP")
    for bad in ([[0, mesh.nv]], [[0, 9]], [[0, 63]]):  # out of range, interior diagonal, not an edge
        with pytest.raises(S.ShellError) as err:
            S.shell_build_stencils(mesh.X, mesh.tris, "FP", MAT, clamped_edges=bad)
        assert err.value.status == S.SHELL_E_INVALID_ARG


def test_invalid_meshes_are_rejected():
    X = I.rng(0).standard_normal((6, 3))
    cases = [(np.array([[0, 1, 2], [1, 2, 3]], np.int32), 3),
             (np.array([[0, 1, 2], [2, 1, 3], [1, 2, 4]], np.int32), 2),
             (np.array([[0, 1, 1]], np.int32), 4),
             (np.array([[0, 1, 9]], np.int32), 1)]
    for tris, code in cases:
        with pytest.raises(S.ShellError) as ei:
            S.shell_build_stencils(X, tris, "EP", MAT)
        assert ei.value.status == code
    Xd = np.array([[0, -1, 0], [-1, 0, 0], [1, 0, 0], [0.3, 0, 0]], float)
    with pytest.raises(S.ShellError) as ei:
        S.shell_build_stencils(Xd, np.array([[0, 1, 2], [3, 2, 1]], np.int32), "EP", MAT)
    assert ei.value.status == 4


# ------------------------------------------------------------------ full-size workloads


@pytest.fixture(scope="module")
def cap_problem():
    mesh = I.workload_sphere_cap(1024, "SS")
    pb = S.Problem(mesh, MAT)  # the benchmark's configuration (default tiles, Morton order)
    yield mesh, pb
    pb.close()


@pytest.fixture(scope="module")
def cap_oracle(cap_problem):
    mesh, _ = cap_problem
    return oracle_stencils("SS", mesh)


def test_full_size_sphere_cap_forces_match_oracle(cap_problem, cap_oracle):
    """1024 x 1024 smoothed-hinge shell cap (2,093,058 stencils): every vertex's force."""
    mesh, pb = cap_problem
    assert pb.info["ns"] == 2 * 1023 * 1023
    ost = cap_oracle
    x = mesh.X + 1e-4 * I.rng(21).standard_normal(mesh.X.shape)
    f_ref, e_ref = ost.forces(x)
    f, e = gpu_forces(pb.st, x)
    assert rel(f, f_ref) <= TOL64 and relmax(f, f_ref) <= TOL64
    assert abs(e - e_ref) <= TOL64 * abs(e_ref)


def test_full_size_operator_properties(cap_problem):
    """At any size K_s annihilates constants and is symmetric: p.Kq = q.Kp."""
    mesh, pb = cap_problem
    n = mesh.nv
    ones = torch.ones((n, 3), dtype=torch.float64, device=dev())
    q = torch.zeros_like(ones)
    S.shell_hessian_apply(pb.h, None, 1.0, ones, q)
    g = I.rng(22)
    p1 = torch.tensor(g.standard_normal((n, 3)), device=dev())
    p2 = torch.tensor(g.standard_normal((n, 3)), device=dev())
    k1 = torch.zeros_like(p1)
    k2 = torch.zeros_like(p2)
    S.shell_hessian_apply(pb.h, None, 1.0, p1, k1)
    S.shell_hessian_apply(pb.h, None, 1.0, p2, k2)
    torch.cuda.synchronize()
    scale = torch.linalg.norm(k1).item()
    assert torch.abs(q).max().item() <= 1e-12 * scale
    a = torch.sum(p2 * k1).item()
    b = torch.sum(p1 * k2).item()
    assert abs(a - b) <= 1e-11 * abs(a)


@pytest.fixture(scope="module")
def cap_oracle_newton(cap_problem, cap_oracle):
    """The oracle's state after one Newton iteration from rest with 20 PCG iterations per coordinate."""
    mesh, _ = cap_problem
    osim = O.Sim(cap_oracle, MAT, mesh.pinned)
    counts = np.full((1, 3), 20, np.int32)
    osim.step(1 / 30, gravity=I.GRAVITY, max_newton=1, replay=counts)
    return counts, osim.x.copy()


@pytest.mark.parametrize("precision", [S.SHELL_PREC_FP64, S.SHELL_PREC_MIXED])
def test_full_size_newton_iteration_matches_oracle(cap_problem, cap_oracle_newton, precision):
    """The benchmark's configuration (1024 x 1024 SS cap, default tiles, PCG launch shape and captured
    graphs): one Newton iteration from rest with 20 replayed PCG iterations per coordinate, every vertex
    against the oracle.  FP64 to 1e-10 (observed 4e-14); mixed to 1e-5 (float matrix, forces and
    increment; observed 1.2e-7)."""
    mesh, pb64 = cap_problem
    counts, x_ref = cap_oracle_newton
    params, _keep = S.step_params(1 / 30, gravity=I.GRAVITY, max_newton=1, replay=counts)
    if precision == S.SHELL_PREC_FP64:
        S.shell_sim_set_state(pb64.sim, mesh.X, np.zeros_like(mesh.X), 0)
        S.shell_step_implicit(pb64.sim, params)
        x, _, _ = S.shell_sim_get_state(pb64.sim, mesh.nv)
    else:
        with S.Problem(mesh, MAT, precision=precision) as pb:
            S.shell_step_implicit(pb.sim, params)
            x, _, _ = S.shell_sim_get_state(pb.sim, mesh.nv)
    err = rel(x - mesh.X, x_ref - mesh.X)
    print(f"full-size Newton iteration, precision {precision}: displacement rel err {err:.2e}")
    assert err <= (TOL64 if precision == S.SHELL_PREC_FP64 else 1e-5)


# ------------------------------------------------------------------ multi-mesh batch


def _batch_meshes():
    """Six meshes, one per model, of uneven sizes (several tiles, ragged tails)."""
    out = []
    for k, model in enumerate(I.MODELS):
        n = (9, 23, 17, 31, 12, 26)[k]
        spec = dict(n=n, model=model, radius=0.4 + 0.2 * k, seed=100 + k)
        out.append(I.mesh_from_spec(spec, spacing=0.02))
    return out


@pytest.mark.parametrize("precision", [S.SHELL_PREC_FP64, S.SHELL_PREC_MIXED])
def test_batch_equals_each_mesh_alone(precision):
    """Each mesh stepped inside a mixed batch equals the same mesh stepped alone.  The alone run is in
    tolerance mode; the batch replays its per-mesh counts (a batch splits a mesh's rows over other
    work-groups than a lone launch, so its dot products sum their partials in another order, and a
    tolerance-mode count may move by one or two when that rounding moves a residual across the
    threshold)."""
    meshes = _batch_meshes()
    params, _ = S.step_params(1 / 60, max_newton=3, pcg_rtol=1e-6)
    alone, inbatch = [], []
    try:
        for m in meshes:
            alone.append(S.Problem(m, MAT, precision=precision, block_vertices=128))
            inbatch.append(S.Problem(m, MAT, precision=precision, block_vertices=128))
        batch = S.shell_batch_create([pb.sim for pb in inbatch])
        try:
            for _ in range(3):
                plist, keep = [], []
                for k, pb in enumerate(alone):
                    _, st = S.shell_step_implicit(pb.sim, params)
                    counts = np.zeros((3, 3), np.int32)
                    counts[: st["newton_iters"]] = st["counts"]
                    p, kp = S.step_params(1 / 60, max_newton=st["newton_iters"], pcg_rtol=1e-6, replay=counts)
                    plist.append(p)
                    keep.append(kp)
                rc, bstats = S.shell_batch_step(batch, plist, len(meshes))
                for k in range(len(meshes)):
                    assert bstats[k]["newton_iters"] == plist[k].max_newton
            tol = 1e-10 if precision == S.SHELL_PREC_FP64 else 1e-5
            for m, a, b in zip(meshes, alone, inbatch):
                xa, va, _ = S.shell_sim_get_state(a.sim, m.nv)
                xb, vb, _ = S.shell_sim_get_state(b.sim, m.nv)
                assert rel(xb - m.X, xa - m.X) <= tol, m.name
        finally:
            S.shell_destroy_batch(batch)
    finally:
        for pb in alone + inbatch:
            pb.close()


def test_batch_of_clamped_and_world_frame_meshes_matches_oracle():
    """One batch of a clamped edge plate and a clamped smoothed plate (each with its own constant clamp
    force), a world-frame edge shell and a plain smoothed shell, FP64, counts replayed per mesh: every
    mesh equals the oracle's run of it to 1e-10."""
    cases = []
    for model, n in (("EP", 19), ("SP", 23)):
        mesh, cl = _clamp_mesh(model, n)
        cases.append((mesh, model, dict(clamped_edges=cl), dict(clamped=cl)))
    cyl = _qt_mesh("ES", 21)
    cases.append((cyl, "ES", dict(flags=S.SHELL_FLAG_WORLD_FRAME), dict(world_frame=True)))
    cap = I.sphere_cap_mesh(27, 0.8, jitter=0.2, seed=7, model="SS")
    cases.append((cap, "SS", {}, {}))
    osims, probs = [], []
    try:
        for mesh, model, gkw, okw in cases:
            ost = O.Stencils(model, mesh.X, mesh.tris, MAT["young"], MAT["poisson"], MAT["thickness"], **okw)
            osims.append(O.Sim(ost, MAT, mesh.pinned))
            probs.append(S.Problem(mesh, MAT, model=model, block_vertices=128, **gkw))
        batch = S.shell_batch_create([pb.sim for pb in probs])
        try:
            for _ in range(2):
                plist, keep = [], []
                for osim in osims:
                    counts, ost = osim.step(1 / 30, max_newton=2, pcg_rtol=1e-8)
                    p, kp = S.step_params(1 / 30, max_newton=ost["newton_iters"], pcg_rtol=1e-8, replay=counts)
                    plist.append(p)
                    keep.append(kp)
                S.shell_batch_step(batch, plist, len(plist))
        finally:
            S.shell_destroy_batch(batch)
        for (mesh, model, _, _), osim, pb in zip(cases, osims, probs):
            x, v, _ = S.shell_sim_get_state(pb.sim, mesh.nv)
            assert rel(x - mesh.X, osim.x - mesh.X) <= TOL64, model
            assert rel(v, osim.v) <= TOL64, model
    finally:
        for pb in probs:
            pb.close()


def test_batch_replay_matches_oracle_per_mesh():
    """A batch of all six models, per-mesh parameters and replayed counts, against the oracle."""
    meshes = _batch_meshes()
    dts = [1 / 60, 1 / 30, 1 / 45, 1 / 60, 1 / 30, 1 / 50]
    osims = []
    for m in meshes:
        ost = oracle_stencils(m.model, m)
        osims.append(O.Sim(ost, MAT, m.pinned))
    probs = [S.Problem(m, MAT, block_vertices=64) for m in meshes]
    batch = S.shell_batch_create([pb.sim for pb in probs])
    try:
        for _ in range(2):
            plist, keep = [], []
            for k, m in enumerate(meshes):
                counts, _ = osims[k].step(dts[k], max_newton=2, pcg_rtol=1e-9)
                p, kp = S.step_params(dts[k], max_newton=2, pcg_rtol=1e-9, replay=counts)
                plist.append(p)
                keep.append(kp)
            S.shell_batch_step(batch, plist, len(meshes))
        for k, m in enumerate(meshes):
            x, v, _ = S.shell_sim_get_state(probs[k].sim, m.nv)
            assert rel(x - m.X, osims[k].x - m.X) <= TOL64, m.name
            assert rel(v, osims[k].v) <= TOL64, m.name
    finally:
        S.shell_destroy_batch(batch)
        for pb in probs:
            pb.close()


def test_batch_of_staged_and_direct_products_with_profiling_matches_oracle():
    """One batch holding meshes of both product forms (LDS-staged and direct gathers), PCG work-groups
    that walk row groups of several meshes, and in-step sampling on: every mesh matches the oracle."""
    meshes = _batch_meshes()[:4]
    flags = [0, S.SHELL_FLAG_DIRECT_PRODUCT, 0, S.SHELL_FLAG_DIRECT_PRODUCT]
    osims = [O.Sim(oracle_stencils(m.model, m), MAT, m.pinned) for m in meshes]
    probs = [S.Problem(m, MAT, block_vertices=64, flags=f) for m, f in zip(meshes, flags)]
    batch = S.shell_batch_create([pb.sim for pb in probs])
    try:
        S.shell_batch_profile(batch, 2)
        for _ in range(2):
            plist, keep = [], []
            for k, m in enumerate(meshes):
                counts, _ = osims[k].step(1 / 45, max_newton=2, pcg_rtol=1e-9)
                p, kp = S.step_params(1 / 45, max_newton=2, pcg_rtol=1e-9, replay=counts, pcg_workgroups=3)
                plist.append(p)
                keep.append(kp)
            S.shell_batch_step(batch, plist, len(meshes))
        prof = S.shell_batch_profile_read(batch)
        assert prof["product"]["count"] > 0 and prof["update"]["count"] > 0 and prof["forces"]["count"] >= 4
        for k, m in enumerate(meshes):
            x, v, _ = S.shell_sim_get_state(probs[k].sim, m.nv)
            assert rel(x - m.X, osims[k].x - m.X) <= TOL64, m.name
            assert rel(v, osims[k].v) <= TOL64, m.name
    finally:
        S.shell_destroy_batch(batch)
        for pb in probs:
            pb.close()


def test_mixed_precision_step_error_against_oracle():
    """Mixed path, replaying the oracle's counts: per-step displacement error stays within 1e-6 (measured
    about 5e-8; float32 operators with float64 Newton refinement) on the
    clamped plate and the cylinder patch."""
    for mesh, model, dt, newton, rtol in ((I.workload_plate32(), "EP", 1 / 60, 2, 1e-10),
                                          (I.workload_cylinder(24, "FS"), "FS", 1 / 30, 3, 1e-8)):
        ost = oracle_stencils(model, mesh)
        osim = O.Sim(ost, MAT, mesh.pinned)
        with S.Problem(mesh, MAT, model=model, precision=S.SHELL_PREC_MIXED, block_vertices=128) as pb:
            for step in range(3):
                counts, _ = osim.step(dt, max_newton=newton, pcg_rtol=rtol)
                params, _k = S.step_params(dt, max_newton=newton, pcg_rtol=rtol, replay=counts)
                S.shell_step_implicit(pb.sim, params)
                x, _, _ = S.shell_sim_get_state(pb.sim, mesh.nv)
                err = rel(x - mesh.X, osim.x - mesh.X)
                print(f"{model} mixed step {step}: displacement rel err {err:.2e}")
                assert err <= 1e-6


# ------------------------------------------------------------------ serving


def test_served_results_equal_each_request_alone():
    """Requests served together by the continuous-batching server (mixed precision) end where the same
    meshes stepped alone end, within the mixed-precision tolerance."""
    from paper_2502_10872_amd import serve as V

    cfg = V.ServeConfig(hbm_budget=1 << 34, builders=2, keep_state=True, max_newton=2, pcg_rtol=1e-6)
    specs = [dict(n=n, model=m, radius=0.5 + 0.1 * k, seed=300 + k)
             for k, (n, m) in enumerate([(20, "EP"), (34, "SS"), (27, "FS"), (15, "ES"), (40, "SP"), (22, "FP")])]
    reqs = [V.Request(rid=k, t_arrival=0.0, spec=sp, steps=4) for k, sp in enumerate(specs)]
    out = V.Server(V.GpuExecutor(cfg), cfg).run(reqs, realtime=False)
    assert out["completed"] == len(specs) and out["max_batch"] >= 2
    for r in reqs:
        mesh = I.mesh_from_spec(r.spec, spacing=0.01)
        with S.Problem(mesh, MAT, precision=S.SHELL_PREC_MIXED) as pb:
            params, _ = S.step_params(cfg.dt, max_newton=2, pcg_rtol=1e-6)
            for _ in range(4):
                S.shell_step_implicit(pb.sim, params)
            x, _, _ = S.shell_sim_get_state(pb.sim, mesh.nv)
        assert rel(r.result - mesh.X, x - mesh.X) <= 1e-4, r.spec
