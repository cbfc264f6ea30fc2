"""Benchmark: implicit steps/s and bending stencils/s at about 1M vertices, against the HBM roofline.

Workload: the irregular sphere-cap shell, 1024 x 1024 vertices (2,093,058 triangle stencils), radius
drawn from U[0.3, 2] m with its seed, in-plane jitter 0.2 of the spacing, smoothed-hinge shell model,
boundary ring pinned, dt = 1/30 s, gravity; each step is one implicit-Euler step (predictor, Newton
iterations with force evaluation, residual and a three-column Jacobi-PCG solve against the constant
Hessian, velocity update).  Inputs are resident in HBM before the timed region.

Prints one JSON line.  Only one GPU is used; --gpus above 1 is refused.
"""

from __future__ import annotations

import argparse
import json
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, published


def algorithmic_bytes(info: dict, hinfo: dict, precision: int, clamp_bias: bool = False) -> dict:
    """Bytes each kernel must move once (no re-reads, no SELL padding), per launch.

    force:  per stencil its k vertex ids, the operator (FP64: r x k entries; mixed: r x (k - 1), the
            origin's column being implied by the zero row sums), (shells) r float64 rest curvatures and
            (mixed edge plate) the tip's two float64 rest-plane coordinates; per vertex the float64 position
            read (mixed triangle plates also the rest position) and the force written; FP64 plates with
            clamped edges also read the constant clamp force per vertex.
    spmv:   (the product kernel, which also forms the new direction p = z + beta p_old) every nonzero's
            value and 16-bit local column id, each row group's distinct-column list, slice widths and
            offsets, and per vertex the direction's inputs (FP64: r and D^-1; mixed: the stored float z)
            and p_old, the mass (-1 on fixed rows, in the vector precision) read, p and q written.
    update: per vertex p, q, y, r, D^-1 read, y and r written (mixed: z written too; y is float in mixed
            precision, r float64 in both)."""
    nv, ns, k, r = info["nv"], info["ns"], info["k"], info["r"]
    shell = info["model"] in (1, 3, 5)
    mixed = precision == 1
    real = 4 if mixed else 8  # stencil operators, matrix values, p, q, z, D^-1, forces
    per_stencil = (4 * k + real * r * (k - 1 if mixed else k) + (8 * r if shell else 0)
                   + (16 if mixed and k == 4 and not shell else 0))
    force = (ns * per_stencil + nv * (24 + 3 * real) + (nv * 24 if clamp_bias and not mixed else 0)
             + (nv * 24 if mixed and k == 6 and not shell else 0))
    ngroups = (nv + 511) // 512  # 512-row groups
    idx = 2 if hinfo["staged"] else 4
    direction_in = 3 * real if mixed else 24 + real
    spmv = (hinfo["nnz"] * (real + idx) + 4 * (hinfo["group_cols"] + ngroups + 1) + 12 * hinfo["nslices"]
            + nv * (direction_in + 3 * real + real + 3 * real + 3 * real))
    update = nv * (3 * real + 3 * real + 3 * real + 24 + real + 3 * real + 24 + (3 * real if mixed else 0))
    return dict(force=force, spmv=spmv, update=update, force_per_stencil=per_stencil)


TRAFFIC_SUMMARY = os.path.join(ROOT, "profiles", "sphere_cap_1024_ss_hbm_traffic.md")
# the device code of the measured kernels, the layouts they read (host_mesh.cpp and precompute.hip build
# them, internal.hpp declares the descriptors) and their launch shapes (solver.hip)
TRAFFIC_SOURCES = ["paper_2502_10872_amd/csrc/spmv.hpp", "paper_2502_10872_amd/csrc/pcg_kernels.hpp",
                   "paper_2502_10872_amd/csrc/forces.hip", "paper_2502_10872_amd/csrc/host_mesh.cpp",
                   "paper_2502_10872_amd/csrc/devmath.hpp", "paper_2502_10872_amd/csrc/precompute.hip",
                   "paper_2502_10872_amd/csrc/solver.hip", "paper_2502_10872_amd/csrc/internal.hpp"]


def sources_digest(files=TRAFFIC_SOURCES) -> str:
    """sha256 prefix of the code of the measured kernels: the sources with comments and blank lines
    removed, so that a change to a comment does not retire the counter summary while any change to the
    code does."""
    import hashlib
    import re

    h = hashlib.sha256()
    for f in files:
        text = open(os.path.join(ROOT, f)).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        lines = [re.sub(r"//.*$", "", line).rstrip() for line in text.splitlines()]
        h.update("\n".join(line for line in lines if line.strip()).encode())
    return h.hexdigest()[:16]


def measured_traffic(key: str):
    """HBM bytes per launch from the committed counter summary, or None when the kernels' code has
    changed since the counters were taken (or the summary is absent)."""
    try:
        text = open(TRAFFIC_SUMMARY).read()
    except OSError:
        return None
    fields = dict(line.split(": ", 1) for line in text.splitlines() if ": " in line and not line.startswith("|"))
    if fields.get("sources_sha256", "").strip() != sources_digest() or key not in fields:
        return None
    return float(fields[key])


def host_cpu() -> dict:
    """The host's processor model and the cores this process may use."""
    model = platform.processor() or "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    nproc = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    return dict(model=model, nproc=nproc, logical_cpus=os.cpu_count(),
                omp_num_threads=os.environ.get("OMP_NUM_THREADS"))


def _oracle_step_sample(O, sim, st, X):
    """One force evaluation, then one Newton solve with 10 and with 40 replayed PCG iterations per
    coordinate; returns the per-part times (force, Newton overhead without forces, one coordinate
    PCG iteration)."""
    t0 = time.perf_counter()
    st.forces(X)
    t_force = time.perf_counter() - t0
    times = {}
    for n in (10, 40):
        sim.x[:] = X
        sim.v[:] = 0.0
        t0 = time.perf_counter()
        sim.step(1 / 30, max_newton=1, replay=np.full((1, 3), n, np.int32))
        times[n] = time.perf_counter() - t0
    t_iter = max(times[40] - times[10], 1e-9) / 90.0  # one PCG iteration of one coordinate
    t_newton = max(times[10] - 30 * t_iter, 0.0)  # predictor, 2 force evaluations and residuals, PCG setup
    return dict(force=t_force, newton_overhead=t_newton, pcg_coord_iter=t_iter, newton_10=times[10],
                newton_40=times[40])


def cpu_baseline(mesh, material, counts_per_step, newton_per_step):
    """The FP64 CPU oracle on the same mesh, on one thread (the plain build) and on all host cores (the
    OpenMP timing build of the same source): one force evaluation and a short replayed PCG run are
    timed, then scaled to the GPU step's measured Newton and PCG iteration counts."""
    import oracle as O

    host = host_cpu()
    O.use_openmp(False)
    st = O.Stencils("SS", mesh.X, mesh.tris, material["young"], material["poisson"], material["thickness"])
    sim = O.Sim(st, material, mesh.pinned)

    def steps_per_s(t):
        t_setup = max(t["newton_overhead"] - 2 * t["force"], 0.0)
        step_s = newton_per_step * t_setup + (newton_per_step + 1) * t["force"] + counts_per_step * t["pcg_coord_iter"]
        return 1.0 / step_s

    legs = {}
    try:
        for omp in (False, True):
            threads = O.use_openmp(omp, host["nproc"] if omp else 0)
            t = _oracle_step_sample(O, sim, st, mesh.X)
            legs[omp] = dict(value=steps_per_s(t), cores=threads, seconds=t)
    finally:
        O.use_openmp(False)
    one, allc = legs[False], legs[True]
    sample = (f"full {int(round(mesh.nv ** 0.5))}^2 SS cap: one force evaluation and one Newton solve with 10 and "
              f"40 replayed PCG iterations per coordinate, scaled to {newton_per_step:.1f} Newton solves and "
              f"{counts_per_step:.0f} PCG coordinate-iterations per step (the GPU step's counts)")
    print(f"[bench] oracle: 1 thread {one['value']:.2e} steps/s, {allc['cores']} threads "
          f"{allc['value']:.2e} steps/s", file=sys.stderr, flush=True)
    return dict(value=allc["value"], unit="steps/s", cores=allc["cores"], kind="oracle",
                build="OpenMP timing build (stencil loop, sparse product and vector loops parallel)",
                sample=sample, host=host, seconds=allc["seconds"],
                single_thread=dict(value=one["value"], unit="steps/s", cores=1, build="plain serial build",
                                   seconds=one["seconds"]),
                parallel_speedup=allc["value"] / one["value"])


CLAMPED_PLATE_ALPHA = 0.0012653  # clamped square plate, w_max = alpha q a^4 / D (Timoshenko & Woinowsky-Krieger)


def static_plate(I, n):
    """The linear plate benchmark's square (side 8, E = 2e11, nu = 0.3, h = 0.01, load 9.81 per unit area),
    n x n vertices, jitter 0.2, every boundary edge clamped and held."""
    m = I.plate_mesh(n, 8.0, 0.2, 5, "SP", "ring")
    mat = dict(young=2e11, poisson=0.3, thickness=0.01, density=1.0)
    area = np.zeros(m.nv)
    t = m.tris
    a = 0.5 * np.linalg.norm(np.cross(m.X[t[:, 1]] - m.X[t[:, 0]], m.X[t[:, 2]] - m.X[t[:, 0]]), axis=1)
    for c in range(3):
        np.add.at(area, t[:, c], a / 3.0)
    load = np.zeros((m.nv, 3))
    load[:, 2] = -9.81 * area
    return m, mat, I.boundary_edges(m.tris), load


def quasi_static(S, I, torch, sizes=(65, 257)):
    """Quasi-static Newton-Raphson (eq 64) on the linear plate benchmark with clamped edges (SP, FP64):
    one solve to PCG rtol 1e-10 (the plate is linear), timed end to end on the device-resident state;
    the centre deflection against the classical clamped-plate value."""
    out = {}
    for n in sizes:
        m, mat, cl, load = static_plate(I, n)
        pb = S.Problem(m, mat, model="SP", clamped_edges=cl)
        eps_f = 1e-8 * float(np.linalg.norm(load))
        S.shell_solve_static(pb.sim, load, eps_f=eps_f, max_newton=1, pcg_rtol=1e-10)  # warm-up (graphs)
        S.shell_sim_set_state(pb.sim, m.X, None, 0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rc, st = S.shell_solve_static(pb.sim, load, eps_f=eps_f, max_newton=2, pcg_rtol=1e-10)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3
        x, _, _ = S.shell_sim_get_state(pb.sim, m.nv)
        D = mat["young"] * mat["thickness"] ** 3 / (12 * (1 - mat["poisson"] ** 2))
        ratio = float(-(x[:, 2] - m.X[:, 2]).min() / (CLAMPED_PLATE_ALPHA * 9.81 * 8.0**4 / D))
        iters = int(np.max(st["counts"][: st["newton_iters"]].sum(axis=0))) if st["newton_iters"] else 0
        out[f"SP_clamped_{n}"] = dict(nv=m.nv, newton_iters=st["newton_iters"], pcg_iters=iters, ms=ms,
                                      us_per_pcg_iteration=ms * 1e3 / max(iters, 1), deflection_ratio=ratio,
                                      residual_rel=st["grad_norm"] / max(st["grad_norm0"], 1e-300), status=rc)
        pb.close()
        print(f"[bench] quasi-static plate {n} done", file=sys.stderr, flush=True)
    return out


def membrane_timing(S, I, torch, reps=20):
    """The membrane pass (SHELL_FLAG_MEMBRANE) on the 1024 x 1024 sphere cap: shell_eval_forces timed with
    and without it on the same state, the difference being the membrane kernel (one thread per triangle,
    atomic adds into the force).  Algorithmic bytes: per triangle its ids and rest data (52 B), per vertex
    the positions (FP64) or rest positions and displacements (mixed) read once and the force read and
    written once."""
    cap = I.workload_sphere_cap(1024, "SS")
    x = torch.tensor(cap.X + 1e-4 * I.rng(5).standard_normal(cap.X.shape), device="cuda")
    out = {}
    for prec in (S.SHELL_PREC_MIXED, S.SHELL_PREC_FP64):
        mixed = prec == S.SHELL_PREC_MIXED
        f = torch.zeros(x.shape, dtype=torch.float32 if mixed else torch.float64, device="cuda")
        ms = {}
        for flags in (0, S.SHELL_FLAG_MEMBRANE):
            st = S.shell_build_stencils(cap.X, cap.tris, "SS", I.MATERIAL, precision=prec, flags=flags)
            S.shell_eval_forces(st, x, f, None)
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(reps):
                S.shell_eval_forces(st, x, f, None)
            e1.record()
            torch.cuda.synchronize()
            ms[flags] = e0.elapsed_time(e1) / reps
            S.shell_destroy_stencils(st)
        nv, nt = cap.nv, len(cap.tris)
        alg = nt * 52 + nv * ((24 + 32 + 24) if mixed else (24 + 48))
        dm = ms[S.SHELL_FLAG_MEMBRANE] - ms[0]
        out["mixed" if mixed else "fp64"] = dict(triangles=nt, eval_forces_ms=ms[0], with_membrane_ms=ms[S.SHELL_FLAG_MEMBRANE],
                                                 membrane_ms=dm, gbs=alg / (dm * 1e-3) / 1e9 if dm > 0 else None)
    print("[bench] membrane timing done", file=sys.stderr, flush=True)
    return out


MEMBRANE_STAGED_MIN_ROWS = 32768  # the library's staged membrane product from this many vertices up


def membrane_product_bytes(nv, nnz_s, nnz_m, mixed=False):
    """Algorithmic bytes of one coupled product launch: K_s (a column id and a value per entry), the
    membrane tangent's 3x3 blocks (a column id and nine values per block), the values float64 (float32 in
    mixed precision), the mass and the held mask, z and the previous direction read once, the new
    direction and q written once (float64 vectors in both precisions).  The staged SELL layout (from
    MEMBRANE_STAGED_MIN_ROWS vertices) has 2-byte group-local column ids, its slice offsets and the
    groups' column lists (a few bytes per row) not counted; the CSR layout has 4-byte ids and two 8-byte
    row offsets per row."""
    real = 4 if mixed else 8
    if nv >= MEMBRANE_STAGED_MIN_ROWS:
        return (2 + real) * nnz_s + (2 + 9 * real) * nnz_m + nv * (8 + 1 + 48 + 48)
    return 16 * (nv + 1) + (4 + real) * nnz_s + (4 + 9 * real) * nnz_m + nv * (8 + 1 + 48 + 48)


def membrane_step_timing(S, I, torch, sizes=(64, 256, 1024), steps=2):
    """The implicit step of the smoothed-hinge shell with its membrane (the membrane tangent, coupled
    Jacobi-PCG, Armijo backtracking) on a cylinder patch of radius 0.5 m held at its ends, dt = 1/30,
    Newton budget 4, PCG rtol 1e-2 (the headline step's settings), FP64 and mixed: time per step and its
    iteration counts, then the coupled product and update launched back to back (shell_sim_time_kernels)
    with the product's fraction of the HBM peak on its algorithmic bytes."""
    out = {}
    for n, prec in [(n, p) for n in sizes for p in (S.SHELL_PREC_FP64, S.SHELL_PREC_MIXED)]:
        mixed = prec == S.SHELL_PREC_MIXED
        mesh = I.cylinder_mesh(n, 0.5, 0.9, 0.8, 0.2, 3, "SS", "ends")
        pb = S.Problem(mesh, I.MATERIAL, model="SS", precision=prec, flags=S.SHELL_FLAG_MEMBRANE)
        params, _ = S.step_params(1 / 30, max_newton=4, newton_rtol=1e-8, pcg_rtol=1e-2)
        S.shell_step_implicit(pb.sim, params)  # warm-up
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        stats = [S.shell_step_implicit(pb.sim, params)[1] for _ in range(steps)]
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / steps
        pcg = sum(st["pcg_total"] for st in stats)
        kt = S.shell_sim_time_kernels(pb.sim, 1 / 30, reps=10)
        nnz_s = S.shell_hessian_info(pb.h)["nnz"]
        t = np.sort(mesh.tris, axis=1)
        edges = np.unique(np.concatenate([t[:, [0, 1]], t[:, [1, 2]], t[:, [0, 2]]]), axis=0)
        nnz_m = mesh.nv + 2 * len(edges)
        pbytes = membrane_product_bytes(mesh.nv, nnz_s, nnz_m, mixed)
        gbs = pbytes / (kt["spmv_ms"] * 1e-3) / 1e9 if kt["spmv_ms"] else None
        out[f"SS_membrane_cylinder_{n}" + ("_mixed" if mixed else "")] = dict(
            nv=mesh.nv, steps_per_s=1e3 / ms, ms_per_step=ms,
            newton_per_step=sum(st["newton_iters"] for st in stats) / steps,
            pcg_per_step=pcg / steps, us_per_pcg_iteration=ms * 1e3 * steps / max(pcg, 1),
            halvings=[int(c[1]) for st in stats for c in st["counts"]],
            grad_ratio=[st["grad_norm"] / max(st["grad_norm0"], 1e-300) for st in stats],
            back_to_back_ms=dict(force=kt["force_ms"], product=kt["spmv_ms"], update=kt["update_ms"]),
            product=dict(kernel="ms_iter_product_staged" if mesh.nv >= MEMBRANE_STAGED_MIN_ROWS else "ms_iter_product",
                         bytes_per_launch=pbytes, achieved_gbs=gbs,
                         frac=gbs / HBM_PEAK_GBS if gbs else None, nnz_s=nnz_s, blocks=nnz_m))
        pb.close()
        print(f"[bench] membrane step {n} {'mixed' if mixed else 'fp64'}: {ms:.1f} ms/step, "
              f"product {1e3 * kt['spmv_ms']:.1f} us", file=sys.stderr, flush=True)
    return out


def cpu_membrane_step(I, n=64):
    """The oracle's step with the membrane on the same 64 x 64 cylinder, one step."""
    import oracle as O

    mesh = I.cylinder_mesh(n, 0.5, 0.9, 0.8, 0.2, 3, "SS", "ends")
    m = I.MATERIAL
    st = O.Stencils("SS", mesh.X, mesh.tris, m["young"], m["poisson"], m["thickness"])
    sim = O.MembraneSim(st, m, mesh.pinned)
    t0 = time.perf_counter()
    _, _, stats = sim.step(1 / 30, max_newton=4, newton_rtol=1e-8, pcg_rtol=1e-2)
    return dict(workload=f"SS_membrane_cylinder_{n}", seconds_per_step=time.perf_counter() - t0,
                pcg_per_step=stats["pcg_total"], cores=1)


def navier_rectangle(a, b, nterm=199):
    """Navier's series for the centre deflection of a simply supported a x b plate, w = alpha q / D."""
    s = 0.0
    for mm in range(1, nterm, 2):
        for nn in range(1, nterm, 2):
            s += (-1) ** ((mm + nn) // 2 - 1) / (mm * nn * (mm * mm / a**2 + nn * nn / b**2) ** 2)
    return 16.0 / np.pi**6 * s


def linear_plate_sweep(S, I, torch, n=65):
    """The linear plate benchmark (simply supported, side 8, the benchmark's material and load) for the
    three plate models on the equilateral, regular and irregular (jitter 0.2) meshes of about n vertices a
    side, each one quasi-static solve on the GPU (FP64, PCG rtol 1e-10): centre deflection over Navier's
    value for the plate's sides, and the time."""
    mat = dict(young=2e11, poisson=0.3, thickness=0.01, density=1.0)
    D = mat["young"] * mat["thickness"] ** 3 / (12 * (1 - mat["poisson"] ** 2))
    out = {}
    for mesh_kind in ("equilateral", "regular", "irregular"):
        for model in ("EP", "FP", "SP"):
            if mesh_kind == "equilateral":
                m = I.equilateral_plate(n, 8.0, model)
                b = m.meta["height"]
            else:
                m = I.plate_mesh(n, 8.0, 0.2 if mesh_kind == "irregular" else 0.0, 5, model, "ring")
                b = 8.0
            area = np.zeros(m.nv)
            t = m.tris
            a3 = 0.5 * np.linalg.norm(np.cross(m.X[t[:, 1]] - m.X[t[:, 0]], m.X[t[:, 2]] - m.X[t[:, 0]]), axis=1)
            for c in range(3):
                np.add.at(area, t[:, c], a3 / 3.0)
            load = np.zeros((m.nv, 3))
            load[:, 2] = -9.81 * area
            pb = S.Problem(m, mat, model=model)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            rc, st = S.shell_solve_static(pb.sim, load, eps_f=1e-8 * float(np.linalg.norm(load)), max_newton=2,
                                          pcg_rtol=1e-10)
            torch.cuda.synchronize()
            ms = (time.perf_counter() - t0) * 1e3
            x, _, _ = S.shell_sim_get_state(pb.sim, m.nv)
            pb.close()
            ratio = float(-(x[:, 2] - m.X[:, 2]).min() / (navier_rectangle(8.0, b) * 9.81 / D))
            out[f"{model}_{mesh_kind}"] = dict(nv=m.nv, deflection_ratio=ratio, ms=ms, status=rc)
    print("[bench] linear plate sweep done", file=sys.stderr, flush=True)
    return out


def cantilever_problem(I, model):
    """Sec. 6 cantilever under end shear: a 10 x 1 strip of 17 x 3 vertices (51), E = 1.2e6, nu = 0.1,
    h = 0.1, the two left vertex columns held, F = 4/3 along Z on each of the three right-end vertices."""
    nx, ny = 17, 3
    X = np.zeros((nx * ny, 3))
    for j in range(ny):
        for i in range(nx):
            X[j * nx + i] = (10.0 * i / (nx - 1), 1.0 * j / (ny - 1), 0.0)
    col = np.arange(nx * ny) % nx
    load = np.zeros((nx * ny, 3))
    load[col == nx - 1, 2] = 4.0 / 3.0
    mesh = I.Mesh("cantilever", X, I.grid_tris(nx, ny), (col <= 1).astype(np.uint8), model, 10.0 / (nx - 1), {})
    return mesh, load, col, dict(young=1.2e6, poisson=0.1, thickness=0.1, density=1.0)


def cantilever(S, I, torch):
    """The cantilever with the membrane, quasi-static Newton-Raphson with the paper's eps_f = 1e-3 and
    eps_u = 0.1 (PCG rtol 1e-10) on the GPU: tip deflection along Z, Newton solves, time.  The paper's
    table gives 6.056 (FP), 6.072 (FS), 6.055 (SP), 6.072 (SS) in 67-68 solves; ABAQUS S4R 6.012."""
    out = {}
    for model in ("FP", "FS", "SP", "SS"):
        mesh, load, col, mat = cantilever_problem(I, model)
        pb = S.Problem(mesh, mat, model=model, flags=S.SHELL_FLAG_MEMBRANE)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rc, st = S.shell_solve_static(pb.sim, load, eps_f=1e-3, eps_u=0.1, max_newton=200, pcg_rtol=1e-10)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3
        x, _, _ = S.shell_sim_get_state(pb.sim, mesh.nv)
        pb.close()
        out[model] = dict(w_tip=float((x - mesh.X)[col == 16][:, 2].mean()), newton_iters=st["newton_iters"],
                          pcg_total=st["pcg_total"], ms=ms, residual=st["grad_norm"], status=rc)
    print("[bench] cantilever done", file=sys.stderr, flush=True)
    return out


def cpu_cantilever(I, model="SS"):
    """The oracle's cantilever solve (the smoothed shell)."""
    import oracle as O

    mesh, load, col, mat = cantilever_problem(I, model)
    st = O.Stencils(model, mesh.X, mesh.tris, mat["young"], mat["poisson"], mat["thickness"])
    t0 = time.perf_counter()
    x, _, stats = O.solve_static_membrane(st, mesh.pinned, load, eps_f=1e-3, eps_u=0.1, max_newton=200,
                                          pcg_rtol=1e-10)
    return dict(workload=f"cantilever_{model}", seconds=time.perf_counter() - t0,
                newton_iters=stats["newton_iters"], w_tip=float((x - mesh.X)[col == 16][:, 2].mean()), cores=1)


def cpu_static(I, n=65):
    """The oracle's quasi-static solve of the same clamped plate (one Newton-Raphson solve, PCG rtol 1e-10)."""
    import oracle as O

    m, mat, cl, load = static_plate(I, n)
    st = O.Stencils("SP", m.X, m.tris, mat["young"], mat["poisson"], mat["thickness"], clamped=cl)
    t0 = time.perf_counter()
    _, counts, stats = O.solve_static(st, m.pinned, load, eps_f=1e-8 * float(np.linalg.norm(load)), max_newton=2,
                                      pcg_rtol=1e-10)
    return dict(workload=f"SP_clamped_{n}", seconds=time.perf_counter() - t0, pcg_coord_iters=stats["pcg_total"],
                cores=1)


def run_linear_plate(args):
    """The quasi-static solves alone (the clamped plate at 65^2 and 257^2 and the sweep of the three plate
    models over three meshes), one JSON line; no other kernels run, so a kernel trace of this workload
    shows the quasi-static PCG by itself."""
    import torch

    from paper_2502_10872_amd import inputs as I
    from paper_2502_10872_amd import shell as S

    S.lib()
    qs = quasi_static(S, I, torch)
    sweep = linear_plate_sweep(S, I, torch)
    qs["cantilever"] = cantilever(S, I, torch)
    big = qs["SP_clamped_257"]
    print(json.dumps(dict(metric="linear plate solve time (SP, clamped, 257x257, FP64, PCG rtol 1e-10)",
                          value=big["ms"] / 1e3, unit="s", higher_is_better=False, n_gpus=1, data="synthetic",
                          quasi_static=qs, linear_plate_sweep=sweep)), flush=True)


def run_membrane(args):
    """The membrane alone (its force pass on the 1M-vertex cap, and the step with it on cylinders), one JSON
    line; a kernel trace of this workload shows the membrane kernels by themselves."""
    import torch

    from paper_2502_10872_amd import inputs as I
    from paper_2502_10872_amd import shell as S

    S.lib()
    sizes = tuple(int(n) for n in args.membrane_sizes.split(","))
    forces = membrane_timing(S, I, torch)
    steps = membrane_step_timing(S, I, torch, sizes=sizes)
    mbatch = None if args.no_membrane_batch else membrane_batch_timing(S, I, torch)
    big = max(sizes)
    print(json.dumps(dict(metric=f"implicit steps/s with the membrane (SS, {big}x{big} cylinder, FP64)",
                          value=1e3 / steps[f"SS_membrane_cylinder_{big}"]["ms_per_step"], unit="steps/s",
                          higher_is_better=True, n_gpus=1, data="synthetic", membrane_forces=forces,
                          membrane_step=steps, membrane_batch=mbatch)), flush=True)


def membrane_batch_timing(S, I, torch, count=32, steps=2, warmup=1):
    """A batch of `count` simulations with the membrane (the 64-mesh batch's size and model mix, its
    first `count` specs: 16^2..512^2 vertices, 1 cm spacing, mixed precision, dt = 1/60, Newton budget 4,
    PCG rtol 1e-2), stepped as one batch (one call; the members' steps in flight together on their own
    streams) against the same simulations stepped one at a time."""
    specs = I.batch_specs(64)[:count]
    meshes = [I.mesh_from_spec(sp, spacing=0.01) for sp in specs]
    probs = [S.Problem(m, I.MATERIAL, precision=S.SHELL_PREC_MIXED, flags=S.SHELL_FLAG_MEMBRANE) for m in meshes]
    nv_total = sum(m.nv for m in meshes)
    params, _ = S.step_params(1.0 / 60.0, gravity=I.GRAVITY, max_newton=4, pcg_rtol=1e-2)
    stream = torch.cuda.current_stream()
    batch = S.shell_batch_create([pb.sim for pb in probs])
    for _ in range(warmup):
        S.shell_batch_step(batch, params, len(probs), stream=stream)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    pcg = 0
    for _ in range(steps):
        rc, st = S.shell_batch_step(batch, params, len(probs), stream=stream)
        pcg += sum(x["pcg_total"] for x in st)
    torch.cuda.synchronize()
    batch_s = (time.perf_counter() - t0) / steps
    S.shell_destroy_batch(batch)
    t0 = time.perf_counter()
    for pb in probs:
        for _ in range(steps):
            S.shell_step_implicit(pb.sim, params, stream=stream)
    torch.cuda.synchronize()
    seq_s = (time.perf_counter() - t0) / steps
    for pb in probs:
        pb.close()
    print(f"[bench] membrane batch of {count}: {1e3 * batch_s:.1f} ms per step, one at a time {1e3 * seq_s:.1f} ms",
          file=sys.stderr, flush=True)
    return dict(workload=f"{count} simulations with the membrane, sizes 16^2..512^2 log-uniform (the first {count} "
                         "specs of the 64-mesh batch, seed 2502108724), all six models, 1 cm spacing, mixed, "
                         "dt=1/60 s, Newton budget 4, PCG rtol 0.01",
                meshes=count, vertices=nv_total, steps=steps, mesh_steps_per_s=count / batch_s,
                batch_ms_per_step=1e3 * batch_s, pcg_iters_per_step=pcg / steps,
                one_at_a_time=dict(mesh_steps_per_s=count / seq_s, ms_per_round=1e3 * seq_s),
                speedup_vs_one_at_a_time=seq_s / batch_s)


def batch64_timing(S, I, torch, precision, steps, warmup=1, max_pcg=400000):
    """64 meshes (16^2..512^2 vertices, log-uniform, all six models, 1 cm spacing, Newton budget 4, PCG
    rtol 1e-2, dt = 1/60) stepped as one batch (one launch per phase over all meshes), against the same
    meshes stepped one at a time for the same number of steps."""
    specs = I.batch_specs(64)
    meshes = [I.mesh_from_spec(sp, spacing=0.01) for sp in specs]
    t0 = time.perf_counter()
    probs = [S.Problem(m, I.MATERIAL, precision=precision) for m in meshes]
    setup_s = time.perf_counter() - t0
    nv_total = sum(m.nv for m in meshes)
    params, _ = S.step_params(1.0 / 60.0, gravity=I.GRAVITY, max_newton=4, max_pcg=max_pcg, pcg_rtol=1e-2)
    batch = S.shell_batch_create([pb.sim for pb in probs])
    stream = torch.cuda.current_stream()
    for _ in range(warmup):
        S.shell_batch_step(batch, params, len(probs), stream=stream)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    pcg = 0
    for k in range(steps):
        rc, st = S.shell_batch_step(batch, params, len(probs), stream=stream)
        pcg += sum(x["pcg_total"] for x in st)
        print(f"[bench] batch step {k}", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    batch_s = (time.perf_counter() - t0) / steps
    S.shell_destroy_batch(batch)
    # one mesh at a time, same number of steps per mesh
    t0 = time.perf_counter()
    for pb in probs:
        for _ in range(steps):
            S.shell_step_implicit(pb.sim, params, stream=stream)
    torch.cuda.synchronize()
    seq_s = (time.perf_counter() - t0) / steps
    for pb in probs:
        pb.close()
    print("[bench] batch64 done", file=sys.stderr, flush=True)
    return dict(workload="64-mesh batch, sizes 16^2..512^2 log-uniform (seed 2502108724), all six models, "
                         "1 cm spacing, dt=1/60 s, Newton budget 4, Jacobi-PCG rtol 0.01",
                meshes=len(meshes), vertices=nv_total, steps=steps, warmup=warmup,
                precision="fp64" if precision == S.SHELL_PREC_FP64 else "mixed",
                mesh_steps_per_s=len(meshes) / batch_s, batch_ms_per_step=1e3 * batch_s,
                vertex_steps_per_s=nv_total / batch_s,
                one_at_a_time=dict(mesh_steps_per_s=len(meshes) / seq_s, ms_per_round=1e3 * seq_s),
                speedup_vs_one_at_a_time=seq_s / batch_s, pcg_coord_iters_per_step=pcg / steps, setup_s=setup_s)


def run_batch64(args):
    """The multi-mesh batch as its own workload; prints one JSON line."""
    import torch

    from paper_2502_10872_amd import inputs as I
    from paper_2502_10872_amd import shell as S

    precision = S.SHELL_PREC_MIXED if args.precision == "mixed" else S.SHELL_PREC_FP64
    b = batch64_timing(S, I, torch, precision, args.steps, args.warmup, args.max_pcg)
    out = dict(metric="batched implicit steps/s (64 meshes per step)", value=1e3 / b["batch_ms_per_step"],
               unit="batch steps/s", n_gpus=1, steps=args.steps, warmup=args.warmup,
               ms_per_step=b["batch_ms_per_step"], higher_is_better=True, scaling="weak", vs_baseline=None,
               dtype="f64" if precision == S.SHELL_PREC_FP64 else "f32+f64", data="synthetic",
               config=dict(workload=b["workload"], meshes=b["meshes"], vertices=b["vertices"],
                           precision=args.precision),
               mesh_steps_per_s=b["mesh_steps_per_s"], vertex_steps_per_s=b["vertex_steps_per_s"],
               one_at_a_time=b["one_at_a_time"], speedup_vs_one_at_a_time=b["speedup_vs_one_at_a_time"],
               pcg_coord_iters_per_step=b["pcg_coord_iters_per_step"], setup_s=b["setup_s"])
    print(json.dumps(out), flush=True)


def config_steps(S, torch, mesh, precision, dt, steps, max_newton, newton_rtol, pcg_rtol, max_pcg=400000):
    """`steps` implicit steps from rest, timed end to end (one untimed step first, then the state is reset
    to rest, so the timed trajectory is the one a fresh run takes).  Returns the timing, the iteration
    counts and the final positions."""
    from paper_2502_10872_amd import inputs as I

    pb = S.Problem(mesh, I.MATERIAL, precision=precision)
    params, _ = S.step_params(dt, gravity=I.GRAVITY, max_newton=max_newton, max_pcg=max_pcg,
                              newton_rtol=newton_rtol, pcg_rtol=pcg_rtol)
    S.shell_step_implicit(pb.sim, params)
    S.shell_sim_set_state(pb.sim, mesh.X, None, 0)
    torch.cuda.synchronize()
    stats, lat = [], []
    t_start = time.perf_counter()
    for _ in range(steps):
        t0 = time.perf_counter()
        stats.append(S.shell_step_implicit(pb.sim, params)[1])
        torch.cuda.synchronize()
        lat.append(time.perf_counter() - t0)
    wall = time.perf_counter() - t_start
    x, _, _ = S.shell_sim_get_state(pb.sim, mesh.nv)
    pb.close()
    lat.sort()
    res = dict(steps=steps, steps_per_s=steps / wall, ms_per_step=1e3 * wall / steps,
               p50_ms=1e3 * lat[len(lat) // 2], max_ms=1e3 * lat[-1],
               newton_per_step=sum(st["newton_iters"] for st in stats) / steps,
               pcg_coord_iters_per_step=sum(st["pcg_total"] for st in stats) / steps,
               newton_capped_steps=sum(int(st.get("newton_capped", 0)) for st in stats),
               last_grad_ratio=stats[-1]["grad_norm"] / max(stats[-1]["grad_norm0"], 1e-300))
    return res, x


def small_configs(S, I, torch):
    """The two smaller workloads as full runs of 10 steps: the clamped 32 x 32 edge-hinge plate (FP64, dt =
    1/60, PCG rtol 1e-10) and the 256 x 256 FVM-hinge cylinder patch (FP64 and mixed, dt = 1/30, Newton
    budget 4, PCG rtol 1e-2, the headline step's settings), with the mixed result's distance from the FP64
    one after the 10 steps."""
    out = {}
    plate = I.workload_plate32()
    r, _ = config_steps(S, torch, plate, S.SHELL_PREC_FP64, 1 / 60, 10, 4, 1e-8, 1e-10)
    r["workload"] = "rest-flat 32x32 square plate, EP, FP64, one side clamped, dt=1/60 s, PCG rtol 1e-10"
    r["nv"] = plate.nv
    out["plate32_ep"] = r
    cyl = I.workload_cylinder(256, "FS")
    xs = {}
    for prec, key in ((S.SHELL_PREC_FP64, "fp64"), (S.SHELL_PREC_MIXED, "mixed")):
        r, xs[key] = config_steps(S, torch, cyl, prec, 1 / 30, 10, 4, 1e-8, 1e-2)
        r["workload"] = (f"cylinder patch R=0.5 m, 256x256, jitter 0.2, FVM shell (FS), {key}, pinned ends, "
                         f"dt=1/30 s, Newton budget 4, PCG rtol 1e-2")
        r["nv"] = cyl.nv
        out[f"cylinder256_fs_{key}"] = r
    # The Newton budget ends each step short of convergence (|g|/|g0| stays near 1 against the constant
    # Hessian on this curved patch), so where a run stops depends on its PCG stopping points: the FP64 path
    # run with a 10x tighter inner tolerance gives the spread of the method itself, beside the mixed path's
    # distance from FP64.
    _, x_tight = config_steps(S, torch, cyl, S.SHELL_PREC_FP64, 1 / 30, 10, 4, 1e-8, 1e-3)
    u64 = np.linalg.norm(xs["fp64"] - cyl.X)
    out["cylinder256_fs_mixed"]["displacement_rel_to_fp64"] = float(
        np.linalg.norm(xs["mixed"] - xs["fp64"]) / max(u64, 1e-300))
    out["cylinder256_fs_fp64"]["displacement_rel_fp64_rtol_1e-3_vs_1e-2"] = float(
        np.linalg.norm(x_tight - xs["fp64"]) / max(u64, 1e-300))
    print("[bench] plate32 and cylinder256 done", file=sys.stderr, flush=True)
    return out


# The combined table of Sec. 6 (hemisphere columns): u_min, v_max, Newton iterations and the authors' CPU
# time for the three shell models and the reference shell element; quoted as context, not as a target.
PAPER_HEMISPHERE = {"ES": (-4.072, 2.799, 56, 27.334), "FS": (-5.752, 3.403, 84, 44.153),
                    "SS": (-5.923, 3.534, 87, 45.035), "reference_S4R": (-5.902, 3.406, 112, None)}


def hemisphere_benchmark(S, I, torch):
    """The pinched hemisphere (R = 10, 18 degree hole, four radial point loads of 200 on the equator,
    E = 6.825e7, nu = 0.3, h = 0.04, 17 x 64 = 1088 vertices; x held on the plane x = 0, y on y = 0, z of
    the hole-rim vertices on x = 0): quasi-static Newton-Raphson with the membrane, eps_f = 1e-3,
    eps_u = 0.1, PCG rtol 1e-10, FP64, timed end to end per shell model."""
    out = {}
    for model in ("ES", "FS", "SS"):
        mesh, held, F, _ = I.hemisphere_problem(17, 64, model=model)
        with S.Problem(mesh, I.HEMISPHERE_MATERIAL, model=model, flags=S.SHELL_FLAG_MEMBRANE, held=held) as pb:
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            rc, st = S.shell_solve_static(pb.sim, F, eps_f=1e-3, eps_u=0.1, max_newton=250, pcg_rtol=1e-10)
            torch.cuda.synchronize()
            sec = time.perf_counter() - t0
            x, _, _ = S.shell_sim_get_state(pb.sim, mesh.nv)
        u = x - mesh.X
        pu, pv, pn, pt = PAPER_HEMISPHERE[model]
        pcg = int(np.asarray(st["counts"])[: st["newton_iters"], 0].sum())
        out[model] = dict(nv=mesh.nv, newton_iters=st["newton_iters"], pcg_iters=pcg, seconds=sec,
                          us_per_pcg_iteration=1e6 * sec / max(pcg, 1), residual=st["grad_norm"], status=rc,
                          u_min=float(u[:, 0].min()), v_max=float(u[:, 1].max()),
                          paper=dict(u_min=pu, v_max=pv, newton_iters=pn, seconds_on_the_authors_cpu=pt))
        print(f"[bench] hemisphere {model}: newton {st['newton_iters']} u_min {u[:, 0].min():.3f} "
              f"v_max {u[:, 1].max():.3f} {sec:.2f} s", file=sys.stderr, flush=True)
    out["reference_S4R"] = dict(zip(("u_min", "v_max", "newton_iters"), PAPER_HEMISPHERE["reference_S4R"][:3]))
    return out


def serving_run(torch, rates=(20.0, 200.0), durations=(3.0, 1.0), max_wait_s=5.0):
    """The serving loop on short Poisson traces (10 steps per request, 2k..1M vertices log-normal, the six
    models, mixed precision, 16 GB HBM budget): continuous batching against one mesh at a time on the
    same trace.  A request that has waited longer than max_wait_s for admission is shed (rejected)."""
    from paper_2502_10872_amd import serve

    out = {}
    for rate, dur in zip(rates, durations):
        for mode in ("continuous", "one_at_a_time"):
            cfg = serve.ServeConfig(max_wait_s=max_wait_s)
            reqs = serve.make_requests(rate, dur)
            if mode == "continuous":
                res = serve.Server(serve.GpuExecutor(cfg), cfg).run(reqs)
            else:
                res = serve.run_sequential(serve.GpuExecutor(cfg), cfg, reqs)
            torch.cuda.synchronize()
            res.update(rate=rate, trace_s=dur, max_wait_s=max_wait_s)
            out[f"rate{int(rate)}_{mode}"] = res
            print(f"[bench] serving rate {rate:g} {mode}: {res['completed']}/{res['requests']} done, {res['shed']} shed, "
                  f"{res['failed']} failed, p99 {res['p99_s']:.2f} s", file=sys.stderr, flush=True)
    return out


def timed_steps(S, torch, pb, params, steps, sample_every, label):
    """`steps` implicit steps on the library's stream; wall time bracketed by stream synchronisation and
    kernel durations sampled in-step with HIP events (see shell_sim_profile)."""
    stream = torch.cuda.current_stream()
    torch.cuda.synchronize()
    S.shell_sim_profile(pb.sim, sample_every)
    stats, lat = [], []
    t_start = time.perf_counter()
    for k in range(steps):
        t0 = time.perf_counter()
        rc, st = S.shell_step_implicit(pb.sim, params, stream=stream)
        torch.cuda.synchronize()
        lat.append(time.perf_counter() - t0)
        stats.append(st)
        print(f"[bench] {label} step {k}: newton {st['newton_iters']} pcg {st['pcg_total']} "
              f"|g|/|g0| {st['grad_norm'] / max(st['grad_norm0'], 1e-300):.3e} {lat[-1]:.2f} s",
              file=sys.stderr, flush=True)
    elapsed = time.perf_counter() - t_start
    prof = S.shell_sim_profile_read(pb.sim)
    S.shell_sim_profile(pb.sim, 0)
    return elapsed, stats, lat, prof


def step_error(S, torch, mesh, pb64, pbm, params, steps, short_iters=200):
    """Displacement error of the mixed path against FP64 from the same state, per step, next to the FP64
    path's own run-to-run difference.

    full:  from the state the FP64 trajectory reached, the FP64 path steps in tolerance mode; then the
           FP64 path again and the mixed path, both from that same state, replay its Newton and PCG
           counts.  The FP64 step is bitwise reproducible, so the rerun lands on the same bits; thousands
           of Krylov iterations stopped at a 1e-2 residual amplify the mixed path's rounding into a
           different inexact step of the same residual tolerance.
    short: one Newton iteration with `short_iters` replayed PCG iterations per coordinate from the same
           state, where the difference is the precision alone.
    converged: one Newton iteration from rest with both solves run to PCG rtol 1e-10 (the mixed one with
           its residual-replacement passes), the two precisions at a matched residual."""
    zero = np.zeros_like(mesh.X)

    def rel_disp(x, ref, x0):
        return float(np.linalg.norm(x - ref) / max(np.linalg.norm(ref - x0), 1e-300))

    S.shell_sim_set_state(pb64.sim, mesh.X, zero, 0)
    full, rerun = [], []
    for k in range(steps):
        x0, v0, s0 = S.shell_sim_get_state(pb64.sim, mesh.nv)
        rc, st = S.shell_step_implicit(pb64.sim, params)
        x64, v64, s64 = S.shell_sim_get_state(pb64.sim, mesh.nv)
        counts = st["counts"][: st["newton_iters"]]
        rp, _keep = S.step_params(params.dt, gravity=tuple(params.gravity), max_newton=st["newton_iters"],
                                  replay=counts)
        S.shell_sim_set_state(pb64.sim, x0, v0, s0)
        S.shell_step_implicit(pb64.sim, rp)
        x64b, _, _ = S.shell_sim_get_state(pb64.sim, mesh.nv)
        S.shell_sim_set_state(pbm.sim, x0, v0, s0)
        S.shell_step_implicit(pbm.sim, rp)
        xm, _, _ = S.shell_sim_get_state(pbm.sim, mesh.nv)
        full.append(rel_disp(xm, x64, x0))
        rerun.append(rel_disp(x64b, x64, x0))
        S.shell_sim_set_state(pb64.sim, x64, v64, s64)
    short, short_rerun = [], []
    rp, _keep = S.step_params(params.dt, gravity=tuple(params.gravity), max_newton=1,
                              replay=np.full((1, 3), short_iters, np.int32))
    for k in range(steps):
        x0, v0, s0 = S.shell_sim_get_state(pb64.sim, mesh.nv)
        S.shell_step_implicit(pb64.sim, rp)
        x64, v64, s64 = S.shell_sim_get_state(pb64.sim, mesh.nv)
        S.shell_sim_set_state(pb64.sim, x0, v0, s0)
        S.shell_step_implicit(pb64.sim, rp)
        x64b, _, _ = S.shell_sim_get_state(pb64.sim, mesh.nv)
        S.shell_sim_set_state(pbm.sim, x0, v0, s0)
        S.shell_step_implicit(pbm.sim, rp)
        xm, _, _ = S.shell_sim_get_state(pbm.sim, mesh.nv)
        short.append(rel_disp(xm, x64, x0))
        short_rerun.append(rel_disp(x64b, x64, x0))
        S.shell_sim_set_state(pb64.sim, x64, v64, s64)
    cp, _keep = S.step_params(params.dt, gravity=tuple(params.gravity), max_newton=1, newton_rtol=0.0,
                              pcg_rtol=1e-10)
    conv_pcg = {}
    for name, pb in (("fp64", pb64), ("mixed", pbm)):
        S.shell_sim_set_state(pb.sim, mesh.X, zero, 0)
        rc, st = S.shell_step_implicit(pb.sim, cp)
        conv_pcg[name] = int(st["pcg_total"])
    x64, _, _ = S.shell_sim_get_state(pb64.sim, mesh.nv)
    xm, _, _ = S.shell_sim_get_state(pbm.sim, mesh.nv)
    conv = rel_disp(xm, x64, mesh.X)
    print(f"[bench] mixed vs fp64 displacement error per step: full {full} (fp64 rerun {rerun}), short {short} "
          f"(fp64 rerun {short_rerun}); one converged Newton iteration {conv:.2e} (PCG {conv_pcg})",
          file=sys.stderr, flush=True)
    return dict(full_step_replayed_counts=full, full_step_fp64_rerun=rerun, one_newton_200_pcg=short,
                one_newton_200_pcg_fp64_rerun=short_rerun, one_newton_converged=conv,
                one_newton_converged_pcg_coord_iters=conv_pcg)


def stream_copy_gbs(torch):
    """Read + write bandwidth of a plain elementwise kernel over 1 GiB (the practical streaming ceiling)."""
    a = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        torch.mul(a, 1.0, out=b)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(10):
        torch.mul(a, 1.0, out=b)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / 10
    del a, b
    return 2 * (1 << 30) / (ms * 1e-3) / 1e9


def force_models(S, I, torch, precisions, reps=20):
    """Force kernel of every model on a 1024 x 1024 mesh (shells: the sphere cap; plates: a flat square
    of the same side), launched back to back on one state (shell_sim_time_kernels); QTS is the edge shell
    with the world-frame operator (App. D) on the cap; EP_clamped and SP_clamped are the plates with every
    boundary edge clamped (eqs 30-31, 59)."""
    out = {}
    cap = I.workload_sphere_cap(1024, "SS")
    side = cap.meta.get("side", 1.2 * cap.meta["radius"])
    for name in list(I.MODELS) + ["QTS", "EP_clamped", "SP_clamped"]:
        model = {"QTS": "ES"}.get(name, name.split("_")[0])
        flags = S.SHELL_FLAG_WORLD_FRAME if name == "QTS" else 0
        if model.endswith("S"):
            mesh = I.workload_sphere_cap(1024, model)
        else:
            mesh = I.plate_mesh(1024, side, 0.2, 2502108723, model, "ring")
        clamped = I.boundary_edges(mesh.tris) if name.endswith("_clamped") else None
        for prec in precisions:
            pb = S.Problem(mesh, I.MATERIAL, model=model, precision=prec, flags=flags, clamped_edges=clamped)
            kt = S.shell_sim_time_kernels(pb.sim, 1.0 / 30.0, reps=reps)
            hinfo = S.shell_hessian_info(pb.h)
            ab = algorithmic_bytes(pb.info, hinfo, prec, clamp_bias=clamped is not None)
            ms = kt["force_ms"]
            out[f"{name}_{'mixed' if prec == S.SHELL_PREC_MIXED else 'fp64'}"] = dict(
                stencils=pb.info["ns"], force_ms=ms, stencils_per_s=pb.info["ns"] / (ms * 1e-3),
                gbs=ab["force"] / (ms * 1e-3) / 1e9, frac=ab["force"] / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS)
            pb.close()
        print(f"[bench] force timing {name} done", file=sys.stderr, flush=True)
    return out


def force_error(S, torch, mesh, pb64, pbm):
    """Relative force error of the mixed path against FP64, at two states: the mixed simulation's current
    state, and a fixed one (the rest shape plus the smooth field u = a (sin kx cos ky, cos kx sin ky,
    sin kx sin ky), k = 2 pi / side, a = side / 100).  The mixed path rounds the curvature C = B x to
    float32 with an error proportional to |B||x_j - x_o|, while the force is proportional to the bending
    strain C n - kappa0, so the relative error grows as the state approaches the rest shape; the fixed
    state makes the figure comparable between runs."""
    x, _, _ = S.shell_sim_get_state(pbm.sim, mesh.nv)
    X = mesh.X
    side = float(X[:, 0].max() - X[:, 0].min())
    k, a = 2.0 * np.pi / side, side / 100.0
    sx, cx = np.sin(k * X[:, 0]), np.cos(k * X[:, 0])
    sy, cy = np.sin(k * X[:, 1]), np.cos(k * X[:, 1])
    fixed = X + a * np.stack([sx * cy, cx * sy, sx * sy], axis=1)
    out = {}
    for name, state in (("trajectory_state", x), ("fixed_state", fixed)):
        xd = torch.tensor(state, device="cuda")
        f64 = torch.zeros_like(xd)
        f32 = torch.zeros(xd.shape, dtype=torch.float32, device="cuda")
        S.shell_eval_forces(pb64.st, xd, f64, None)
        S.shell_eval_forces(pbm.st, xd, f32, None)
        torch.cuda.synchronize()
        out[name] = float(torch.linalg.norm(f32.double() - f64) / torch.linalg.norm(f64))
    return out


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=6,
                    help="timed steps (the PCG iteration count per step varies by tens of percent along the "
                         "trajectory, so several steps are averaged)")
    ap.add_argument("--error-steps", type=int, default=2, help="steps of the mixed-vs-FP64 error runs")
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--size", type=int, default=1024)
    ap.add_argument("--precision", choices=("fp64", "mixed"), default="mixed",
                    help="the path whose steps/s is the headline value")
    ap.add_argument("--no-compare", action="store_true",
                    help="skip the other precision's timed steps and the per-step error run")
    ap.add_argument("--max-newton", type=int, default=4)
    ap.add_argument("--pcg-rtol", type=float, default=1e-2)
    ap.add_argument("--reps", type=int, default=20, help="launches per kernel of the isolated back-to-back timing")
    ap.add_argument("--sample-every", type=int, default=17,
                    help="in the timed steps, time every n-th PCG iteration's kernels with HIP events (17: prime "
                         "to the 16-iteration period of the mixed update's fold, so every phase of it is sampled)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--hot-path-only", action="store_true",
                    help="skip the quasi-static solves and the membrane (their launches are kept out of the "
                         "counter and trace profiles of the hot path)")
    ap.add_argument("--max-pcg", type=int, default=400000, help="PCG iteration cap per coordinate solve")
    ap.add_argument("--workload", choices=("sphere-cap", "batch64", "linear-plate", "membrane"), default="sphere-cap")
    ap.add_argument("--membrane-sizes", default="64,256,1024",
                    help="membrane workload: cylinder sizes n (n x n vertices) of the step timing")
    ap.add_argument("--no-membrane-batch", action="store_true", help="membrane workload: skip the batch timing")
    ap.add_argument("--no-force-models", action="store_true",
                    help="skip the per-model force kernel timing (six 1M-vertex meshes, both precisions)")
    ap.add_argument("--no-other-workloads", action="store_true",
                    help="skip the 10-step plate and cylinder runs, the 64-mesh batch and the serving traces")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run a plain 512 MiB read + 512 MiB write elementwise kernel (counter calibration)")
    args = ap.parse_args(argv)
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the path is single-device by design",
              file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2502_10872_amd import inputs as I
    from paper_2502_10872_amd import shell as S

    assert torch.cuda.is_available(), "needs a HIP device"
    torch.cuda.set_device(0)
    if args.workload == "batch64":
        return run_batch64(args)
    if args.workload == "linear-plate":
        return run_linear_plate(args)
    if args.workload == "membrane":
        return run_membrane(args)
    head = S.SHELL_PREC_MIXED if args.precision == "mixed" else S.SHELL_PREC_FP64
    other = S.SHELL_PREC_FP64 if head == S.SHELL_PREC_MIXED else S.SHELL_PREC_MIXED
    mat = I.MATERIAL
    mesh = I.workload_sphere_cap(args.size, "SS")
    print(f"[bench] building {mesh.nv} vertices, SS, {args.precision}", file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    pb = S.Problem(mesh, mat, precision=head)
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    pb_other = None if args.no_compare else S.Problem(mesh, mat, precision=other)
    hinfo = S.shell_hessian_info(pb.h)
    dt = 1.0 / 30.0
    params, _ = S.step_params(dt, gravity=I.GRAVITY, max_newton=args.max_newton, max_pcg=args.max_pcg,
                              newton_rtol=1e-8, pcg_rtol=args.pcg_rtol)
    for w in range(args.warmup):
        for q in (pb, pb_other):
            if q is not None:
                rc, st = S.shell_step_implicit(q.sim, params)
                print(f"[bench] warmup {w}: newton {st['newton_iters']} pcg {st['pcg_total']}", file=sys.stderr,
                      flush=True)
    elapsed, stats, lat, prof = timed_steps(S, torch, pb, params, args.steps, args.sample_every, args.precision)
    steps_per_s = args.steps / elapsed
    compare = None
    if pb_other is not None:
        e2, st2, lat2, prof2 = timed_steps(S, torch, pb_other, params, args.steps, args.sample_every,
                                           "fp64" if other == S.SHELL_PREC_FP64 else "mixed")
        pb64, pbm = (pb_other, pb) if head == S.SHELL_PREC_MIXED else (pb, pb_other)
        ferr = force_error(S, torch, mesh, pb64, pbm)
        errs = step_error(S, torch, mesh, pb64, pbm, params, args.error_steps)
        errs["force_rel_err"] = ferr["trajectory_state"]
        errs["force_rel_err_fixed_state"] = ferr["fixed_state"]
        compare = dict(precision="fp64" if other == S.SHELL_PREC_FP64 else "mixed", steps_per_s=args.steps / e2,
                       ms_per_step=1e3 * e2 / args.steps,
                       pcg_coord_iters=float(np.mean([s["pcg_total"] for s in st2])),
                       product_ms=prof2["product"]["avg_ms"], update_ms=prof2["update"]["avg_ms"],
                       grad_ratio=[x["grad_norm"] / max(x["grad_norm0"], 1e-300) for x in st2],
                       mixed_vs_fp64_displacement_rel_err=errs)

    # the same kernels launched back to back on one state (their working set then partly stays in the
    # 256 MB last-level cache, so these read faster than the in-step figures; reported for reference)
    stream = torch.cuda.current_stream()
    kt = S.shell_sim_time_kernels(pb.sim, dt, reps=args.reps, stream=stream)
    if args.calibrate_copy:
        a = torch.ones(1 << 27, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            torch.mul(a, 1.0, out=b)
        torch.cuda.synchronize()
        del a, b
    ab = algorithmic_bytes(pb.info, hinfo, head)

    def rate(nbytes, ms):
        return nbytes / (ms * 1e-3) / 1e9 if ms else None

    spmv_ms = prof["product"]["avg_ms"]
    update_ms = prof["update"]["avg_ms"]
    force_ms = prof["forces"]["avg_ms"]
    spmv_gbs = rate(ab["spmv"], spmv_ms)
    update_gbs = rate(ab["update"], update_ms)
    force_gbs = rate(ab["force"], force_ms)
    stencils_per_s = pb.info["ns"] / (force_ms * 1e-3) if force_ms else None
    key = "mixed" if head == S.SHELL_PREC_MIXED else "fp64"
    default_workload = args.size == 1024
    traffic_spmv = measured_traffic(f"{key}_spmv_traffic_bytes_per_launch") if default_workload else None
    traffic_update = measured_traffic(f"{key}_update_traffic_bytes_per_launch") if default_workload else None
    traffic_force = measured_traffic(f"{key}_force_traffic_bytes_per_launch") if default_workload else None
    pcg_per_step = float(np.mean([s["pcg_total"] for s in stats]))
    # shared iterations (the three coordinate recurrences share each launch): the longest per Newton solve
    pcg_iters = float(np.mean([sum(int(c.max()) for c in s["counts"]) for s in stats]))
    newton_per_step = float(np.mean([s["newton_iters"] for s in stats]))
    lat_sorted = sorted(lat)

    out = dict(
        metric="implicit steps/s & bending stencils/s at 1M verts vs HBM roofline; p50/p99 latency",
        value=steps_per_s, unit="steps/s", n_gpus=1, steps=args.steps, warmup=args.warmup,
        ms_per_step=1e3 * elapsed / args.steps, higher_is_better=True, scaling="weak", vs_baseline=None,
        dtype="f64" if head == S.SHELL_PREC_FP64 else "f32+f64", data="synthetic",
        config=dict(workload=f"sphere-cap smoothed-hinge shell (SS), {args.size}x{args.size} vertices, "
                             f"R={mesh.meta['radius']:.4f} m, jitter 0.2, ring pinned, dt=1/30 s, "
                             f"Newton budget {args.max_newton}, Jacobi-PCG rtol {args.pcg_rtol:g}",
                    nv=mesh.nv, stencils=pb.info["ns"], nnz=hinfo["nnz"], precision=args.precision,
                    parallelism="single GPU"),
        roofline=dict(bound="hbm", kernel="k_pcg_spmv (PCG state, direction update, 3-column SELL-64 product)",
                      achieved=spmv_gbs, peak=HBM_PEAK_GBS, unit="GB/s",
                      frac=spmv_gbs / HBM_PEAK_GBS if spmv_gbs else None, traffic=traffic_spmv,
                      bytes_per_launch=ab["spmv"], avg_ms=spmv_ms, sampled_launches=prof["product"]["count"]),
        update_kernel=dict(kernel="k_pcg_update", achieved_gbs=update_gbs,
                           frac=update_gbs / HBM_PEAK_GBS if update_gbs else None, bytes_per_launch=ab["update"],
                           avg_ms=update_ms, traffic=traffic_update),
        force_kernel=dict(kernel="force_tiles", stencils_per_s=stencils_per_s, achieved_gbs=force_gbs,
                          frac=force_gbs / HBM_PEAK_GBS if force_gbs else None, bytes_per_launch=ab["force"],
                          bytes_per_stencil_stream=ab["force_per_stencil"], avg_ms=force_ms, traffic=traffic_force,
                          sampled_launches=prof["forces"]["count"]),
        latency_s=dict(per_step=lat, p50=lat_sorted[len(lat) // 2], p99=lat_sorted[min(len(lat) - 1,
                                                                                       int(0.99 * len(lat)))]),
        pcg=dict(coord_iters_per_step=pcg_per_step, iterations_per_step=pcg_iters,
                 ms_per_iteration_in_step=1e3 * elapsed / max(pcg_iters * args.steps, 1.0)),
        compare=compare,
        isolated_back_to_back_ms=dict(force=kt["force_ms"], product=kt["spmv_ms"], update=kt["update_ms"]),
        hessian=dict(nnz=hinfo["nnz"], slots=hinfo["slots"], group_cols=hinfo["group_cols"],
                     max_group_cols=hinfo["max_group_cols"], staged=bool(hinfo["staged"])),
        per_step=dict(newton_iters=newton_per_step, pcg_coord_iters=pcg_per_step,
                      grad_ratio=[s["grad_norm"] / max(s["grad_norm0"], 1e-300) for s in stats]),
        setup_s=setup_s,
        tiles=dict(block_vertices=pb.info["block_vertices"], nblocks=pb.info["nblocks"],
                   halo_factor=pb.info["ns_tiled"] / max(pb.info["ns"], 1)),
    )
    out["roofline"]["stream_copy_gbs"] = stream_copy_gbs(torch)
    pb.close()
    if pb_other is not None:
        pb_other.close()
    if not args.no_force_models and args.size == 1024:
        out["force_models_isolated"] = force_models(S, I, torch, (S.SHELL_PREC_MIXED, S.SHELL_PREC_FP64))
        if not args.hot_path_only:
            out["membrane_forces"] = membrane_timing(S, I, torch)
            out["membrane_step"] = membrane_step_timing(S, I, torch)
            out["membrane_batch"] = membrane_batch_timing(S, I, torch)
            out["quasi_static"] = quasi_static(S, I, torch)
            out["quasi_static"]["linear_plate_sweep"] = linear_plate_sweep(S, I, torch)
            out["quasi_static"]["cantilever"] = cantilever(S, I, torch)
            out["quasi_static"]["hemisphere"] = hemisphere_benchmark(S, I, torch)
    if not args.no_other_workloads and not args.hot_path_only and args.size == 1024:
        out["other_workloads"] = small_configs(S, I, torch)
        out["other_workloads"]["batch64"] = batch64_timing(S, I, torch, S.SHELL_PREC_MIXED, steps=3, warmup=1)
        out["other_workloads"]["serving"] = serving_run(torch)
    if not args.no_cpu_baseline and args.size == 1024:
        print("[bench] timing the CPU oracle sample", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(mesh, mat, pcg_per_step, newton_per_step)
        if not args.hot_path_only:
            out["cpu_baseline"]["quasi_static"] = cpu_static(I)
            out["cpu_baseline"]["membrane_step"] = cpu_membrane_step(I)
            out["cpu_baseline"]["cantilever"] = cpu_cantilever(I)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
