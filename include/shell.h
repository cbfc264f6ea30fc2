/*
 * shell.h - C ABI of the MI355X (gfx950) library for the per-timestep hot path
 * of the corotational hinge-based thin plate/shell bending models
 * ("Corotational Hinge-based Thin Plates/Shells"):
 *
 *   EP, ES  edge-based hinge, plate / shell      (Sec. 4.3, eqs 4-29)
 *   FP, FS  FVM hinge, plate / shell             (Sec. 4.4, eqs 32-45, App. C)
 *   SP, SS  smoothed hinge, plate / shell        (Sec. 4.5, eqs 46-61)
 *
 * and the implicit-Euler step against their constant bending Hessian
 * (Sec. 5, eqs 62-63; constant Hessians eqs 21, 41, 53).
 *
 * Conventions for every entry point:
 *  - Return value: SHELL_OK (0) or a shell_status_t error; no C++ exception
 *    crosses the ABI.  shell_last_error() gives a thread-local message.
 *  - "host" pointers are read (or written) before the call returns; "device"
 *    pointers are HIP device memory, read/written asynchronously on `stream`
 *    and must stay valid until the stream reaches the work.
 *  - `stream` is a hipStream_t; NULL selects the null stream.
 *  - Vertex arrays are [nv][3] row-major float64 in the caller's vertex order.
 *    The library keeps its own order internally (by default recursive
 *    coordinate bisection into compact tiles, Morton order inside a tile; see
 *    shell_config_t.reorder) and converts at the boundary.
 *  - Handles are owned by the library and released by shell_destroy_*; one
 *    handle must not be used by two threads at once.  Distinct handles may be
 *    driven from distinct threads.  Steps capture their PCG iterations into HIP
 *    graphs, and the runtime refuses some calls made by another thread during a
 *    capture (a device-wide synchronisation is one), invalidating the capture.
 *    The library never synchronises the whole device, and its allocations,
 *    releases, stream creation and captures take one process-wide lock.  A
 *    caller's own such call from another thread, made during a step, can still
 *    fail that step with SHELL_E_HIP; SHELL_STEP_NO_GRAPHS steps without
 *    captures.
 *  - Models are identified by shell_model_t; a model's curvature size r is 1
 *    (edge) or 3 (triangle), its stencil size k is 4 (edge) or 6 (triangle).
 */
#ifndef SHELL_H
#define SHELL_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    SHELL_OK = 0,
    SHELL_E_INVALID_ARG = 1,  /* a null pointer, a size out of range, an unknown model */
    SHELL_E_NONMANIFOLD = 2,  /* an edge shared by more than two triangles */
    SHELL_E_ORIENTATION = 3,  /* two triangles traverse a shared edge in the same direction */
    SHELL_E_DEGENERATE = 4,   /* a zero-area triangle, a zero height, or an ill-conditioned fit */
    SHELL_E_NONFINITE = 5,    /* a NaN/Inf in a state or residual */
    SHELL_E_BUDGET = 6,       /* PCG budget exhausted before the tolerance; state advanced, stats filled */
    SHELL_E_OOM = 7,          /* device or host allocation failed */
    SHELL_E_HIP = 8,          /* a HIP runtime call failed */
    SHELL_E_UNSUPPORTED = 9   /* a valid request this library does not implement */
} shell_status_t;

typedef enum { SHELL_EP = 0, SHELL_ES = 1, SHELL_FP = 2, SHELL_FS = 3, SHELL_SP = 4, SHELL_SS = 5 } shell_model_t;

typedef enum {
    SHELL_PREC_FP64 = 0,  /* all arithmetic in float64 */
    SHELL_PREC_MIXED = 1  /* float32 operators, stencil forces, SpMV and Jacobi preconditioner on float64
                             stencil-local differences; float64 dot products, solution/residual updates,
                             Newton residual and all rest precomputation */
} shell_precision_t;

/* Material (Sec. 3, eq 1; bending rigidity k_b = E h^3 / (12 (1 - nu^2)), Sec. 4.3). */
typedef struct {
    double young;      /* E [Pa] */
    double poisson;    /* nu, in (-1, 0.5] */
    double thickness;  /* h [m] */
    double density;    /* rho [kg/m^3], used for the lumped mass rho h A/3 */
} shell_material_t;

typedef struct {
    int32_t precision;       /* shell_precision_t */
    int32_t block_vertices;  /* vertices per force work-group tile, 64..4096; 0 selects the default (2048) */
    int32_t reorder;         /* internal vertex order: 1 (default) recursive coordinate bisection into compact
                                tiles of block_vertices, 2 Morton order, 0 the caller's order */
    int32_t flags;           /* 0, or SHELL_FLAG_DIRECT_PRODUCT, SHELL_FLAG_WORLD_FRAME, SHELL_FLAG_MEMBRANE */
} shell_config_t;

/* The PCG product gathers each neighbour's entries straight from memory instead of staging every 512-row
 * group's distinct columns in LDS.  Chosen by itself when a group has more than 4096 distinct columns;
 * the flag forces it (to compare the two forms). */
#define SHELL_FLAG_DIRECT_PRODUCT 1

/* Edge models only (EP, ES): the quadratic thin plate/shell variant of App. D (eq 79), whose curvature
 * operator L_n takes the heights and the feet on the hinge of the rest stencil as it lies in the world
 * frame instead of on its projection onto the tangent plane (for a rest dihedral phi0, L_n = cos^2(phi0/2)
 * L_m; identical on a flat rest).  The force and step kernels are those of EP and ES.  With a triangle
 * model the build returns SHELL_E_INVALID_ARG. */
#define SHELL_FLAG_WORLD_FRAME 2

/* Adds the membrane of Sec. 3 (eq 1): constant strain triangles with the Saint Venant-Kirchhoff model,
 * D_m = h E_el (plane stress), energy A/2 eps^T D_m eps of the Green strain per triangle, on every
 * triangle of the mesh and for any model.  shell_eval_forces adds its force and energy (both precisions).
 * The implicit step takes it one simulation at a time, in either precision: each Newton iteration assembles the
 * membrane tangent K_m into 3x3 blocks (per triangle the Gauss-Newton part A B(F)^T D_m B(F) plus the
 * stress part A (g_a^T S+ g_b) I3, S+ the positive semi-definite part of the 2x2 second Piola-Kirchhoff
 * stress and g the shape-function gradients: the exact Hessian under tension, the Gauss-Newton tangent
 * under compression, positive semi-definite always), solves (M + dt^2 (K_s (x) I3 + K_m)) y = -g by one
 * Jacobi-PCG over all coordinates (the membrane couples them; 1/(m + dt^2 (K_s,ii + tr(K_m,ii)/3)) per
 * vertex), then backtracks x += 2^-h y,
 * h the fewest halvings (at most 6) that satisfy Armijo's condition E(x + a y) <= E(x) + 1e-4 a g.y on
 * the incremental potential.  In its step statistics counts[k][0] is the PCG count and counts[k][1] the
 * halvings of Newton iteration k; REPLAY takes both from replay_counts the same way.  The quasi-static
 * solve takes it the same way (no mass term, no line search: eq 64's eps_u scaling; counts[k][0]).
 * In mixed precision the bending and membrane forces are the float32 kernels' (widened to float64 for the
 * Newton loop), and the product reads float32 copies of K_s and of the tangent's blocks in difference
 * form, q_i = m_i p_i + dt^2 sum_j (K_s,ij I + K_m,ij)(p_j - p_i), which keeps translations in their null
 * space whatever the rounding; the vectors, dot products and the Newton loop stay float64.  On meshes of
 * 32768 vertices or more, unless SHELL_FLAG_DIRECT_PRODUCT is set, the product takes the rows in groups
 * of 128, 256 or 512 (at least 256 groups where possible) with the group's directions staged in LDS, K_s
 * from the bending Hessian's SELL-64 slots and the blocks in SELL-64 slices; smaller meshes read both as
 * CSR.
 * A batch of such simulations steps each member as it would step alone (see shell_batch_create).  A
 * degenerate triangle is SHELL_E_DEGENERATE. */
#define SHELL_FLAG_MEMBRANE 4

typedef struct shell_stencils_s* shell_stencils_t;
typedef struct shell_hessian_s* shell_hessian_t;
typedef struct shell_sim_s* shell_sim_t;
typedef struct shell_batch_s* shell_batch_t;
typedef void* shell_stream_t; /* hipStream_t */

/*
 * shell_build_stencils - topology and rest precomputation of one mesh for one model.
 *
 * X     host [nv][3] rest positions (Sec. 4.1, x = X + u).
 * tris  host [nt][3] vertex ids of a consistently oriented 2-manifold triangle mesh, boundary allowed.
 * Edge models get one stencil (1,2,3,4) per interior edge (Sec. 4.3, Fig. of the edge hinge);
 * triangle models one stencil (1,...,6) per triangle, flap i+3 across the edge opposite vertex i
 * (Secs 4.4-4.5, App. C).  Boundary edges are free (Sec. 4.3: no energy; Secs 4.4-4.5: virtual
 * node reflected through the edge midpoint and folded, eq 61; FVM additionally drops the twist
 * across the free edge).  The rest operators (eqs 10, 37-38, 50, App. C eqs 76-78), rest curvature
 * (eqs 14, 43, 51; shells only) and stencil areas are computed on the GPU in float64.
 * clamped_edges  host [n_clamped][2] vertex pairs (either order) of boundary edges with the clamped
 *                condition (eqs 30-31, 59), or NULL with n_clamped = 0; any pair that is not an edge of
 *                exactly one triangle is SHELL_E_INVALID_ARG.  The virtual node moves with the vertex it
 *                mirrors, so its operator column is added to that vertex's.  Edge plate (EP): one extra
 *                stencil (L, M, N, L') per clamped edge, weighted by its one real triangle's area; the
 *                edge shell (ES) gets none (along its own triangle's normal the folded stencil has no
 *                transverse displacement, so its energy vanishes identically).  Triangle models: the
 *                missing flap is folded onto L; FVM keeps the twist across a clamped edge.  Plates
 *                measure the curvature of a stencil with a clamped edge from the rest shape,
 *                C = B (x - X), since the clamped fold does not annihilate the flat rest coordinates.
 *                In the shell forms the clamped and free folds give the same curvature change (the
 *                central triangle's vertices have no transverse displacement in the stencil frame);
 *                only K_s and FVM's twist differ.  A shell edge is held by fixing its vertex rows.
 * Errors: SHELL_E_INVALID_ARG, SHELL_E_NONMANIFOLD, SHELL_E_ORIENTATION, SHELL_E_DEGENERATE,
 * SHELL_E_OOM, SHELL_E_HIP.  The call synchronises `stream` before returning.
 */
shell_status_t shell_build_stencils(const double* X, int64_t nv, const int32_t* tris, int64_t nt, int32_t model,
                                    const shell_material_t* mat, const int32_t* clamped_edges, int64_t n_clamped,
                                    const shell_config_t* cfg, shell_stream_t stream, shell_stencils_t* out);

typedef struct {
    int64_t nv, nt;
    int64_t ns;             /* unique stencils */
    int64_t ns_tiled;       /* stencil copies in the tiled force layout (halo stencils repeat) */
    int64_t nblocks;        /* force work-group tiles */
    int32_t model, k, r, precision;
    int32_t block_vertices;
    int32_t reserved;
} shell_stencils_info_t;

shell_status_t shell_stencils_info(shell_stencils_t st, shell_stencils_info_t* info);

/*
 * shell_stencils_export - host copies of the per-stencil rest data, for inspection and tests.
 * idx     host [ns][k] vertex ids in the caller's order, -1 for a missing flap (may be NULL).
 * B       host [ns][r][k] operator scaled by the square root of the stencil's stiffness:
 *         edge sqrt(k_b A_E) L_m, triangle sqrt(A) R L_p (FVM) or sqrt(A) L_g (smoothed), free folds
 *         applied (may be NULL).
 * kappa0  host [ns][r] rest curvature scaled the same way; zero for plates (may be NULL).
 * Stencils come in the library's internal order; match them by idx.
 */
shell_status_t shell_stencils_export(shell_stencils_t st, int32_t* idx, double* B, double* kappa0);

/*
 * shell_eval_forces - bending force f = -dPsi/dx of all stencils at positions x.
 * Plates: f = -(K_s (x) I3) x through the per-stencil operator (eqs 20-22, 39-41, 52-53).
 * Shells: the corotational gradient with the current stencil normal (eqs 24-26, 43-45, 55-57;
 * normal gradients App. B).  x device [nv][3] float64; f device [nv][3], float64 for
 * SHELL_PREC_FP64 stencils and float32 for SHELL_PREC_MIXED, overwritten.  energy: device float64
 * scalar receiving the bending energy, or NULL.  Asynchronous on `stream`.
 */
shell_status_t shell_eval_forces(shell_stencils_t st, const double* x, void* f, double* energy,
                                 shell_stream_t stream);

/*
 * shell_eval_forces_noalloc - shell_eval_forces for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid allocation): the same kernels and
 * results, with the scratch (the positions in internal order, the force before it is scattered back to
 * caller order, the per-tile energy partials, the descriptor and the tile list) in a file-scope device
 * array of 64 MiB, which each device the library runs on holds until the process ends.  Allocates
 * nothing (its first call on a device looks up that device's address of the array).  Meshes beyond about
 * 1.39 million vertices (those whose scratch would exceed 64 MiB) are SHELL_E_INVALID_ARG.  Every call on
 * a device shares that device's array: calls that overlap on one device (concurrent streams or threads)
 * race and must be serialised by the caller.  Arguments, precision and errors as shell_eval_forces.
 */
shell_status_t shell_eval_forces_noalloc(shell_stencils_t st, const double* x, void* f, double* energy,
                                         shell_stream_t stream);

/*
 * shell_assemble_constant_hessian - the constant bending Hessian K = K_s (x) I3 assembled once
 * from the rest operators (eqs 21, 41, 53; the shells reuse the plate Hessian as the paper states
 * for each model).  Only the scalar K_s is stored.  Synchronises `stream`.
 */
shell_status_t shell_assemble_constant_hessian(shell_stencils_t st, shell_stream_t stream, shell_hessian_t* out);

/*
 * shell_hessian_export_csr - host copy of K_s in the caller's vertex order, CSR with sorted columns.
 * Call with col == val == NULL to get nnz; rowptr is [nv+1] and may be NULL in that call.
 */
shell_status_t shell_hessian_export_csr(shell_hessian_t h, int64_t* nnz, int64_t* rowptr, int32_t* col, double* val);

/*
 * shell_hessian_info - storage figures of the assembled K_s (for byte models and inspection).
 * SELL-64 stores 64-row slices padded to the slice's longest row; rows are grouped 512 at a time and,
 * when every group's distinct column set fits in LDS (max_group_cols <= 4096), the product stages
 * each group's p entries once and stores 16-bit group-local column ids (staged == 1).
 */
typedef struct {
    int64_t nv;              /* rows */
    int64_t nnz;             /* structural nonzeros */
    int64_t slots;           /* stored SELL-64 entries, padding included */
    int64_t nslices;         /* 64-row slices */
    int64_t group_cols;      /* sum over the 512-row groups of their distinct column counts (0 unless staged) */
    int32_t max_group_cols;  /* largest distinct column count of a group */
    int32_t staged;          /* 1: staged product with 16-bit local ids; 0: direct gathers, 32-bit ids */
} shell_hessian_info_t;

shell_status_t shell_hessian_info(shell_hessian_t h, shell_hessian_info_t* info);

/*
 * shell_hessian_apply - q = diag(mass) p + dt2 (K_s (x) I3) p, the operator of the implicit step.
 * mass device [nv] float64 or NULL (no mass term); p, q device [nv][3] float64, caller order.
 */
shell_status_t shell_hessian_apply(shell_hessian_t h, const double* mass, double dt2, const double* p, double* q,
                                   shell_stream_t stream);

/*
 * shell_sim_create - simulation state for the implicit step (Sec. 5).
 * x0, v0 host [nv][3] (v0 may be NULL = zero); pinned host [nv], 1 = all three coordinates held at
 * x0 (fixed boundary nodes, Sec. 4.3), may be NULL.  The lumped mass rho h sum(A_T)/3 is computed
 * from the rest mesh.  The stencils and Hessian must outlive the simulation.  Stencils built with
 * SHELL_FLAG_MEMBRANE give the step with the membrane (either precision).
 */
shell_status_t shell_sim_create(shell_stencils_t st, shell_hessian_t h, const double* x0, const double* v0,
                                const uint8_t* pinned, shell_sim_t* out);

#define SHELL_MAX_NEWTON 256

typedef enum { SHELL_PCG_TOLERANCE = 0, SHELL_PCG_REPLAY = 1 } shell_pcg_mode_t;

typedef struct {
    double dt;             /* time step [s] */
    double gravity[3];     /* acceleration [m/s^2]; f_ext = m g */
    int32_t max_newton;    /* Newton solves per step, 0..SHELL_MAX_NEWTON */
    int32_t max_pcg;       /* PCG iteration cap per column (tolerance mode) */
    double newton_rtol;    /* stop when ||g_k|| <= newton_rtol ||g_0|| */
    double pcg_rtol;       /* per column: stop when ||r|| <= pcg_rtol ||b||.  Mixed precision uses it for
                              its float32 inner solve as well (there is no separate inner tolerance): the
                              recurrence residual r is float64, the Newton loop re-forms the residual in
                              float64 each iteration; below 1e-6 (tolerance mode), a converged solve is
                              restarted from its true residual, formed with the float64 K_s, at most
                              twice (residual replacement; the passes' iterations count in the stats) */
    int32_t mode;          /* shell_pcg_mode_t */
    int32_t chunk;         /* PCG iterations launched between host convergence checks; 0 = default */
    int32_t pcg_workgroups; /* work-groups of each PCG kernel (each takes consecutive 512-row groups),
                               0..1024; 0 = default (512: two per CU).  Batches use the first entry's value */
    int32_t flags;         /* 0 or SHELL_STEP_NO_GRAPHS; batches use the first entry's value */
    const int32_t* replay_counts; /* host [max_newton][3], REPLAY only: exact PCG iterations */
} shell_step_params_t;

/* PCG iterations are launched as captured HIP graphs of 8..128 iterations (replayed from a cache
 * keyed by the launch shape); this flag launches every kernel directly instead.  Graphs are not used
 * while in-step sampling is on. */
#define SHELL_STEP_NO_GRAPHS 1

typedef struct {
    int32_t newton_iters;  /* Newton solves performed */
    int32_t pcg_total;     /* PCG iterations summed over solves and columns */
    int32_t status;        /* shell_status_t of the step (SHELL_E_BUDGET is a warning) */
    int32_t newton_capped; /* 1: the Newton loop stopped at max_newton solves before its residual test held
                              (||g|| > newton_rtol ||g_0||, or for the quasi-static solve ||r|| >= eps_f);
                              the state is that of the last solve.  0: the residual test stopped it */
    double grad_norm0;     /* ||g|| at the predictor */
    double grad_norm;      /* ||g|| at the returned state */
    int32_t counts[SHELL_MAX_NEWTON][3]; /* PCG iterations per Newton solve and coordinate */
} shell_step_stats_t;

/*
 * shell_step_implicit - one implicit-Euler step x^t -> x^{t+1}: predictor x_hat = x + dt v + dt^2 g,
 * Newton iterations on the incremental potential E(x) = 1/2 (x-x_hat)^T M (x-x_hat) + dt^2 Psi(x)
 * (eq 62 without contact terms) against the constant matrix M + dt^2 K_s (x) I3, each solve by three
 * Jacobi-PCG recurrences (one per coordinate) sharing one sparse product, then v = (x^{t+1}-x^t)/dt.
 * stats (host, may be NULL): when given, the call synchronises `stream` and fills it.
 * Returns SHELL_E_BUDGET when a PCG column hit max_pcg (the state is still advanced).
 */
shell_status_t shell_step_implicit(shell_sim_t sim, const shell_step_params_t* params, shell_step_stats_t* stats,
                                   shell_stream_t stream);

/*
 * shell_solve_static - quasi-static equilibrium (Sec. 5, eq 64) by Newton-Raphson in one load step: from
 * the simulation's current positions, iterate x += s dx with K dx = -r, r = dPsi/dx - F the residual
 * force (fixed rows excluded), K = K_s (x) I3 the constant bending Hessian (no mass term), each solve by
 * the three Jacobi-PCG recurrences of the implicit step; stop when ||r|| < eps_f or after max_newton
 * solves.  s = eps_u / ||dx||_inf when that is below one (the incremental displacement limit), else 1.
 * Plates are linear (f = -K (x - X)), so one solve is exact; the bending-only shells' in-plane modes
 * have no stiffness of their own, so their iteration stalls at a residual of second order in the load.
 * With SHELL_FLAG_MEMBRANE the residual includes the membrane and the matrix its tangent,
 * K_s (x) I3 + K_m(x), solved by one coupled Jacobi-PCG (PCG count in counts[k][0]).
 * The velocity and the step counter are not touched.  stats (host, may be NULL) as for the step:
 * grad_norm0 = ||r|| at the start, grad_norm = at the returned state.  Synchronises `stream`.
 * Errors: SHELL_E_INVALID_ARG, SHELL_E_BUDGET (a PCG column hit max_pcg; the state is still updated),
 * SHELL_E_NONFINITE, SHELL_E_HIP.
 */
typedef struct {
    const double* load;    /* host [nv][3] applied force F in caller order, or NULL (no load) */
    double eps_f;          /* residual force tolerance, >= 0 */
    double eps_u;          /* incremental displacement limit (max norm), > 0; 0 = no limit */
    int32_t max_newton;    /* Newton-Raphson solves, 0..SHELL_MAX_NEWTON */
    int32_t max_pcg;       /* PCG iteration cap per column (tolerance mode) */
    double pcg_rtol;       /* per column: stop when ||r_pcg|| <= pcg_rtol ||b|| */
    int32_t mode;          /* shell_pcg_mode_t */
    int32_t chunk;         /* as in shell_step_params_t */
    int32_t pcg_workgroups;
    int32_t flags;         /* 0 or SHELL_STEP_NO_GRAPHS */
    const int32_t* replay_counts; /* host [max_newton][3], REPLAY only */
} shell_static_params_t;

shell_status_t shell_solve_static(shell_sim_t sim, const shell_static_params_t* params, shell_step_stats_t* stats,
                                  shell_stream_t stream);

shell_status_t shell_sim_get_stats(shell_sim_t sim, shell_step_stats_t* out);
/* host copies in caller order; x, v may be NULL; synchronises the simulation's last stream */
shell_status_t shell_sim_get_state(shell_sim_t sim, double* x, double* v, int64_t* step);
shell_status_t shell_sim_set_state(shell_sim_t sim, const double* x, const double* v, int64_t step);
/*
 * shell_sim_set_held - which coordinates of each vertex are held (kept at their current value by the
 * step and the quasi-static solve): held host [nv] in caller order, bit c (1, 2, 4) holding coordinate
 * c (x, y, z) of the vertex, 7 the whole vertex, as a symmetry plane holds the coordinate normal to it
 * (the hemisphere benchmark of Sec. 6 holds x on the plane x = 0, y on y = 0 and z of two hole-rim
 * vertices).  It replaces the set given to shell_sim_create (whose nonzero entries hold all three);
 * NULL holds nothing.  A held coordinate's residual row is zero and its increment stays zero.  Takes
 * effect at the next step or solve; synchronises the simulation's last stream.
 * Errors: SHELL_E_INVALID_ARG (an entry above 7).
 */
shell_status_t shell_sim_set_held(shell_sim_t sim, const uint8_t* held);
/* device views of the state in the library's internal order (for timing harnesses), may be NULL */
shell_status_t shell_sim_device_state(shell_sim_t sim, double** x, double** v);

/*
 * Multi-mesh batch: simulations stepped together, one launch per phase over all of them (force
 * tiles of every mesh, row groups of every mesh; reductions and Newton/PCG control per mesh).  Each
 * mesh keeps its own model, size, parameters and iteration counts; the result of each mesh is that of
 * stepping it alone (up to summation order of the tile accumulation).
 *
 * shell_batch_create: sims host [n] distinct handles of one precision, n >= 1; the simulations must
 * outlive the batch and must not be stepped alone while the batch is in use.  Simulations with the
 * membrane (SHELL_FLAG_MEMBRANE) form batches of their own (mixing them with simulations without it is
 * SHELL_E_INVALID_ARG): each member takes the step it takes alone (bit for bit), on a stream of its own
 * that starts after the work already on `stream`; the calling thread keeps the members' steps in flight
 * together and returns when every one has finished.  Members may share stencils and Hessian handles.
 * Sampled timing (shell_batch_profile) refuses such a batch (SHELL_E_UNSUPPORTED).
 * shell_batch_step: params host [nparams], nparams = 1 (shared) or n; stats host [n] or NULL.  Returns
 * the worst per-mesh status (SHELL_E_NONFINITE, then SHELL_E_BUDGET); per-mesh statuses are in stats.
 * Synchronises `stream` at the end of every Newton round.
 */
shell_status_t shell_batch_create(const shell_sim_t* sims, int32_t n, shell_batch_t* out);
shell_status_t shell_batch_step(shell_batch_t batch, const shell_step_params_t* params, int32_t nparams,
                                shell_step_stats_t* stats, shell_stream_t stream);
/* shell_batch_reset: rebind an existing batch to another set of simulations (continuous batching: members
 * join and leave between steps); buffers are reused and only grow.  Same rules as shell_batch_create. */
shell_status_t shell_batch_reset(shell_batch_t batch, const shell_sim_t* sims, int32_t n);

/* shell_sim_device_bytes: device memory held by the simulation's stencils, Hessian and state (host
 * int64 outputs, each may be NULL); for admission by HBM footprint.  The state counts the solver's work
 * arrays, the membrane solver's when the simulation has one, and buffers made on first use (the quasi-
 * static load and mass, the mixed refinement's product) once they exist. */
shell_status_t shell_sim_device_bytes(shell_sim_t sim, int64_t* stencil_bytes, int64_t* hessian_bytes,
                                      int64_t* sim_bytes);
void shell_destroy_batch(shell_batch_t batch);

/*
 * shell_sim_time_kernels - timing harness: average duration of one launch of each hot kernel of the
 * step, measured with HIP events on `stream` over `reps` back-to-back launches on the simulation's
 * current state (forces at x, then the PCG kernels on a freshly initialised recurrence).  The position
 * and velocity are not modified; the solver's work vectors are.  Synchronises `stream`.  For a
 * simulation with the membrane: the bending and membrane force tiles, the coupled product (with the
 * membrane tangent at x) and its update.
 */
typedef struct {
    double force_ms;      /* force kernels over all stencils (internal vertex order); with the membrane,
                             bending and membrane tiles together */
    double spmv_ms;       /* PCG direction update p = D^-1 r + beta p and product q = (M + dt^2 K_s) p
                             (with the membrane: + dt^2 K_m p, coordinates coupled) */
    double update_ms;     /* PCG y/r update with its dot products */
    double direction_ms;  /* always 0: the direction update is part of the product kernel */
    int32_t reps;
    int32_t reserved;
} shell_kernel_times_t;

shell_status_t shell_sim_time_kernels(shell_sim_t sim, double dt, int32_t reps, shell_kernel_times_t* out,
                                      shell_stream_t stream);

/*
 * Sampled kernel timing inside real steps.  With sampling on, every step of the batch (or simulation)
 * records HIP events on its stream around every force launch set and around every `every`-th PCG
 * iteration's two kernels, and sums the sampled durations per phase; the events are read at the
 * step's existing host synchronisations, so the step's launches and results are unchanged.
 *   shell_batch_profile(b, every)  every > 0: start sampling and clear the sums; every == 0: stop.
 *   shell_batch_profile_read(b, out)  copy the sums (sampling continues).
 * The simulation forms act on a simulation's own one-member batch.
 */
enum {
    SHELL_PHASE_FORCES = 0,   /* force kernels of one Newton iteration (all tiles of all models) */
    SHELL_PHASE_PRODUCT = 1,  /* PCG state advance, direction update and sparse product */
    SHELL_PHASE_UPDATE = 2,   /* PCG step length, y/r update and dot products */
    SHELL_NUM_PHASES = 3
};
typedef struct {
    double ms[SHELL_NUM_PHASES];     /* summed durations of the sampled launches, milliseconds */
    int64_t count[SHELL_NUM_PHASES]; /* number of sampled launches */
} shell_profile_t;

shell_status_t shell_batch_profile(shell_batch_t batch, int32_t every);
shell_status_t shell_batch_profile_read(shell_batch_t batch, shell_profile_t* out);
shell_status_t shell_sim_profile(shell_sim_t sim, int32_t every);
shell_status_t shell_sim_profile_read(shell_sim_t sim, shell_profile_t* out);

void shell_destroy_stencils(shell_stencils_t st);
void shell_destroy_hessian(shell_hessian_t h);
void shell_destroy_sim(shell_sim_t sim);

const char* shell_status_string(shell_status_t s);
const char* shell_last_error(void);

#ifdef __cplusplus
}
#endif
#endif
