/*
 * Plain FP64 CPU oracle for the corotational hinge plate/shell bending models
 * (EP, ES, FP, FS, SP, SS of "Corotational Hinge-based Thin Plates/Shells").
 *
 * TEST INFRASTRUCTURE ONLY.  This library is the slow, obviously-correct
 * definition the HIP library is checked against.  Only the test-suite, the
 * smoke check and the CPU-baseline leg of the benchmark may load it; the
 * product path never calls it.  It shares no code, header or table with the
 * HIP library.
 *
 * Every function returns 0 on success or a negative ORC_E_* code.
 * Arrays are caller-owned, row-major, host memory.
 *
 * Parity status: every function is pinned by tests under tests/ (closed
 * forms, invariants, finite differences, brute force) except the FVM
 * free-edge twist reading (see orc_build), which is "parity unpinned" beyond
 * the invariants, finite-difference and Hessian pins.
 */
#ifndef SHELL_ORACLE_H
#define SHELL_ORACLE_H
#include <stdint.h>

#define ORC_OK 0
#define ORC_E_ARG (-1)
#define ORC_E_NONMANIFOLD (-2)
#define ORC_E_ORIENTATION (-3)
#define ORC_E_DEGENERATE (-4)
#define ORC_E_BUDGET (-5)

/* model ids: 0 EP, 1 ES, 2 FP, 3 FS, 4 SP, 5 SS */
int orc_stencil_size(int model);   /* 4 (edge) or 6 (triangle) */
int orc_curv_size(int model);      /* 1 (edge) or 3 (triangle) */

/* Stencil topology.  idx == NULL: only *ns is returned.  Edge stencils are
 * (1,2,3,4) per interior edge with 2->3 the directed edge of the lower-id
 * orientation; triangle stencils are (1,2,3,4,5,6) per triangle with flap
 * i+3 across the edge opposite vertex i, -1 when that edge is a boundary.
 * clamped [n_clamped][2]: vertex pairs of boundary edges to clamp (any other
 * pair is ORC_E_ARG).  The edge plate (EP) then also gets one stencil
 * (L, M, N, -1) per clamped edge, after the interior ones, bc = 1; the edge
 * shell (ES) gets none.  Triangle stencils: bc bit i = flap i+3 is missing
 * and its edge clamped.  bc [ns] is required with idx. */
int orc_topology(int model, int64_t nv, int64_t nt, const int32_t* tris, int64_t n_clamped,
                 const int32_t* clamped, int64_t* ns, int32_t* idx, uint8_t* bc);

/* Rest precompute: operator B [ns][r][k], rest curvature kappa0 [ns][r]
 * (zero for plates), material D [ns][r][r] (k_b*A_E for edges, A*D_b for
 * triangles), rest curvature vectors Crest [ns][r][3] = B X of plate
 * stencils with a clamped edge (zero otherwise).  Free and clamped folds
 * (eqs 30-31, 59-61) are applied to B per bc from orc_topology.  flags: ORC_WORLD_FRAME
 * (edge models only) builds the quadratic thin plate/shell operator L_n of
 * App. D (eq 79), heights and feet taken on the unprojected rest stencil. */
#define ORC_WORLD_FRAME 1
int orc_build(int model, int64_t nv, const double* X, int64_t ns, const int32_t* idx, const uint8_t* bc,
              double young, double poisson, double thickness, int flags,
              double* B, double* kappa0, double* D, double* Crest);

/* Bending energy and force f = -dPsi/dx over all stencils. f [nv][3] is overwritten.
 * Crest (may be NULL): plate curvature vectors are C = B x - Crest. */
int orc_forces(int model, int64_t nv, const double* x, int64_t ns, const int32_t* idx,
               const double* B, const double* kappa0, const double* Crest, const double* D, double* f,
               double* energy);

/* Constant bending Hessian, scalar part K_s (K = K_s (x) I3), CSR with sorted
 * columns.  rowptr [nv+1]; col/val == NULL: only *nnz is returned. */
int orc_hessian(int model, int64_t nv, int64_t ns, const int32_t* idx, const double* B, const double* D,
                int64_t* nnz, int64_t* rowptr, int32_t* col, double* val);

/* Lumped mass m_v = rho*h*sum(A_T)/3 over the rest triangles around v. */
int orc_mass(int64_t nv, const double* X, int64_t nt, const int32_t* tris, double density, double thickness,
             double* mass);

/* q = diag(mass) p + dt2 * (K_s (x) I3) p, p and q [nv][3]. */
int orc_apply(int64_t nv, const int64_t* rowptr, const int32_t* col, const double* val,
              const double* mass, double dt2, const double* p, double* q);

/* One implicit-Euler step (incremental potential without contact) by a
 * Newton iteration against the constant matrix M + dt^2 K, each linear solve
 * by three Jacobi-PCG recurrences (one per coordinate) sharing the operator.
 * x, v: in x^t, v^t; out x^{t+1}, v^{t+1}.  replay [max_newton][3] or NULL:
 * when given, every solve runs exactly that many PCG iterations per column.
 * counts [max_newton][3] receives the iterations taken; stats[4] =
 * {newton_iters, pcg_total, grad_norm0, grad_norm_final}.  pinned [nv] (here and in every solver below):
 * the held coordinates of each vertex, bit d holding coordinate d (x, y, z), 7 the whole vertex; a held
 * coordinate keeps its value and its residual row is zero. */
int orc_step(int model, int64_t nv, int64_t ns, const int32_t* idx, const double* B, const double* kappa0,
             const double* Crest, const double* D, const int64_t* rowptr, const int32_t* col, const double* val,
             const double* mass, const uint8_t* pinned, double* x, double* v,
             double dt, const double* gravity, int max_newton, double newton_rtol,
             double pcg_rtol, int max_pcg, const int32_t* replay, int32_t* counts, double* stats);

/* Normal of an edge stencil by the literal height-vector construction
 * (sum of the unit height vectors of vertices 1 and 4), used only as a cross-check. */
/* Quasi-static Newton-Raphson (eq 64): x [nv][3] in/out; load [nv][3] the applied force F (may be NULL);
 * stop when ||dPsi/dx - F|| < eps_f (fixed rows excluded) or after max_newton solves of K dx = -r;
 * eps_u > 0 caps ||dx||_inf by scaling dx.  replay/counts [max_newton][3] as in orc_step; stats [4] =
 * (Newton solves, PCG iterations, ||r_0||, ||r||). */
int orc_static(int model, int64_t nv, int64_t ns, const int32_t* idx, const double* B, const double* kappa0,
               const double* Crest, const double* D, const int64_t* rowptr, const int32_t* col, const double* val,
               const uint8_t* pinned, const double* load, double* x, double eps_f, double eps_u, int max_newton,
               double pcg_rtol, int max_pcg, const int32_t* replay, int32_t* counts, double* stats);

/* Membrane (Sec. 3, eq 1): constant strain triangles, Saint Venant-Kirchhoff, D_m = h E_el.
 * orc_membrane adds the force into f [nv][3] and returns the energy; orc_membrane_rest_hessian writes
 * the rest Hessian per triangle, K9 [nt][9][9] (vertex-major, coordinate-minor). */
int orc_membrane(int64_t nv, const double* x, int64_t nt, const int32_t* tris, const double* X, double young,
                 double poisson, double thickness, double* f, double* energy);
int orc_membrane_rest_hessian(int64_t nt, const int32_t* tris, const double* X, double young, double poisson,
                              double thickness, double* K9);
/* Gauss-Newton membrane tangent at x per triangle, K9 [nt][9][9] (PSD; the rest Hessian at x = X). */
int orc_membrane_gn_hessian(int64_t nt, const int32_t* tris, const double* X, const double* x, double young,
                            double poisson, double thickness, double* K9);
/* Membrane tangent of the solvers: the Gauss-Newton part plus the stress part of the exact Hessian with
 * the stress replaced by its positive semi-definite part (exact under tension, Gauss-Newton under
 * compression, PSD throughout), K9 [nt][9][9]. */
int orc_membrane_tangent(int64_t nt, const int32_t* tris, const double* X, const double* x, double young,
                         double poisson, double thickness, double* K9);
/* Implicit-Euler step with bending and membrane: Newton matrix M + dt^2 (K_s (x) I3 + K_GN(x)), one
 * Jacobi-PCG over all coordinates, Armijo backtracking (at most 6 halvings) on the incremental potential.
 * replay_pcg, replay_halvings [max_newton] (may be NULL); counts, halvings [max_newton] out. */
int orc_step_membrane(int model, int64_t nv, int64_t ns, const int32_t* idx, const double* B, const double* kappa0,
                      const double* Crest, const double* D, const int64_t* rowptr, const int32_t* col,
                      const double* val, int64_t nt, const int32_t* tris, const double* X, double young,
                      double poisson, double thickness, const double* mass, const uint8_t* pinned, double* x,
                      double* v, double dt, const double* gravity, int max_newton, double newton_rtol,
                      double pcg_rtol, int max_pcg, const int32_t* replay_pcg, const int32_t* replay_halvings,
                      int32_t* counts, int32_t* halvings, double* stats);

/* Quasi-static equilibrium with the membrane (eq 64, Psi_shell = Psi_b + Psi_m): Newton-Raphson against
 * K_s (x) I3 + K_GN(x), one coupled PCG per solve, eps_f / eps_u as in orc_static; replay/counts
 * [max_newton]. */
int orc_static_membrane(int model, int64_t nv, int64_t ns, const int32_t* idx, const double* B,
                        const double* kappa0, const double* Crest, const double* D, const int64_t* rowptr,
                        const int32_t* col, const double* val, int64_t nt, const int32_t* tris, const double* X,
                        double young, double poisson, double thickness, const uint8_t* pinned, const double* load,
                        double* x, double eps_f, double eps_u, int max_newton, double pcg_rtol, int max_pcg,
                        const int32_t* replay, int32_t* counts, double* stats);

int orc_edge_normal_literal(const double* x1, const double* x2, const double* x3, const double* x4, double* n);

/* Threads of the parallel loops: sets the count when n > 0 and returns the count in use
   (always 1 in the serial build, which ignores n). */
int orc_threads(int n);

#endif
