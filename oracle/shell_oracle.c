/*
 * Plain FP64 CPU oracle for the corotational hinge plate/shell bending models.
 *
 * TEST INFRASTRUCTURE ONLY: loaded by tests/, the smoke check and the
 * benchmark's CPU-baseline leg, never by the product path.  Shares no code
 * with the HIP library.
 *
 * Everything is written as plain loops in the order the paper states it:
 *   Sec. 4.3  edge-based hinge: operator L_m (eqs 7, 9-10), curvature
 *             kappa = L_m N^T x (eq 13), plate energy (eq 20), shell energy
 *             and gradient (eqs 23-26), free boundary edges emit nothing.
 *   Sec. 4.4  FVM hinge: directional operator L_p (eqs 37, 40 and App. C
 *             eqs 76-78), transform R (eq 38), energies eqs 39-45, free-edge
 *             fold and zero twist on free edges.
 *   Sec. 4.5  smoothed hinge: quadratic fit C_p, L_g = (L_p C_p)^-1 L_p
 *             (eqs 48-51), energies eqs 52-57, virtual-node folds eqs 58-61.
 *   App. A    corotational frames (eq 65), App. B normal gradients (eqs 66-75).
 *   Sec. 5    implicit Euler as the minimiser of the incremental potential
 *             (eqs 62-63) with no contact terms, by Newton against the
 *             constant Hessian of eqs 21/41/53; quasi-static equilibrium
 *             (eq 64) by Newton-Raphson with the eps_f / eps_u controls.
 *   Sec. 3    membrane energy (eq 1) on constant strain triangles with the
 *             Saint Venant-Kirchhoff model, its Hessian at rest, its
 *             Gauss-Newton tangent, and the implicit step of the shell with
 *             its membrane (Gauss-Newton matrix, Armijo backtracking).
 *
 * Built plain (serial, fixed summation order) for every check.  The same
 * source built with -fopenmp is a timing build only, for the all-cores CPU
 * baseline: the stencil loop, the sparse product and the vector loops of the
 * implicit step then run in parallel, and the force scatter uses atomic adds,
 * so its sums have no fixed order.
 *
 * Readings where the paper is silent or ambiguous (each is also listed in the
 * design notes of the repository):
 *  - foot ratios are signed, s_p = (X1-X2).e/|e|^2 (the App. B definition),
 *    so the operator annihilates constants even on obtuse stencils;
 *  - heights and feet are measured on the projected (corotational) stencil;
 *  - the edge-stencil normal is normalize(n_T123 + n_T432), the same line as
 *    eq 8's sum of unit height vectors but with a sign that does not flip with
 *    the bend direction (eq 8 itself is kept as orc_edge_normal_literal);
 *  - D_b = k_b [[1,nu,0],[nu,1,0],[0,0,(1-nu)/2]] with k_b = E h^3/(12(1-nu^2)),
 *    Voigt curvature [w_XX, w_YY, 2 w_XY];
 *  - A_E is the sum of the two rest triangle areas; A the central triangle's;
 *  - a missing flap L+3 is the point reflection of L through the midpoint of
 *    the boundary edge, and the free fold w_{L'} = w_M + w_N - w_L is applied
 *    to the operator's columns (eq 61) for both triangle models;
 *  - FVM: when a stencil has a free edge, the twist component is zeroed in the
 *    frame whose x axis runs along its first free edge (parity unpinned beyond
 *    invariants, finite differences and Hessian checks);
 *  - clamped edges (eqs 30-31, 59): the virtual node moves with L, so its
 *    operator column joins L's; the edge plate's boundary stencil weighs its one
 *    real triangle's area; a plate stencil with a clamped edge measures its
 *    curvature vectors from the rest shape, C = B (x - X), since the clamped
 *    fold does not annihilate the flat rest coordinates; FVM keeps the twist on
 *    clamped edges; the edge shell emits no clamped stencil (its energy would
 *    vanish identically in its own triangle's frame);
 *  - mass is lumped, m_v = rho h sum(A_T)/3; x_hat = x + dt v + dt^2 g;
 *    v^{t+1} = (x^{t+1} - x^t)/dt; held coordinates keep their value (the
 *    fixed set is a per-vertex mask of coordinates, bit d holding coordinate d,
 *    so a symmetry plane holds one coordinate of its vertices);
 *  - linear solver: Jacobi-preconditioned CG per coordinate, x0 = 0, stop when
 *    ||r|| <= rtol ||b||; alpha = 0 when p.q = 0, beta = 0 when r.z was 0.
 */
#include "shell_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

/* held coordinates: pinned[i] bit d holds coordinate d of vertex i; 7 holds the whole vertex */
static int held(const uint8_t* pinned, int64_t i, int d) { return (pinned[i] >> d) & 1; }
static int held_all(const uint8_t* pinned, int64_t i) { return (pinned[i] & 7) == 7; }
#ifdef _OPENMP
#include <omp.h>
#endif

/* ---------------------------------------------------------------- vectors */

static void sub3(const double* a, const double* b, double* o) { o[0] = a[0] - b[0]; o[1] = a[1] - b[1]; o[2] = a[2] - b[2]; }
static double dot3(const double* a, const double* b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }
static void cross3(const double* a, const double* b, double* o) {
    o[0] = a[1] * b[2] - a[2] * b[1];
    o[1] = a[2] * b[0] - a[0] * b[2];
    o[2] = a[0] * b[1] - a[1] * b[0];
}
static double norm3(const double* a) { return sqrt(dot3(a, a)); }
static void scale3(const double* a, double s, double* o) { o[0] = a[0] * s; o[1] = a[1] * s; o[2] = a[2] * s; }
static void axpy3(double s, const double* a, double* o) { o[0] += s * a[0]; o[1] += s * a[1]; o[2] += s * a[2]; }

/* unit normal of triangle (a,b,c) and the length of (b-a)x(c-a) */
static double tri_normal(const double* a, const double* b, const double* c, double* n) {
    double ab[3], ac[3], u[3];
    sub3(b, a, ab);
    sub3(c, a, ac);
    cross3(ab, ac, u);
    double len = norm3(u);
    if (len > 0) scale3(u, 1.0 / len, n);
    else n[0] = n[1] = n[2] = 0;
    return len;
}

int orc_stencil_size(int model) { return (model == 0 || model == 1) ? 4 : 6; }
int orc_curv_size(int model) { return (model == 0 || model == 1) ? 1 : 3; }
static int is_edge(int model) { return model == 0 || model == 1; }
static int is_shell(int model) { return model == 1 || model == 3 || model == 5; }
static int is_fvm(int model) { return model == 2 || model == 3; }

/* --------------------------------------------------------------- topology */

typedef struct { int32_t from, to, opp; } dedge_t;

static int cmp_dedge(const void* pa, const void* pb) {
    const dedge_t* a = (const dedge_t*)pa;
    const dedge_t* b = (const dedge_t*)pb;
    if (a->from != b->from) return a->from < b->from ? -1 : 1;
    if (a->to != b->to) return a->to < b->to ? -1 : 1;
    return 0;
}

/* all directed edges of the mesh, sorted by (from, to); validates the mesh */
static int directed_edges(int64_t nv, int64_t nt, const int32_t* tris, dedge_t** out) {
    dedge_t* de = (dedge_t*)malloc(sizeof(dedge_t) * (size_t)(3 * nt + 1));
    if (!de) return ORC_E_ARG;
    for (int64_t t = 0; t < nt; ++t) {
        const int32_t* v = tris + 3 * t;
        for (int i = 0; i < 3; ++i) {
            if (v[i] < 0 || v[i] >= nv) { free(de); return ORC_E_ARG; }
        }
        if (v[0] == v[1] || v[1] == v[2] || v[2] == v[0]) { free(de); return ORC_E_DEGENERATE; }
        for (int i = 0; i < 3; ++i) {
            de[3 * t + i].from = v[i];
            de[3 * t + i].to = v[(i + 1) % 3];
            de[3 * t + i].opp = v[(i + 2) % 3];
        }
    }
    qsort(de, (size_t)(3 * nt), sizeof(dedge_t), cmp_dedge);
    for (int64_t e = 1; e < 3 * nt; ++e) {
        if (de[e].from == de[e - 1].from && de[e].to == de[e - 1].to) {
            /* the same directed edge in two triangles: a fan of three or more triangles when the
               reverse direction is also present, otherwise two inconsistently oriented triangles */
            dedge_t key = {de[e].to, de[e].from, 0};
            int fan = bsearch(&key, de, (size_t)(3 * nt), sizeof(dedge_t), cmp_dedge) != NULL;
            free(de);
            return fan ? ORC_E_NONMANIFOLD : ORC_E_ORIENTATION;
        }
    }
    *out = de;
    return ORC_OK;
}

static const dedge_t* find_dedge(const dedge_t* de, int64_t n, int32_t from, int32_t to) {
    dedge_t key = {from, to, 0};
    return (const dedge_t*)bsearch(&key, de, (size_t)n, sizeof(dedge_t), cmp_dedge);
}

/* undirected vertex pair, smaller id first, for the clamped-edge lookup */
typedef struct { int32_t a, b; } upair_t;

static int cmp_upair(const void* pa, const void* pb) {
    const upair_t* x = (const upair_t*)pa;
    const upair_t* y = (const upair_t*)pb;
    if (x->a != y->a) return x->a < y->a ? -1 : 1;
    if (x->b != y->b) return x->b < y->b ? -1 : 1;
    return 0;
}

static int is_clamped(const upair_t* cl, int64_t ncl, int32_t u, int32_t v) {
    upair_t key = {u < v ? u : v, u < v ? v : u};
    return ncl > 0 && bsearch(&key, cl, (size_t)ncl, sizeof(upair_t), cmp_upair) != NULL;
}

int orc_topology(int model, int64_t nv, int64_t nt, const int32_t* tris, int64_t n_clamped,
                 const int32_t* clamped, int64_t* ns, int32_t* idx, uint8_t* bc) {
    if (model < 0 || model > 5 || nv < 0 || nt < 0 || !ns || n_clamped < 0 || (n_clamped > 0 && !clamped) ||
        (idx && !bc))
        return ORC_E_ARG;
    dedge_t* de = NULL;
    int rc = directed_edges(nv, nt, tris, &de);
    if (rc) return rc;
    int64_t nde = 3 * nt;
    /* clamped edges (Sec. 4.3 boundary conditions): each must be a boundary edge, i.e. traversed by
       exactly one triangle */
    upair_t* cl = (upair_t*)malloc(sizeof(upair_t) * (size_t)(n_clamped + 1));
    if (!cl) { free(de); return ORC_E_ARG; }
    for (int64_t e = 0; e < n_clamped; ++e) {
        int32_t u = clamped[2 * e], v = clamped[2 * e + 1];
        int one = (find_dedge(de, nde, u, v) != NULL) + (find_dedge(de, nde, v, u) != NULL);
        if (u < 0 || v < 0 || u >= nv || v >= nv || one != 1) { free(cl); free(de); return ORC_E_ARG; }
        cl[e].a = u < v ? u : v;
        cl[e].b = u < v ? v : u;
    }
    qsort(cl, (size_t)n_clamped, sizeof(upair_t), cmp_upair);
    /* an undirected edge shared by two triangles must appear once in each direction;
       a third triangle on the same pair of vertices makes the edge non-manifold */
    int64_t count = 0;
    for (int64_t e = 0; e < nde; ++e) {
        const dedge_t* tw = find_dedge(de, nde, de[e].to, de[e].from);
        if (tw && de[e].from < de[e].to) {
            /* both directions present exactly once (directed_edges rejects repeats) */
            if (is_edge(model)) {
                if (idx) {
                    int32_t* s = idx + 4 * count;
                    s[0] = de[e].opp; /* vertex 1: T123 traverses 2->3 */
                    s[1] = de[e].from;
                    s[2] = de[e].to;
                    s[3] = tw->opp; /* vertex 4: T432 traverses 3->2 */
                    bc[count] = 0;
                }
                ++count;
            }
        }
    }
    if (is_edge(model) && !is_shell(model)) {
        /* plate: a clamped boundary edge gets the stencil (L, M, N, L') of its one triangle, the virtual
           node L' (-1 here) being the reflection of L through the edge's midpoint.  The edge shell's
           boundary stencil is not emitted: measured along its own triangle's normal, every transverse
           displacement of the folded stencil is zero, so its energy vanishes identically. */
        for (int64_t e = 0; e < nde; ++e) {
            if (find_dedge(de, nde, de[e].to, de[e].from)) continue;
            if (!is_clamped(cl, n_clamped, de[e].from, de[e].to)) continue;
            if (idx) {
                int32_t* s = idx + 4 * count;
                s[0] = de[e].opp;
                s[1] = de[e].from;
                s[2] = de[e].to;
                s[3] = -1;
                bc[count] = 1;
            }
            ++count;
        }
    }
    if (!is_edge(model)) {
        count = nt;
        if (idx) {
            for (int64_t t = 0; t < nt; ++t) {
                const int32_t* v = tris + 3 * t;
                int32_t* s = idx + 6 * t;
                s[0] = v[0];
                s[1] = v[1];
                s[2] = v[2];
                for (int i = 0; i < 3; ++i) {
                    /* flap i+3 lies across the edge opposite vertex i, i.e. (v[i+1], v[i+2]);
                       the neighbour traverses that edge as v[i+2] -> v[i+1] */
                    const dedge_t* nb = find_dedge(de, nde, v[(i + 2) % 3], v[(i + 1) % 3]);
                    s[3 + i] = nb ? nb->opp : -1;
                }
                /* bit i: the missing flap i+3 lies across a clamped edge */
                bc[t] = 0;
                for (int i = 0; i < 3; ++i)
                    if (s[3 + i] < 0 && is_clamped(cl, n_clamped, v[(i + 1) % 3], v[(i + 2) % 3]))
                        bc[t] |= (uint8_t)(1 << i);
            }
        }
    }
    free(cl);
    free(de);
    *ns = count;
    return ORC_OK;
}

/* ------------------------------------------------------ rest precompute */

/* Edge-based hinge (Sec. 4.3): L_m = 2 L_theta/(h1+h4) on the projected stencil.  world != 0: the
   quadratic thin plate/shell variant (App. D, eq 79), whose operator L_n takes the heights and feet of
   the rest stencil as it lies in the world frame, without the projection. */
static int build_edge(int shell, int world, int clamped, const double* X1, const double* X2, const double* X3,
                      const double* X4, double kb, double* L, double* kappa0, double* D) {
    double na[3], nb[3], n0[3];
    double Aa = 0.5 * tri_normal(X1, X2, X3, na);
    double Ab = 0.5 * tri_normal(X4, X3, X2, nb);
    if (!(Aa > 0) || !(Ab > 0)) return ORC_E_DEGENERATE;
    double m[3] = {na[0] + nb[0], na[1] + nb[1], na[2] + nb[2]};
    double mlen = norm3(m);
    if (!(mlen > 1e-12)) return ORC_E_DEGENERATE;
    scale3(m, 1.0 / mlen, n0);
    /* corotational stencil: projection onto the tangent plane through X2 (X3 lies on it) */
    const double* Xs[4] = {X1, X2, X3, X4};
    double Xc[4][3];
    for (int j = 0; j < 4; ++j) {
        double d[3];
        sub3(Xs[j], X2, d);
        double w = world ? 0.0 : dot3(n0, d);
        for (int c = 0; c < 3; ++c) Xc[j][c] = Xs[j][c] - w * n0[c];
    }
    double e[3], d1[3], d4[3];
    sub3(Xc[2], Xc[1], e);
    double ee = dot3(e, e);
    sub3(Xc[0], Xc[1], d1);
    sub3(Xc[3], Xc[1], d4);
    double sp = dot3(d1, e) / ee; /* signed foot ratio of vertex 1 along 2->3 */
    double sq = dot3(d4, e) / ee; /* signed foot ratio of vertex 4 */
    double p[3], q[3];
    for (int c = 0; c < 3; ++c) {
        p[c] = d1[c] - sp * e[c];
        q[c] = d4[c] - sq * e[c];
    }
    double h1 = norm3(p), h4 = norm3(q);
    double elen = sqrt(ee);
    if (!(h1 > 1e-12 * elen) || !(h4 > 1e-12 * elen)) return ORC_E_DEGENERATE;
    double c = 2.0 / (h1 + h4);
    L[0] = c * (1.0 / h1);
    L[1] = -c * ((1.0 - sp) / h1 + (1.0 - sq) / h4);
    L[2] = -c * (sp / h1 + sq / h4);
    L[3] = c * (1.0 / h4);
    D[0] = kb * (Aa + Ab);
    if (clamped) {
        /* clamped boundary edge (eqs 30-31): the virtual node moves with L, so its column joins L's; the
           stencil's area is its one real triangle's, the virtual one lying outside the plate */
        L[0] += L[3];
        L[3] = 0.0;
        D[0] = kb * Aa;
    }
    kappa0[0] = 0.0;
    if (shell) {
        for (int j = 0; j < 4; ++j) kappa0[0] += L[j] * dot3(n0, Xs[j]);
    }
    return ORC_OK;
}

/* 3x3 inverse by the adjugate; returns the 1-norm condition number (inf if singular). */
static double inv3(const double M[3][3], double Mi[3][3]) {
    double det = M[0][0] * (M[1][1] * M[2][2] - M[1][2] * M[2][1])
               - M[0][1] * (M[1][0] * M[2][2] - M[1][2] * M[2][0])
               + M[0][2] * (M[1][0] * M[2][1] - M[1][1] * M[2][0]);
    if (det == 0.0 || !isfinite(det)) return INFINITY;
    Mi[0][0] = (M[1][1] * M[2][2] - M[1][2] * M[2][1]) / det;
    Mi[0][1] = (M[0][2] * M[2][1] - M[0][1] * M[2][2]) / det;
    Mi[0][2] = (M[0][1] * M[1][2] - M[0][2] * M[1][1]) / det;
    Mi[1][0] = (M[1][2] * M[2][0] - M[1][0] * M[2][2]) / det;
    Mi[1][1] = (M[0][0] * M[2][2] - M[0][2] * M[2][0]) / det;
    Mi[1][2] = (M[0][2] * M[1][0] - M[0][0] * M[1][2]) / det;
    Mi[2][0] = (M[1][0] * M[2][1] - M[1][1] * M[2][0]) / det;
    Mi[2][1] = (M[0][1] * M[2][0] - M[0][0] * M[2][1]) / det;
    Mi[2][2] = (M[0][0] * M[1][1] - M[0][1] * M[1][0]) / det;
    double n1 = 0, n2 = 0;
    for (int j = 0; j < 3; ++j) {
        double s1 = 0, s2 = 0;
        for (int i = 0; i < 3; ++i) {
            s1 += fabs(M[i][j]);
            s2 += fabs(Mi[i][j]);
        }
        if (s1 > n1) n1 = s1;
        if (s2 > n2) n2 = s2;
    }
    return n1 * n2;
}

/* Triangle-centred stencil (Secs 4.4, 4.5; App. A, C).  Xs[j] == NULL for a missing flap. */
static int build_tri(int model, int clampmask, const double* Xs[6], const double Db[3][3], double* B, double* kappa0,
                     double* D) {
    const double *X1 = Xs[0], *X2 = Xs[1], *X3 = Xs[2];
    /* rest corotational frame (eq 65): origin X1, x axis along X12, z the triangle normal */
    double ex[3], ez[3], ey[3], d12[3];
    double twoA = tri_normal(X1, X2, X3, ez);
    if (!(twoA > 0)) return ORC_E_DEGENERATE;
    sub3(X2, X1, d12);
    scale3(d12, 1.0 / norm3(d12), ex);
    cross3(ez, ex, ey);
    /* projected 2D coordinates of the six points */
    double P[6][2];
    int missing[3] = {0, 0, 0};
    for (int j = 0; j < 6; ++j) {
        if (Xs[j]) {
            double d[3];
            sub3(Xs[j], X1, d);
            P[j][0] = dot3(d, ex);
            P[j][1] = dot3(d, ey);
        }
    }
    for (int L = 0; L < 3; ++L) {
        if (!Xs[L + 3]) {
            /* virtual node: reflection of L through the midpoint of the boundary edge (M,N) */
            int M = (L + 1) % 3, N = (L + 2) % 3;
            missing[L] = 1;
            P[L + 3][0] = P[M][0] + P[N][0] - P[L][0];
            P[L + 3][1] = P[M][1] + P[N][1] - P[L][1];
        }
    }
    /* directional operator L_p (3x6): row i is the hinge operator across the edge opposite i */
    double Lp[3][6];
    memset(Lp, 0, sizeof(Lp));
    double emin = INFINITY;
    for (int i = 0; i < 3; ++i) {
        int a = (i + 1) % 3, b = (i + 2) % 3, f = i + 3;
        double e[2] = {P[b][0] - P[a][0], P[b][1] - P[a][1]};
        double ee = e[0] * e[0] + e[1] * e[1];
        if (sqrt(ee) < emin) emin = sqrt(ee);
        double dt[2] = {P[i][0] - P[a][0], P[i][1] - P[a][1]};
        double df[2] = {P[f][0] - P[a][0], P[f][1] - P[a][1]};
        double st = (dt[0] * e[0] + dt[1] * e[1]) / ee;
        double sf = (df[0] * e[0] + df[1] * e[1]) / ee;
        double ht = hypot(dt[0] - st * e[0], dt[1] - st * e[1]);
        double hf = hypot(df[0] - sf * e[0], df[1] - sf * e[1]);
        if (!(ht > 1e-12 * sqrt(ee)) || !(hf > 1e-12 * sqrt(ee))) return ORC_E_DEGENERATE;
        double c = 2.0 / (ht + hf);
        Lp[i][i] = c / ht;
        Lp[i][a] = -c * ((1.0 - st) / ht + (1.0 - sf) / hf);
        Lp[i][b] = -c * (st / ht + sf / hf);
        Lp[i][f] = c / hf;
    }
    double Bm[3][6];
    if (is_fvm(model)) {
        /* R (eq 38): column i from the unit normal m of edge i in the rest X~Y~ plane */
        double R[3][3];
        for (int i = 0; i < 3; ++i) {
            int a = (i + 1) % 3, b = (i + 2) % 3;
            double e[2] = {P[b][0] - P[a][0], P[b][1] - P[a][1]};
            double len = hypot(e[0], e[1]);
            double ms = e[1] / len, mt = -e[0] / len;
            R[0][i] = ms * ms;
            R[1][i] = mt * mt;
            R[2][i] = 2.0 * ms * mt;
        }
        for (int r = 0; r < 3; ++r)
            for (int j = 0; j < 6; ++j) {
                double s = 0;
                for (int i = 0; i < 3; ++i) s += R[r][i] * Lp[i][j];
                Bm[r][j] = s;
            }
    } else {
        /* quadratic fit (eqs 48-50): C_p rows [X^2/2, Y^2/2, XY/2]; L_g = (L_p C_p)^-1 L_p */
        double Cp[6][3];
        for (int j = 0; j < 6; ++j) {
            Cp[j][0] = 0.5 * P[j][0] * P[j][0];
            Cp[j][1] = 0.5 * P[j][1] * P[j][1];
            Cp[j][2] = 0.5 * P[j][0] * P[j][1];
        }
        double M3[3][3], Mi[3][3];
        for (int r = 0; r < 3; ++r)
            for (int c = 0; c < 3; ++c) {
                double s = 0;
                for (int j = 0; j < 6; ++j) s += Lp[r][j] * Cp[j][c];
                M3[r][c] = s;
            }
        double cond = inv3(M3, Mi);
        if (!(cond < 1e12)) return ORC_E_DEGENERATE;
        for (int r = 0; r < 3; ++r)
            for (int j = 0; j < 6; ++j) {
                double s = 0;
                for (int i = 0; i < 3; ++i) s += Mi[r][i] * Lp[i][j];
                Bm[r][j] = s;
            }
    }
    /* boundary folds, superimposed per missing flap: clamped w_{L+3} = w_L (eq 59), free
       w_{L+3} = w_M + w_N - w_L (eq 61) */
    for (int L = 0; L < 3; ++L) {
        if (!missing[L]) continue;
        int M = (L + 1) % 3, N = (L + 2) % 3, F = L + 3;
        for (int r = 0; r < 3; ++r) {
            if (clampmask & (1 << L)) {
                Bm[r][L] += Bm[r][F];
            } else {
                Bm[r][M] += Bm[r][F];
                Bm[r][N] += Bm[r][F];
                Bm[r][L] -= Bm[r][F];
            }
            Bm[r][F] = 0.0;
        }
    }
    /* FVM free edge: zero the twist (mixed second derivative) in the frame of the first free edge;
       clamped edges keep it */
    if (is_fvm(model)) {
        for (int L = 0; L < 3; ++L) {
            if (!missing[L] || (clampmask & (1 << L))) continue;
            int M = (L + 1) % 3, N = (L + 2) % 3;
            double e[2] = {P[N][0] - P[M][0], P[N][1] - P[M][1]};
            double len = hypot(e[0], e[1]);
            double c = e[0] / len, s = e[1] / len;
            /* Voigt curvature rotation into the edge frame, T(phi), and back, T(-phi) */
            double T[3][3] = {{c * c, s * s, c * s}, {s * s, c * c, -c * s}, {-2 * c * s, 2 * c * s, c * c - s * s}};
            double Ti[3][3] = {{c * c, s * s, -c * s}, {s * s, c * c, c * s}, {2 * c * s, -2 * c * s, c * c - s * s}};
            double Pz[3][3];
            for (int r = 0; r < 3; ++r)
                for (int q = 0; q < 3; ++q) {
                    double acc = 0;
                    for (int m = 0; m < 2; ++m) acc += Ti[r][m] * T[m][q]; /* drop the twist row */
                    Pz[r][q] = acc;
                }
            double Bn[3][6];
            for (int r = 0; r < 3; ++r)
                for (int j = 0; j < 6; ++j) {
                    double acc = 0;
                    for (int q = 0; q < 3; ++q) acc += Pz[r][q] * Bm[q][j];
                    Bn[r][j] = acc;
                }
            memcpy(Bm, Bn, sizeof(Bm));
            break;
        }
    }
    (void)emin;
    double A = 0.5 * twoA;
    for (int r = 0; r < 3; ++r)
        for (int j = 0; j < 6; ++j) B[r * 6 + j] = Bm[r][j];
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) D[r * 3 + c] = A * Db[r][c];
    for (int r = 0; r < 3; ++r) {
        kappa0[r] = 0.0;
        if (is_shell(model)) {
            /* rest curvature kappa0 = B N0^T X (eqs 43, 51) */
            for (int j = 0; j < 6; ++j)
                if (Xs[j]) kappa0[r] += Bm[r][j] * dot3(ez, Xs[j]);
        }
    }
    return ORC_OK;
}

int orc_build(int model, int64_t nv, const double* X, int64_t ns, const int32_t* idx, const uint8_t* bc,
              double young, double poisson, double thickness, int flags, double* B, double* kappa0, double* D,
              double* Crest) {
    if (model < 0 || model > 5 || !X || !idx || !bc || !B || !kappa0 || !D || !Crest) return ORC_E_ARG;
    if ((flags & ~ORC_WORLD_FRAME) || ((flags & ORC_WORLD_FRAME) && !is_edge(model))) return ORC_E_ARG;
    double kb = young * thickness * thickness * thickness / (12.0 * (1.0 - poisson * poisson));
    double Db[3][3] = {{kb, kb * poisson, 0}, {kb * poisson, kb, 0}, {0, 0, kb * (1.0 - poisson) / 2.0}};
    int k = orc_stencil_size(model), r = orc_curv_size(model);
    for (int64_t s = 0; s < ns; ++s) {
        const int32_t* id = idx + k * s;
        int edge_boundary = is_edge(model) && bc[s];
        if (edge_boundary && (is_shell(model) || id[3] >= 0)) return ORC_E_ARG;
        for (int j = 0; j < k; ++j)
            if (id[j] >= nv || (id[j] < 0 && (j < 3 || (is_edge(model) && !edge_boundary)))) return ORC_E_ARG;
        int rc;
        if (is_edge(model)) {
            double Xv[3];
            const double* X4 = X + 3 * id[3];
            if (edge_boundary) {
                /* virtual node: reflection of vertex 1 through the midpoint of the boundary edge 2-3 */
                for (int c = 0; c < 3; ++c) Xv[c] = X[3 * id[1] + c] + X[3 * id[2] + c] - X[3 * id[0] + c];
                X4 = Xv;
            }
            rc = build_edge(is_shell(model), (flags & ORC_WORLD_FRAME) != 0, edge_boundary, X + 3 * id[0],
                            X + 3 * id[1], X + 3 * id[2], X4, kb, B + 4 * s, kappa0 + s, D + s);
        } else {
            const double* Xs[6];
            for (int j = 0; j < 6; ++j) Xs[j] = id[j] >= 0 ? X + 3 * id[j] : NULL;
            rc = build_tri(model, bc[s], Xs, Db, B + 18 * s, kappa0 + 3 * s, D + 9 * s);
        }
        if (rc) return rc;
        /* plate stencil with a clamped edge: its curvature vectors are measured from the rest shape,
           C = B (x - X), since the clamped fold does not annihilate the flat rest coordinates */
        double* Cr = Crest + 3 * r * s;
        for (int q = 0; q < 3 * r; ++q) Cr[q] = 0.0;
        if (!is_shell(model) && bc[s]) {
            const double* Bs = B + (size_t)(r * k) * s;
            for (int i = 0; i < r; ++i)
                for (int j = 0; j < k; ++j)
                    if (id[j] >= 0) axpy3(Bs[i * k + j], X + 3 * id[j], Cr + 3 * i);
        }
    }
    return ORC_OK;
}

/* ------------------------------------------------------ energy and force */

/* (dn/dx_j)^T v for n = u/|u|, u = (b-a)x(c-a) at the triangle's vertices a, b, c:
   w = (I - n n^T) v / |u|, then (du/da)^T w = w x (c-b), (du/db)^T w = w x (a-c),
   (du/dc)^T w = w x (b-a)  (App. B, eqs 67, 73). Adds the results to ga, gb, gc. */
static void normal_vjp(const double* a, const double* b, const double* c, const double* v, double* ga, double* gb,
                       double* gc) {
    double ab[3], ac[3], u[3], n[3];
    sub3(b, a, ab);
    sub3(c, a, ac);
    cross3(ab, ac, u);
    double len = norm3(u);
    scale3(u, 1.0 / len, n);
    double w[3];
    double vn = dot3(v, n);
    for (int i = 0; i < 3; ++i) w[i] = (v[i] - vn * n[i]) / len;
    double cb[3], ca[3], ba[3], t[3];
    sub3(c, b, cb);
    sub3(a, c, ca);
    sub3(b, a, ba);
    cross3(w, cb, t);
    axpy3(1.0, t, ga);
    cross3(w, ca, t);
    axpy3(1.0, t, gb);
    cross3(w, ba, t);
    axpy3(1.0, t, gc);
}

int orc_forces(int model, int64_t nv, const double* x, int64_t ns, const int32_t* idx, const double* B,
               const double* kappa0, const double* Crest, const double* D, double* f, double* energy) {
    if (model < 0 || model > 5 || !x || !f) return ORC_E_ARG;
    int k = orc_stencil_size(model), r = orc_curv_size(model);
    memset(f, 0, sizeof(double) * (size_t)(3 * nv));
    double E = 0.0;
#pragma omp parallel for reduction(+ : E) schedule(static)
    for (int64_t s = 0; s < ns; ++s) {
        const int32_t* id = idx + k * s;
        const double* Bs = B + (size_t)(r * k) * s;
        const double* Ds = D + (size_t)(r * r) * s;
        const double* xs[6];
        for (int j = 0; j < k; ++j) xs[j] = id[j] >= 0 ? x + 3 * id[j] : NULL;
        /* curvature vectors C_i = sum_j B_ij x_j (eqs 13, 40, 47 with N^T applied later) */
        double C[3][3];
        for (int i = 0; i < r; ++i) {
            C[i][0] = C[i][1] = C[i][2] = 0.0;
            for (int j = 0; j < k; ++j)
                if (xs[j]) axpy3(Bs[i * k + j], xs[j], C[i]);
            if (Crest && !is_shell(model)) axpy3(-1.0, Crest + 3 * (r * s + i), C[i]);
        }
        double fs[6][3];
        memset(fs, 0, sizeof(fs));
        if (!is_shell(model)) {
            /* plate: Psi = 1/2 sum_d C_d^T D C_d (eqs 20, 39, 52), f = -H x (eq 22) */
            double DC[3][3];
            for (int i = 0; i < r; ++i)
                for (int d = 0; d < 3; ++d) {
                    double acc = 0;
                    for (int m = 0; m < r; ++m) acc += Ds[i * r + m] * C[m][d];
                    DC[i][d] = acc;
                }
            for (int i = 0; i < r; ++i) E += 0.5 * dot3(C[i], DC[i]);
            for (int j = 0; j < k; ++j)
                for (int i = 0; i < r; ++i) axpy3(-Bs[i * k + j], DC[i], fs[j]);
        } else {
            /* shell: delta = B N^T x - kappa0 (eqs 24, 43, 55), Psi = 1/2 delta^T D delta,
               f_j = -sum_i g_i (B_ij n + (dn/dx_j)^T C_i), g = D delta (eqs 25-26, 44-45, 56-57) */
            double n[3];
            if (is_edge(model)) {
                double na[3], nb[3];
                tri_normal(xs[0], xs[1], xs[2], na);
                tri_normal(xs[3], xs[2], xs[1], nb);
                double m[3] = {na[0] + nb[0], na[1] + nb[1], na[2] + nb[2]};
                scale3(m, 1.0 / norm3(m), n);
            } else {
                tri_normal(xs[0], xs[1], xs[2], n);
            }
            const double* k0 = kappa0 + r * s;
            double delta[3], g[3];
            for (int i = 0; i < r; ++i) delta[i] = dot3(n, C[i]) - k0[i];
            for (int i = 0; i < r; ++i) {
                g[i] = 0;
                for (int m = 0; m < r; ++m) g[i] += Ds[i * r + m] * delta[m];
            }
            for (int i = 0; i < r; ++i) E += 0.5 * delta[i] * g[i];
            double Cg[3] = {0, 0, 0};
            for (int i = 0; i < r; ++i) axpy3(g[i], C[i], Cg);
            for (int j = 0; j < k; ++j) {
                double bj = 0;
                for (int i = 0; i < r; ++i) bj += g[i] * Bs[i * k + j];
                axpy3(-bj, n, fs[j]);
            }
            double gn[6][3];
            memset(gn, 0, sizeof(gn));
            if (is_edge(model)) {
                /* n = m/|m|, m = n_a + n_b: chain through the two unit triangle normals */
                double na[3], nb[3];
                tri_normal(xs[0], xs[1], xs[2], na);
                tri_normal(xs[3], xs[2], xs[1], nb);
                double m[3] = {na[0] + nb[0], na[1] + nb[1], na[2] + nb[2]};
                double mlen = norm3(m);
                double w[3], cn = dot3(Cg, n);
                for (int c = 0; c < 3; ++c) w[c] = (Cg[c] - cn * n[c]) / mlen;
                normal_vjp(xs[0], xs[1], xs[2], w, gn[0], gn[1], gn[2]);
                normal_vjp(xs[3], xs[2], xs[1], w, gn[3], gn[2], gn[1]);
            } else {
                normal_vjp(xs[0], xs[1], xs[2], Cg, gn[0], gn[1], gn[2]);
            }
            for (int j = 0; j < k; ++j) axpy3(-1.0, gn[j], fs[j]);
        }
        for (int j = 0; j < k; ++j)
            if (id[j] >= 0)
                for (int c = 0; c < 3; ++c) {
#pragma omp atomic
                    f[3 * id[j] + c] += fs[j][c];
                }
    }
    if (energy) *energy = E;
    return ORC_OK;
}

/* ------------------------------------------------------ constant Hessian */

typedef struct { int32_t col; double val; } entry_t;

int orc_hessian(int model, int64_t nv, int64_t ns, const int32_t* idx, const double* B, const double* D,
                int64_t* nnz, int64_t* rowptr, int32_t* col, double* val) {
    if (model < 0 || model > 5 || !nnz || !rowptr) return ORC_E_ARG;
    int k = orc_stencil_size(model), r = orc_curv_size(model);
    /* per-row entry counts including duplicates */
    int64_t* cnt = (int64_t*)calloc((size_t)nv + 1, sizeof(int64_t));
    for (int64_t s = 0; s < ns; ++s) {
        const int32_t* id = idx + k * s;
        int present = 0;
        for (int j = 0; j < k; ++j) present += id[j] >= 0;
        for (int j = 0; j < k; ++j)
            if (id[j] >= 0) cnt[id[j] + 1] += present;
    }
    for (int64_t i = 0; i < nv; ++i) cnt[i + 1] += cnt[i];
    entry_t* ent = (entry_t*)malloc(sizeof(entry_t) * (size_t)(cnt[nv] + 1));
    int64_t* fill = (int64_t*)malloc(sizeof(int64_t) * (size_t)(nv + 1));
    memcpy(fill, cnt, sizeof(int64_t) * (size_t)(nv + 1));
    /* stencil Gram blocks G = B^T D B (eqs 21, 41, 53; scalar part of the Kronecker product) */
    for (int64_t s = 0; s < ns; ++s) {
        const int32_t* id = idx + k * s;
        const double* Bs = B + (size_t)(r * k) * s;
        const double* Ds = D + (size_t)(r * r) * s;
        for (int j = 0; j < k; ++j) {
            if (id[j] < 0) continue;
            for (int l = 0; l < k; ++l) {
                if (id[l] < 0) continue;
                double g = 0;
                for (int i = 0; i < r; ++i)
                    for (int m = 0; m < r; ++m) g += Bs[i * k + j] * Ds[i * r + m] * Bs[m * k + l];
                ent[fill[id[j]]].col = id[l];
                ent[fill[id[j]]].val = g;
                fill[id[j]]++;
            }
        }
    }
    /* per row: stable insertion sort by column, then merge duplicates in stencil order */
    int64_t out = 0;
    rowptr[0] = 0;
    for (int64_t i = 0; i < nv; ++i) {
        entry_t* row = ent + cnt[i];
        int64_t len = cnt[i + 1] - cnt[i];
        for (int64_t a = 1; a < len; ++a) {
            entry_t t = row[a];
            int64_t b = a - 1;
            while (b >= 0 && row[b].col > t.col) {
                row[b + 1] = row[b];
                --b;
            }
            row[b + 1] = t;
        }
        for (int64_t a = 0; a < len;) {
            int32_t c = row[a].col;
            double acc = 0;
            while (a < len && row[a].col == c) acc += row[a++].val;
            if (col) {
                col[out] = c;
                val[out] = acc;
            }
            ++out;
        }
        rowptr[i + 1] = out;
    }
    *nnz = out;
    free(cnt);
    free(ent);
    free(fill);
    return ORC_OK;
}

int orc_mass(int64_t nv, const double* X, int64_t nt, const int32_t* tris, double density, double thickness,
             double* mass) {
    if (!X || !tris || !mass) return ORC_E_ARG;
    memset(mass, 0, sizeof(double) * (size_t)nv);
    for (int64_t t = 0; t < nt; ++t) {
        const int32_t* v = tris + 3 * t;
        double n[3];
        double A = 0.5 * tri_normal(X + 3 * v[0], X + 3 * v[1], X + 3 * v[2], n);
        for (int i = 0; i < 3; ++i) mass[v[i]] += density * thickness * A / 3.0;
    }
    return ORC_OK;
}

int orc_apply(int64_t nv, const int64_t* rowptr, const int32_t* col, const double* val, const double* mass,
              double dt2, const double* p, double* q) {
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < nv; ++i) {
        double acc[3] = {0, 0, 0};
        for (int64_t e = rowptr[i]; e < rowptr[i + 1]; ++e) axpy3(val[e], p + 3 * col[e], acc);
        for (int d = 0; d < 3; ++d) q[3 * i + d] = (mass ? mass[i] * p[3 * i + d] : 0.0) + dt2 * acc[d];
    }
    return ORC_OK;
}

/* ------------------------------------------------------ implicit step */

/* one column of (M + dt^2 K_s)_ff y = b by Jacobi-PCG; returns the iteration count */
static int pcg_column(int64_t nv, const int64_t* rowptr, const int32_t* col, const double* val, const double* mass,
                      const uint8_t* pinned, int dcol, double dt2, const double* dinv, const double* b, double* y,
                      double rtol, int max_pcg, int replay_count, int* budget_hit) {
    double *r = (double*)malloc(sizeof(double) * (size_t)nv), *z = (double*)malloc(sizeof(double) * (size_t)nv);
    double *p = (double*)malloc(sizeof(double) * (size_t)nv), *q = (double*)malloc(sizeof(double) * (size_t)nv);
    double bn = 0;
#pragma omp parallel for reduction(+ : bn) schedule(static)
    for (int64_t i = 0; i < nv; ++i) {
        y[i] = 0.0;
        r[i] = held(pinned, i, dcol) ? 0.0 : b[i];
        bn += r[i] * r[i];
    }
    bn = sqrt(bn);
    int target = replay_count >= 0 ? replay_count : max_pcg;
    int it = 0;
    double rz = 0;
#pragma omp parallel for reduction(+ : rz) schedule(static)
    for (int64_t i = 0; i < nv; ++i) {
        z[i] = dinv[i] * r[i];
        p[i] = z[i];
        rz += r[i] * z[i];
    }
    while (it < target) {
        if (replay_count < 0) {
            double rn = 0;
#pragma omp parallel for reduction(+ : rn) schedule(static)
            for (int64_t i = 0; i < nv; ++i) rn += r[i] * r[i];
            if (sqrt(rn) <= rtol * bn) break;
        }
        double pq = 0;
#pragma omp parallel for reduction(+ : pq) schedule(static)
        for (int64_t i = 0; i < nv; ++i) {
            double acc = 0;
            for (int64_t e = rowptr[i]; e < rowptr[i + 1]; ++e) acc += val[e] * p[col[e]];
            q[i] = held(pinned, i, dcol) ? 0.0 : mass[i] * p[i] + dt2 * acc;
            pq += p[i] * q[i];
        }
        double alpha = pq != 0.0 ? rz / pq : 0.0;
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < nv; ++i) {
            y[i] += alpha * p[i];
            r[i] -= alpha * q[i];
        }
        ++it;
        double rz_new = 0;
#pragma omp parallel for reduction(+ : rz_new) schedule(static)
        for (int64_t i = 0; i < nv; ++i) {
            z[i] = dinv[i] * r[i];
            rz_new += r[i] * z[i];
        }
        double beta = rz != 0.0 ? rz_new / rz : 0.0;
        rz = rz_new;
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < nv; ++i) p[i] = z[i] + beta * p[i];
    }
    if (replay_count < 0 && it >= max_pcg) {
        double rn = 0;
        for (int64_t i = 0; i < nv; ++i) rn += r[i] * r[i];
        if (sqrt(rn) > rtol * bn) *budget_hit = 1;
    }
    free(r);
    free(z);
    free(p);
    free(q);
    return it;
}

int orc_step(int model, int64_t nv, int64_t ns, const int32_t* idx, const double* B, const double* kappa0,
             const double* Crest, const double* D, const int64_t* rowptr, const int32_t* col, const double* val, const double* mass,
             const uint8_t* pinned, double* x, double* v, double dt, const double* gravity, int max_newton,
             double newton_rtol, double pcg_rtol, int max_pcg, const int32_t* replay, int32_t* counts, double* stats) {
    if (!x || !v || !mass || !pinned || dt <= 0 || max_newton < 0) return ORC_E_ARG;
    size_t n3 = (size_t)(3 * nv);
    double* xt = (double*)malloc(sizeof(double) * n3);
    double* xhat = (double*)malloc(sizeof(double) * n3);
    double* f = (double*)malloc(sizeof(double) * n3);
    double* g = (double*)malloc(sizeof(double) * n3);
    double* dinv = (double*)malloc(sizeof(double) * (size_t)nv);
    double* bcol = (double*)malloc(sizeof(double) * (size_t)nv);
    double* ycol = (double*)malloc(sizeof(double) * (size_t)nv);
    double dt2 = dt * dt;
    memcpy(xt, x, sizeof(double) * n3);
    /* predictor x_hat = x^t + dt v^t + dt^2 M^-1 f_ext with f_ext = m g (eq 62) */
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < nv; ++i)
        for (int d = 0; d < 3; ++d)
            xhat[3 * i + d] = held(pinned, i, d) ? xt[3 * i + d] : xt[3 * i + d] + dt * v[3 * i + d] + dt2 * gravity[d];
    memcpy(x, xhat, sizeof(double) * n3);
    /* Jacobi preconditioner: inverse diagonal of M_s + dt^2 K_s */
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < nv; ++i) {
        double kii = 0;
        for (int64_t e = rowptr[i]; e < rowptr[i + 1]; ++e)
            if (col[e] == i) kii = val[e];
        dinv[i] = held_all(pinned, i) ? 0.0 : 1.0 / (mass[i] + dt2 * kii);
    }
    int newton = 0, pcg_total = 0, budget_hit = 0;
    double gn0 = 0, gn = 0;
    for (int k = 0;; ++k) {
        /* gradient of the incremental potential, g = M(x - x_hat) - dt^2 f(x), pinned rows zero */
        orc_forces(model, nv, x, ns, idx, B, kappa0, Crest, D, f, NULL);
        double s = 0;
#pragma omp parallel for reduction(+ : s) schedule(static)
        for (int64_t i = 0; i < nv; ++i)
            for (int d = 0; d < 3; ++d) {
                double gi = held(pinned, i, d) ? 0.0 : mass[i] * (x[3 * i + d] - xhat[3 * i + d]) - dt2 * f[3 * i + d];
                g[3 * i + d] = gi;
                s += gi * gi;
            }
        gn = sqrt(s);
        if (k == 0) gn0 = gn;
        if (gn0 == 0.0 || (k > 0 && gn <= newton_rtol * gn0) || k == max_newton) break;
        /* Newton direction against the constant matrix, one PCG per coordinate */
        for (int d = 0; d < 3; ++d) {
#pragma omp parallel for schedule(static)
            for (int64_t i = 0; i < nv; ++i) bcol[i] = -g[3 * i + d];
            int rc_count = replay ? replay[3 * k + d] : -1;
            int it = pcg_column(nv, rowptr, col, val, mass, pinned, d, dt2, dinv, bcol, ycol, pcg_rtol, max_pcg,
                                rc_count, &budget_hit);
            if (counts) counts[3 * k + d] = it;
            pcg_total += it;
#pragma omp parallel for schedule(static)
            for (int64_t i = 0; i < nv; ++i) x[3 * i + d] += ycol[i];
        }
        ++newton;
    }
    for (size_t i = 0; i < n3; ++i) v[i] = (x[i] - xt[i]) / dt;
    if (stats) {
        stats[0] = newton;
        stats[1] = pcg_total;
        stats[2] = gn0;
        stats[3] = gn;
    }
    free(xt);
    free(xhat);
    free(f);
    free(g);
    free(dinv);
    free(bcol);
    free(ycol);
    return budget_hit ? ORC_E_BUDGET : ORC_OK;
}

/* eq 8 as printed: n_c = p/|p| + q/|q| with p = x1 - x_P, q = x4 - x_Q the height vectors
   to the feet on the hinge 2->3 (feet from the current geometry, App. B eqs 70-71) */
/* ------------------------------------------------------ membrane (CST) */

/* Rest frame of a triangle for the constant strain triangle: e1 along X1-X0, e2 = n x e1 in its plane;
   G = Dm^-1 with Dm the 2x2 matrix of the rest edge vectors X1-X0, X2-X0 in (e1, e2); returns the area. */
static double cst_frame(const double* X0, const double* X1, const double* X2, double e1[3], double e2[3],
                        double G[2][2]) {
    double a[3], b[3], n[3];
    sub3(X1, X0, a);
    sub3(X2, X0, b);
    double twoA = tri_normal(X0, X1, X2, n);
    double la = norm3(a);
    scale3(a, 1.0 / la, e1);
    cross3(n, e1, e2);
    double Dm[2][2] = {{dot3(a, e1), dot3(b, e1)}, {dot3(a, e2), dot3(b, e2)}};
    double det = Dm[0][0] * Dm[1][1] - Dm[0][1] * Dm[1][0];
    G[0][0] = Dm[1][1] / det;
    G[0][1] = -Dm[0][1] / det;
    G[1][0] = -Dm[1][0] / det;
    G[1][1] = Dm[0][0] / det;
    return 0.5 * twoA;
}

/* Membrane energy of Sec. 3 (eq 1) on constant strain triangles with the Saint Venant-Kirchhoff model:
   F = Ds Dm^-1 (Ds the current edge vectors x1-x0, x2-x0), Green strain E = (F^T F - I)/2 in Voigt form
   [E11, E22, 2 E12], D_m = h E_el with the plane-stress matrix E_el, Psi_m = A/2 eps^T D_m eps per
   triangle.  The force is -dPsi/dx = -A F S Dm^-T on the edge vectors (S the second Piola-Kirchhoff
   stress from D_m eps), and minus their sum on vertex 0.  Adds into f; *energy receives the sum. */
int orc_membrane(int64_t nv, const double* x, int64_t nt, const int32_t* tris, const double* X, double young,
                 double poisson, double thickness, double* f, double* energy) {
    if (!x || !tris || !X || !f) return ORC_E_ARG;
    double c = young * thickness / (1.0 - poisson * poisson);
    double E = 0.0;
    for (int64_t t = 0; t < nt; ++t) {
        const int32_t* v = tris + 3 * t;
        if (v[0] < 0 || v[1] < 0 || v[2] < 0 || v[0] >= nv || v[1] >= nv || v[2] >= nv) return ORC_E_ARG;
        double e1[3], e2[3], G[2][2];
        double A = cst_frame(X + 3 * v[0], X + 3 * v[1], X + 3 * v[2], e1, e2, G);
        if (!(A > 0)) return ORC_E_DEGENERATE;
        double d1[3], d2[3], F[3][2];
        sub3(x + 3 * v[1], x + 3 * v[0], d1);
        sub3(x + 3 * v[2], x + 3 * v[0], d2);
        for (int i = 0; i < 3; ++i)
            for (int b = 0; b < 2; ++b) F[i][b] = d1[i] * G[0][b] + d2[i] * G[1][b];
        double C[2][2];
        for (int a = 0; a < 2; ++a)
            for (int b = 0; b < 2; ++b) C[a][b] = F[0][a] * F[0][b] + F[1][a] * F[1][b] + F[2][a] * F[2][b];
        double eps[3] = {0.5 * (C[0][0] - 1.0), 0.5 * (C[1][1] - 1.0), C[0][1]};
        double sig[3] = {c * (eps[0] + poisson * eps[1]), c * (poisson * eps[0] + eps[1]),
                         c * 0.5 * (1.0 - poisson) * eps[2]};
        E += 0.5 * A * (eps[0] * sig[0] + eps[1] * sig[1] + eps[2] * sig[2]);
        double S[2][2] = {{sig[0], sig[2]}, {sig[2], sig[1]}};
        /* P = A F S, then dPsi/dDs = P G^T */
        double P[3][2], H[3][2];
        for (int i = 0; i < 3; ++i)
            for (int b = 0; b < 2; ++b) P[i][b] = A * (F[i][0] * S[0][b] + F[i][1] * S[1][b]);
        for (int i = 0; i < 3; ++i)
            for (int k = 0; k < 2; ++k) H[i][k] = P[i][0] * G[k][0] + P[i][1] * G[k][1];
        for (int i = 0; i < 3; ++i) {
            f[3 * v[1] + i] -= H[i][0];
            f[3 * v[2] + i] -= H[i][1];
            f[3 * v[0] + i] += H[i][0] + H[i][1];
        }
    }
    if (energy) *energy = E;
    return ORC_OK;
}

/* Hessian of the membrane energy at the rest shape, per triangle: K = A B^T D_m B (9x9, vertex-major,
   coordinate-minor), B the linear strain of the rest frame, rows [g_j0 e1^T], [g_j1 e2^T],
   [g_j1 e1^T + g_j0 e2^T] for vertex j with shape-function gradient g_j (the stress vanishes at rest, so
   this is the whole Hessian there). */
int orc_membrane_rest_hessian(int64_t nt, const int32_t* tris, const double* X, double young, double poisson,
                              double thickness, double* K9) {
    if (!tris || !X || !K9) return ORC_E_ARG;
    double c = young * thickness / (1.0 - poisson * poisson);
    double Dm[3][3] = {{c, c * poisson, 0}, {c * poisson, c, 0}, {0, 0, c * 0.5 * (1.0 - poisson)}};
    for (int64_t t = 0; t < nt; ++t) {
        const int32_t* v = tris + 3 * t;
        double e1[3], e2[3], G[2][2];
        double A = cst_frame(X + 3 * v[0], X + 3 * v[1], X + 3 * v[2], e1, e2, G);
        if (!(A > 0)) return ORC_E_DEGENERATE;
        double g[3][2] = {{-G[0][0] - G[1][0], -G[0][1] - G[1][1]}, {G[0][0], G[0][1]}, {G[1][0], G[1][1]}};
        double B[3][9];
        for (int j = 0; j < 3; ++j)
            for (int i = 0; i < 3; ++i) {
                B[0][3 * j + i] = g[j][0] * e1[i];
                B[1][3 * j + i] = g[j][1] * e2[i];
                B[2][3 * j + i] = g[j][1] * e1[i] + g[j][0] * e2[i];
            }
        double* K = K9 + 81 * t;
        for (int p = 0; p < 9; ++p)
            for (int q = 0; q < 9; ++q) {
                double acc = 0;
                for (int a = 0; a < 3; ++a)
                    for (int b = 0; b < 3; ++b) acc += B[a][p] * Dm[a][b] * B[b][q];
                K[9 * p + q] = A * acc;
            }
    }
    return ORC_OK;
}

/* Gauss-Newton tangent of the membrane energy at the state x, per triangle: K = A B(F)^T D_m B(F) (9x9,
   vertex-major, coordinate-minor), B(F) the linearised Green strain, rows [g_j0 F0^T], [g_j1 F1^T],
   [g_j1 F0^T + g_j0 F1^T] for vertex j (F0, F1 the columns of F); positive semi-definite, and the rest
   Hessian at x = X. */
int orc_membrane_gn_hessian(int64_t nt, const int32_t* tris, const double* X, const double* x, double young,
                            double poisson, double thickness, double* K9) {
    if (!tris || !X || !x || !K9) return ORC_E_ARG;
    double c = young * thickness / (1.0 - poisson * poisson);
    double Dm[3][3] = {{c, c * poisson, 0}, {c * poisson, c, 0}, {0, 0, c * 0.5 * (1.0 - poisson)}};
    for (int64_t t = 0; t < nt; ++t) {
        const int32_t* v = tris + 3 * t;
        double e1[3], e2[3], G[2][2];
        double A = cst_frame(X + 3 * v[0], X + 3 * v[1], X + 3 * v[2], e1, e2, G);
        if (!(A > 0)) return ORC_E_DEGENERATE;
        double d1[3], d2[3], F[3][2];
        sub3(x + 3 * v[1], x + 3 * v[0], d1);
        sub3(x + 3 * v[2], x + 3 * v[0], d2);
        for (int i = 0; i < 3; ++i)
            for (int b = 0; b < 2; ++b) F[i][b] = d1[i] * G[0][b] + d2[i] * G[1][b];
        double g[3][2] = {{-G[0][0] - G[1][0], -G[0][1] - G[1][1]}, {G[0][0], G[0][1]}, {G[1][0], G[1][1]}};
        double Bm[3][9];
        for (int j = 0; j < 3; ++j)
            for (int i = 0; i < 3; ++i) {
                Bm[0][3 * j + i] = g[j][0] * F[i][0];
                Bm[1][3 * j + i] = g[j][1] * F[i][1];
                Bm[2][3 * j + i] = g[j][1] * F[i][0] + g[j][0] * F[i][1];
            }
        double* K = K9 + 81 * t;
        for (int p = 0; p < 9; ++p)
            for (int q = 0; q < 9; ++q) {
                double acc = 0;
                for (int a = 0; a < 3; ++a)
                    for (int b = 0; b < 3; ++b) acc += Bm[a][p] * Dm[a][b] * Bm[b][q];
                K[9 * p + q] = A * acc;
            }
    }
    return ORC_OK;
}

/* One Jacobi-PCG over all 3 nv coordinates for (M + dt^2 (K_s (x) I3 + K9)) y = -g, y0 = 0 (mass NULL: no
   mass term); the per-triangle blocks K9 are applied triangle by triangle.  Stops when ||r|| <= rtol ||b||
   (or after exactly replay_count iterations when that is >= 0); sets *budget_hit when max_pcg ran out.
   r, z, p, q: work vectors [3 nv].  Returns the iteration count. */
static int coupled_pcg(int64_t nv, const int64_t* rowptr, const int32_t* col, const double* val, int64_t nt,
                       const int32_t* tris, const double* K9, const double* mass, const uint8_t* pinned, double dt2,
                       const double* dinv, const double* g, double* y, double rtol, int max_pcg, int replay_count,
                       int* budget_hit, double* r, double* z, double* p, double* q) {
    size_t n3 = (size_t)(3 * nv);
    double bn = 0, rz = 0;
    for (size_t i = 0; i < n3; ++i) {
        y[i] = 0.0;
        r[i] = -g[i];
        bn += r[i] * r[i];
        z[i] = dinv[i / 3] * r[i];
        p[i] = z[i];
        rz += r[i] * z[i];
    }
    bn = sqrt(bn);
    int target = replay_count >= 0 ? replay_count : max_pcg, it = 0;
    while (it < target) {
        if (replay_count < 0) {
            double rn = 0;
            for (size_t i = 0; i < n3; ++i) rn += r[i] * r[i];
            if (sqrt(rn) <= rtol * bn) break;
        }
        for (int64_t i = 0; i < nv; ++i) {
            double acc[3] = {0, 0, 0};
            for (int64_t e = rowptr[i]; e < rowptr[i + 1]; ++e) axpy3(val[e], p + 3 * col[e], acc);
            for (int d = 0; d < 3; ++d) q[3 * i + d] = (mass ? mass[i] * p[3 * i + d] : 0.0) + dt2 * acc[d];
        }
        for (int64_t t = 0; t < nt; ++t) {
            const int32_t* tv = tris + 3 * t;
            const double* K = K9 + 81 * t;
            for (int a = 0; a < 9; ++a) {
                double acc = 0;
                for (int b = 0; b < 9; ++b) acc += K[9 * a + b] * p[3 * tv[b / 3] + b % 3];
                q[3 * tv[a / 3] + a % 3] += dt2 * acc;
            }
        }
        double pq = 0;
        for (int64_t i = 0; i < nv; ++i)
            for (int d = 0; d < 3; ++d) {
                if (held(pinned, i, d)) q[3 * i + d] = 0.0;
                pq += p[3 * i + d] * q[3 * i + d];
            }
        double alpha = pq != 0.0 ? rz / pq : 0.0;
        double rz_new = 0;
        for (size_t i = 0; i < n3; ++i) {
            y[i] += alpha * p[i];
            r[i] -= alpha * q[i];
            z[i] = dinv[i / 3] * r[i];
            rz_new += r[i] * z[i];
        }
        double beta = rz != 0.0 ? rz_new / rz : 0.0;
        rz = rz_new;
        for (size_t i = 0; i < n3; ++i) p[i] = z[i] + beta * p[i];
        ++it;
    }
    if (replay_count < 0 && it >= max_pcg) {
        double rn = 0;
        for (size_t i = 0; i < n3; ++i) rn += r[i] * r[i];
        if (sqrt(rn) > rtol * bn) *budget_hit = 1;
    }
    return it;
}

/* Jacobi diagonal of M + dt^2 (K_s (x) I3 + K9): 1/(m + dt^2 (K_s,ii + tr(K9_ii)/3)) per vertex, 0 on fixed
   rows and rows without stiffness (mass NULL: no mass term) */
static void coupled_dinv(int64_t nv, const int64_t* rowptr, const int32_t* col, const double* val, int64_t nt,
                         const int32_t* tris, const double* K9, const double* mass, const uint8_t* pinned, double dt2,
                         double* dinv) {
    for (int64_t i = 0; i < nv; ++i) {
        double kii = 0;
        for (int64_t e = rowptr[i]; e < rowptr[i + 1]; ++e)
            if (col[e] == i) kii = val[e];
        dinv[i] = kii;
    }
    for (int64_t t = 0; t < nt; ++t)
        for (int j = 0; j < 3; ++j)
            for (int d = 0; d < 3; ++d) dinv[tris[3 * t + j]] += K9[81 * t + (3 * j + d) * 9 + 3 * j + d] / 3.0;
    for (int64_t i = 0; i < nv; ++i) {
        double den = (mass ? mass[i] : 0.0) + dt2 * dinv[i];
        dinv[i] = (held_all(pinned, i) || den == 0.0) ? 0.0 : 1.0 / den;
    }
}

/* Membrane tangent used by the solvers: the Gauss-Newton part plus the stress (geometric) part of the
   exact Hessian, A (g_a^T S g_b) I3 for the vertex pair (a, b) with g the shape-function gradients and S
   the second Piola-Kirchhoff stress, with S replaced by its positive semi-definite part (negative
   principal stresses dropped).  Under tension this is the exact Hessian of the membrane energy; under
   compression it is the Gauss-Newton tangent; it is PSD throughout.  K9 [nt][9][9] as above. */
int orc_membrane_tangent(int64_t nt, const int32_t* tris, const double* X, const double* x, double young,
                         double poisson, double thickness, double* K9) {
    int rc = orc_membrane_gn_hessian(nt, tris, X, x, young, poisson, thickness, K9);
    if (rc) return rc;
    double c = young * thickness / (1.0 - poisson * poisson);
    for (int64_t t = 0; t < nt; ++t) {
        const int32_t* v = tris + 3 * t;
        double e1[3], e2[3], G[2][2];
        double A = cst_frame(X + 3 * v[0], X + 3 * v[1], X + 3 * v[2], e1, e2, G);
        double d1[3], d2[3], F[3][2];
        sub3(x + 3 * v[1], x + 3 * v[0], d1);
        sub3(x + 3 * v[2], x + 3 * v[0], d2);
        for (int i = 0; i < 3; ++i)
            for (int b = 0; b < 2; ++b) F[i][b] = d1[i] * G[0][b] + d2[i] * G[1][b];
        double C[2][2];
        for (int a = 0; a < 2; ++a)
            for (int b = 0; b < 2; ++b) C[a][b] = F[0][a] * F[0][b] + F[1][a] * F[1][b] + F[2][a] * F[2][b];
        double eps[3] = {0.5 * (C[0][0] - 1.0), 0.5 * (C[1][1] - 1.0), C[0][1]};
        double s11 = c * (eps[0] + poisson * eps[1]), s22 = c * (poisson * eps[0] + eps[1]);
        double s12 = c * 0.5 * (1.0 - poisson) * eps[2];
        /* positive part of the 2x2 stress from its principal values l1 >= l2 */
        double mean = 0.5 * (s11 + s22), half = 0.5 * (s11 - s22);
        double rad = sqrt(half * half + s12 * s12);
        double l1 = mean + rad, l2 = mean - rad;
        double P[2][2];
        if (l2 >= 0.0) {
            P[0][0] = s11;
            P[0][1] = P[1][0] = s12;
            P[1][1] = s22;
        } else if (l1 <= 0.0) {
            P[0][0] = P[0][1] = P[1][0] = P[1][1] = 0.0;
        } else {
            /* l1 v v^T with v v^T = (S - l2 I) / (l1 - l2) */
            double w = l1 / (l1 - l2);
            P[0][0] = w * (s11 - l2);
            P[0][1] = P[1][0] = w * s12;
            P[1][1] = w * (s22 - l2);
        }
        double g[3][2] = {{-G[0][0] - G[1][0], -G[0][1] - G[1][1]}, {G[0][0], G[0][1]}, {G[1][0], G[1][1]}};
        double* K = K9 + 81 * t;
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) {
                double gsg = 0;
                for (int p = 0; p < 2; ++p)
                    for (int q = 0; q < 2; ++q) gsg += g[a][p] * P[p][q] * g[b][q];
                for (int i = 0; i < 3; ++i) K[9 * (3 * a + i) + 3 * b + i] += A * gsg;
            }
    }
    return ORC_OK;
}

/* incremental potential of the step with the membrane: 1/2 (x - x_hat)^T M (x - x_hat) + dt^2 (Psi_b + Psi_m);
   also returns the total force (bending plus membrane) in f */
static double membrane_step_energy(int model, int64_t nv, const double* x, int64_t ns, const int32_t* idx,
                                   const double* B, const double* kappa0, const double* Crest, const double* D,
                                   int64_t nt, const int32_t* tris, const double* X, double young, double poisson,
                                   double thickness, const double* mass, const double* xhat, double dt2,
                                   double* f) {
    double eb = 0, em = 0, ei = 0;
    orc_forces(model, nv, x, ns, idx, B, kappa0, Crest, D, f, &eb);
    orc_membrane(nv, x, nt, tris, X, young, poisson, thickness, f, &em);
    for (int64_t i = 0; i < nv; ++i)
        for (int d = 0; d < 3; ++d) {
            double u = x[3 * i + d] - xhat[3 * i + d];
            ei += 0.5 * mass[i] * u * u;
        }
    return ei + dt2 * (eb + em);
}

/* One implicit-Euler step (eq 62) of the shell with its membrane.  Each Newton iteration solves
   (M + dt^2 (K_s (x) I3 + K_GN(x))) y = -g by one Jacobi-PCG over all 3 nv coordinates (the membrane
   couples them; the preconditioner is 1/(m + dt^2 (K_s,ii + tr(K_GN,ii)/3)) per vertex), then takes
   x += 2^-h y with h the fewest halvings (at most 6) that satisfy Armijo's condition
   E(x + a y) <= E(x) + 1e-4 a g.y on the incremental potential E.  replay_pcg / replay_halvings
   [max_newton] (may be NULL) fix the iteration counts and the halvings; counts and halvings
   [max_newton] receive them. */
int orc_step_membrane(int model, int64_t nv, int64_t ns, const int32_t* idx, const double* B, const double* kappa0,
                      const double* Crest, const double* D, const int64_t* rowptr, const int32_t* col,
                      const double* val, int64_t nt, const int32_t* tris, const double* X, double young,
                      double poisson, double thickness, const double* mass, const uint8_t* pinned, double* x,
                      double* v, double dt, const double* gravity, int max_newton, double newton_rtol,
                      double pcg_rtol, int max_pcg, const int32_t* replay_pcg, const int32_t* replay_halvings,
                      int32_t* counts, int32_t* halvings, double* stats) {
    if (!x || !v || !mass || !pinned || dt <= 0 || max_newton < 0) return ORC_E_ARG;
    size_t n3 = (size_t)(3 * nv);
    double* xt = (double*)malloc(sizeof(double) * n3);
    double* xhat = (double*)malloc(sizeof(double) * n3);
    double* xtry = (double*)malloc(sizeof(double) * n3);
    double* f = (double*)malloc(sizeof(double) * n3);
    double* g = (double*)malloc(sizeof(double) * n3);
    double* r = (double*)malloc(sizeof(double) * n3);
    double* z = (double*)malloc(sizeof(double) * n3);
    double* p = (double*)malloc(sizeof(double) * n3);
    double* q = (double*)malloc(sizeof(double) * n3);
    double* y = (double*)malloc(sizeof(double) * n3);
    double* dinv = (double*)malloc(sizeof(double) * (size_t)nv);
    double* K9 = (double*)malloc(sizeof(double) * (size_t)(81 * nt + 1));
    double dt2 = dt * dt;
    memcpy(xt, x, sizeof(double) * n3);
    for (int64_t i = 0; i < nv; ++i)
        for (int d = 0; d < 3; ++d)
            xhat[3 * i + d] = held(pinned, i, d) ? xt[3 * i + d] : xt[3 * i + d] + dt * v[3 * i + d] + dt2 * gravity[d];
    memcpy(x, xhat, sizeof(double) * n3);
    int newton = 0, pcg_total = 0, budget_hit = 0, rc = ORC_OK;
    double gn0 = 0, gn = 0;
    double E = membrane_step_energy(model, nv, x, ns, idx, B, kappa0, Crest, D, nt, tris, X, young, poisson,
                                    thickness, mass, xhat, dt2, f);
    for (int k = 0;; ++k) {
        double s2 = 0;
        for (int64_t i = 0; i < nv; ++i)
            for (int d = 0; d < 3; ++d) {
                double gi = held(pinned, i, d) ? 0.0 : mass[i] * (x[3 * i + d] - xhat[3 * i + d]) - dt2 * f[3 * i + d];
                g[3 * i + d] = gi;
                s2 += gi * gi;
            }
        gn = sqrt(s2);
        if (k == 0) gn0 = gn;
        if (gn0 == 0.0 || (k > 0 && gn <= newton_rtol * gn0) || k == max_newton) break;
        rc = orc_membrane_tangent(nt, tris, X, x, young, poisson, thickness, K9);
        if (rc) break;
        coupled_dinv(nv, rowptr, col, val, nt, tris, K9, mass, pinned, dt2, dinv);
        int it = coupled_pcg(nv, rowptr, col, val, nt, tris, K9, mass, pinned, dt2, dinv, g, y, pcg_rtol, max_pcg,
                             replay_pcg ? replay_pcg[k] : -1, &budget_hit, r, z, p, q);
        if (counts) counts[k] = it;
        pcg_total += it;
        /* backtracking line search on the incremental potential */
        double slope = 0;
        for (size_t i = 0; i < n3; ++i) slope += g[i] * y[i];
        int h = 0;
        double a = 1.0, Etry = 0;
        for (;;) {
            for (size_t i = 0; i < n3; ++i) xtry[i] = x[i] + a * y[i];
            Etry = membrane_step_energy(model, nv, xtry, ns, idx, B, kappa0, Crest, D, nt, tris, X, young, poisson,
                                        thickness, mass, xhat, dt2, f);
            int done = replay_halvings ? (h >= replay_halvings[k]) : (Etry <= E + 1e-4 * a * slope || h == 6);
            if (done) break;
            a *= 0.5;
            ++h;
        }
        if (halvings) halvings[k] = h;
        memcpy(x, xtry, sizeof(double) * n3);
        E = Etry;  /* f already holds the force at the new x */
        ++newton;
    }
    for (size_t i = 0; i < n3; ++i) v[i] = (x[i] - xt[i]) / dt;
    if (stats) {
        stats[0] = newton;
        stats[1] = pcg_total;
        stats[2] = gn0;
        stats[3] = gn;
    }
    free(xt);
    free(xhat);
    free(xtry);
    free(f);
    free(g);
    free(r);
    free(z);
    free(p);
    free(q);
    free(y);
    free(dinv);
    free(K9);
    if (rc) return rc;
    return budget_hit ? ORC_E_BUDGET : ORC_OK;
}

/* Quasi-static equilibrium of the shell with its membrane (eq 64 with Psi_shell = Psi_b + Psi_m):
   Newton-Raphson on r = dPsi_shell/dx - F (fixed rows zero) with the matrix K_s (x) I3 + K_GN(x), one
   coupled Jacobi-PCG per iteration, the increment scaled by eps_u/||dx||_inf when that exceeds eps_u > 0;
   stop when ||r|| < eps_f or after max_newton solves.  replay/counts [max_newton] (one PCG per solve). */
int orc_static_membrane(int model, int64_t nv, int64_t ns, const int32_t* idx, const double* B,
                        const double* kappa0, const double* Crest, const double* D, const int64_t* rowptr,
                        const int32_t* col, const double* val, int64_t nt, const int32_t* tris, const double* X,
                        double young, double poisson, double thickness, const uint8_t* pinned, const double* load,
                        double* x, double eps_f, double eps_u, int max_newton, double pcg_rtol, int max_pcg,
                        const int32_t* replay, int32_t* counts, double* stats) {
    if (!x || !pinned || max_newton < 0) return ORC_E_ARG;
    size_t n3 = (size_t)(3 * nv);
    double* f = (double*)malloc(sizeof(double) * n3);
    double* g = (double*)malloc(sizeof(double) * n3);
    double* y = (double*)malloc(sizeof(double) * n3);
    double* r = (double*)malloc(sizeof(double) * n3);
    double* z = (double*)malloc(sizeof(double) * n3);
    double* p = (double*)malloc(sizeof(double) * n3);
    double* q = (double*)malloc(sizeof(double) * n3);
    double* dinv = (double*)malloc(sizeof(double) * (size_t)nv);
    double* K9 = (double*)malloc(sizeof(double) * (size_t)(81 * nt + 1));
    int newton = 0, pcg_total = 0, budget_hit = 0, rc = ORC_OK;
    double rn0 = 0, rn = 0;
    for (int k = 0;; ++k) {
        orc_forces(model, nv, x, ns, idx, B, kappa0, Crest, D, f, NULL);
        orc_membrane(nv, x, nt, tris, X, young, poisson, thickness, f, NULL);
        double s2 = 0;
        for (int64_t i = 0; i < nv; ++i)
            for (int d = 0; d < 3; ++d) {
                double gi = held(pinned, i, d) ? 0.0 : -f[3 * i + d] - (load ? load[3 * i + d] : 0.0);
                g[3 * i + d] = gi;
                s2 += gi * gi;
            }
        rn = sqrt(s2);
        if (k == 0) rn0 = rn;
        if (rn == 0.0 || rn < eps_f || k == max_newton) break;
        rc = orc_membrane_tangent(nt, tris, X, x, young, poisson, thickness, K9);
        if (rc) break;
        coupled_dinv(nv, rowptr, col, val, nt, tris, K9, NULL, pinned, 1.0, dinv);
        int it = coupled_pcg(nv, rowptr, col, val, nt, tris, K9, NULL, pinned, 1.0, dinv, g, y, pcg_rtol, max_pcg,
                             replay ? replay[k] : -1, &budget_hit, r, z, p, q);
        if (counts) counts[k] = it;
        pcg_total += it;
        double dmax = 0;
        for (size_t i = 0; i < n3; ++i) dmax = fmax(dmax, fabs(y[i]));
        double scale = (eps_u > 0.0 && dmax > eps_u) ? eps_u / dmax : 1.0;
        for (size_t i = 0; i < n3; ++i) x[i] += scale * y[i];
        ++newton;
    }
    if (stats) {
        stats[0] = newton;
        stats[1] = pcg_total;
        stats[2] = rn0;
        stats[3] = rn;
    }
    free(f);
    free(g);
    free(y);
    free(r);
    free(z);
    free(p);
    free(q);
    free(dinv);
    free(K9);
    if (rc) return rc;
    return budget_hit ? ORC_E_BUDGET : ORC_OK;
}

/* Quasi-static equilibrium (Sec. 5, eq 64) by Newton-Raphson in one load step: the residual
   r = dPsi/dx - F (F the applied load, the bending force f = -dPsi/dx, fixed rows zero) is driven below
   eps_f; each iteration solves K dx = -r against the constant Hessian (one Jacobi-PCG per coordinate, no
   mass term) and, when ||dx||_inf exceeds eps_u > 0, scales dx by eps_u/||dx||_inf before x += dx. */
int orc_static(int model, int64_t nv, int64_t ns, const int32_t* idx, const double* B, const double* kappa0,
               const double* Crest, const double* D, const int64_t* rowptr, const int32_t* col, const double* val,
               const uint8_t* pinned, const double* load, double* x, double eps_f, double eps_u, int max_newton,
               double pcg_rtol, int max_pcg, const int32_t* replay, int32_t* counts, double* stats) {
    if (!x || !pinned || max_newton < 0) return ORC_E_ARG;
    size_t n3 = (size_t)(3 * nv);
    double* f = (double*)malloc(sizeof(double) * n3);
    double* r = (double*)malloc(sizeof(double) * n3);
    double* dx = (double*)malloc(sizeof(double) * n3);
    double* zero = (double*)calloc((size_t)nv + 1, sizeof(double));
    double* dinv = (double*)malloc(sizeof(double) * (size_t)nv);
    double* bcol = (double*)malloc(sizeof(double) * (size_t)nv);
    double* ycol = (double*)malloc(sizeof(double) * (size_t)nv);
    /* Jacobi preconditioner of K_s alone */
    for (int64_t i = 0; i < nv; ++i) {
        double kii = 0;
        for (int64_t e = rowptr[i]; e < rowptr[i + 1]; ++e)
            if (col[e] == i) kii = val[e];
        dinv[i] = (held_all(pinned, i) || kii == 0.0) ? 0.0 : 1.0 / kii;
    }
    int newton = 0, pcg_total = 0, budget_hit = 0;
    double rn0 = 0, rn = 0;
    for (int k = 0;; ++k) {
        orc_forces(model, nv, x, ns, idx, B, kappa0, Crest, D, f, NULL);
        double s2 = 0;
        for (int64_t i = 0; i < nv; ++i)
            for (int d = 0; d < 3; ++d) {
                double ri = held(pinned, i, d) ? 0.0 : -f[3 * i + d] - (load ? load[3 * i + d] : 0.0);
                r[3 * i + d] = ri;
                s2 += ri * ri;
            }
        rn = sqrt(s2);
        if (k == 0) rn0 = rn;
        if (rn == 0.0 || rn < eps_f || k == max_newton) break;
        for (int d = 0; d < 3; ++d) {
            for (int64_t i = 0; i < nv; ++i) bcol[i] = -r[3 * i + d];
            int it = pcg_column(nv, rowptr, col, val, zero, pinned, d, 1.0, dinv, bcol, ycol, pcg_rtol, max_pcg,
                                replay ? replay[3 * k + d] : -1, &budget_hit);
            if (counts) counts[3 * k + d] = it;
            pcg_total += it;
            for (int64_t i = 0; i < nv; ++i) dx[3 * i + d] = ycol[i];
        }
        /* incremental displacement limit */
        double dmax = 0;
        for (size_t i = 0; i < n3; ++i) dmax = fmax(dmax, fabs(dx[i]));
        double scale = (eps_u > 0.0 && dmax > eps_u) ? eps_u / dmax : 1.0;
        for (size_t i = 0; i < n3; ++i) x[i] += scale * dx[i];
        ++newton;
    }
    if (stats) {
        stats[0] = newton;
        stats[1] = pcg_total;
        stats[2] = rn0;
        stats[3] = rn;
    }
    free(f);
    free(r);
    free(dx);
    free(zero);
    free(dinv);
    free(bcol);
    free(ycol);
    return budget_hit ? ORC_E_BUDGET : ORC_OK;
}

int orc_edge_normal_literal(const double* x1, const double* x2, const double* x3, const double* x4, double* n) {
    double e[3], d1[3], d4[3], p[3], q[3];
    sub3(x3, x2, e);
    sub3(x1, x2, d1);
    sub3(x4, x2, d4);
    double ee = dot3(e, e);
    double sp = dot3(d1, e) / ee, sq = dot3(d4, e) / ee;
    for (int c = 0; c < 3; ++c) {
        p[c] = d1[c] - sp * e[c];
        q[c] = d4[c] - sq * e[c];
    }
    double pl = norm3(p), ql = norm3(q);
    double m[3];
    for (int c = 0; c < 3; ++c) m[c] = p[c] / pl + q[c] / ql;
    double ml = norm3(m);
    if (!(ml > 0)) return ORC_E_DEGENERATE;
    scale3(m, 1.0 / ml, n);
    return ORC_OK;
}

int orc_threads(int n) {
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
    return omp_get_max_threads();
#else
    (void)n;
    return 1;
#endif
}
