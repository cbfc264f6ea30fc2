// Per-stencil bending forces, the per-timestep hot kernel.
//
// Layout: vertices are numbered in tiles of T consecutive ids (compact surface patches).  One
// work-group owns one tile and walks the list of every stencil that touches the tile (stencils on a
// tile boundary appear in each tile they touch).  Each stencil's force on the tile's own vertices is
// added into a float64 LDS accumulator; contributions to other tiles' vertices are left to those
// tiles.  The tile is then written to HBM once: no global atomics, no zero-fill, one coalesced store
// per vertex.  The accumulation is exact in fixed-point parts (TileAcc), so its result does not depend
// on the order in which the waves add.  Stencil data is streamed in blocks of 64 stencils, in 16-byte chunks of fields (a
// wave's 64 loads of one chunk are one contiguous 1 KB run, so every load is coalesced and a wave
// touches one region of memory); a tile's list stays in spatial order so the gathers of one wave touch
// few cache lines.
//
// Per stencil (operator B already scaled by the square root of its stiffness):
//   C_i = sum_j B_ij (x_j - x_o)            curvature vectors, x_o the stencil origin (rows of B
//                                          sum to zero, so local differences give the same C)
//   plate: f_j = -sum_i B_ij (D C)_i                          eqs 20-22, 39-41, 52-53
//   shell: delta = n.C - kappa0, g = D delta,
//          f_j = -(sum_i g_i B_ij) n - (dn/dx_j)^T sum_i g_i C_i   eqs 24-26, 43-45, 55-57
// with D = 1 (edge) or D_b / k_b-form [[1,nu,0],[nu,1,0],[0,0,(1-nu)/2]] * k_b (triangle), n the
// unit normal of the central triangle (eq 15) or the bisector of the two hinge triangle normals
// (edge; the line of eq 8), its gradient by the chain rule of App. B (eqs 67, 73).
//
// Mixed precision.  The positions are gathered in float64 and differenced in float64; what float32
// rounds is chosen so that it never cancels against the size of an edge:
//  - shells take the bending strain from the heights h_j = (x_j - x_o) . n over the current normal
//    (float64 dot products with the float32 normal): delta = B~ h - kappa0~, summed in float64, with B~
//    the float32 operator and kappa0~ = B~ h0 the rest curvature of that same rounded operator (float64,
//    computed at build time).  The normal is renormalised in float64; its remaining direction error adds a
//    linear function of the positions to h, which B annihilates up to the tangential part of the
//    curvature vectors (eq 12's argument), so delta stays accurate whatever the rigid motion or the size of
//    the stencil, also near the rest shape where it is small.  The curvature vectors C = B~ (x_j - x_o) and the normal gradient (which
//    meet only g = D delta, and the tangent plane) are float32.
//  - plates remove the stencil's affine part before rounding: the map A that carries the rest edges of
//    the central triangle (edge stencils: of the first hinge triangle, in the rest tangent plane) onto
//    the current ones is applied in float64, and C = sum_j B~_j (x_j - x_o - A (X_j - X_o)) over the
//    flaps, the only vertices where that difference is not zero.  B annihilates affine fields of the
//    rest stencil (eqs 12, 49), so this is B x^e, and float32 now rounds the deformation of the stencil
//    instead of its position, also under rotations.  Triangle plates gather the rest positions and
//    solve for A's coefficients in float64; the edge plate reads its tip's two coefficients from its
//    record.  Plate stencils with a clamped edge are rest-relative, C = B~ (u_j - u_o), u = x - X.
// After that everything is float32, with float64 tile accumulation.
#include <hip/hip_ext.h>

#include <algorithm>

#include "devmath.hpp"
#include "internal.hpp"

namespace shell {

namespace {

// Normal of an edge stencil (vertices 0-3, hinge 1-2) from a = x0 - x1, c = x2 - x1, b = x3 - x1: the two
// hinge triangles' unit normals and their normalised bisector.
template <typename R>
struct EdgeFrame {
    V3<R> na, nb, n;
    R ila, ilb, ilm;
};
template <typename R>
__device__ __forceinline__ EdgeFrame<R> edge_frame(V3<R> a, V3<R> c, V3<R> b) {
    EdgeFrame<R> e;
    const V3<R> ua = cross(c, a), ub = cross(b, c);
    e.ila = inv_norm(ua);
    e.ilb = inv_norm(ub);
    e.na = e.ila * ua;
    e.nb = e.ilb * ub;
    const V3<R> m = e.na + e.nb;
    e.ilm = inv_norm(m);
    e.n = e.ilm * m;
    return e;
}

// Edge stencil force from the curvature vector C = sum_j L_j x_j and, for shells, the bending strain
// delta and the frame.
template <typename R, bool SHELL>
__device__ __forceinline__ void edge_force(V3<R> a, V3<R> c, V3<R> b, V3<R> C, const R (&L)[4],
                                           const EdgeFrame<R>& e, R delta, V3<R> (&f)[4], R& energy) {
    if constexpr (!SHELL) {
        energy = R(0.5) * dot(C, C);
#pragma unroll
        for (int j = 0; j < 4; ++j) f[j] = (-L[j]) * C;
    } else {
        energy = R(0.5) * delta * delta;
        // w = (I - n n^T) C / |m|, then through each unit triangle normal
        const V3<R> w = e.ilm * (C - dot(C, e.n) * e.n);
        const V3<R> wa = e.ila * (w - dot(w, e.na) * e.na);
        const V3<R> wb = e.ilb * (w - dot(w, e.nb) * e.nb);
        const V3<R> g1 = cross(wa, c);
        const V3<R> g2 = cross(wa, a - c) + cross(wb, c - b);
        const V3<R> g3 = cross(wb, b) - cross(wa, a);
        const V3<R> g4 = cross(c, wb);
        f[0] = (-delta) * (L[0] * e.n + g1);
        f[1] = (-delta) * (L[1] * e.n + g2);
        f[2] = (-delta) * (L[2] * e.n + g3);
        f[3] = (-delta) * (L[3] * e.n + g4);
    }
}

// Triangle stencil force from the differences d_j = x_j - x_0 (d_0 = 0), the curvature vectors
// C_i = sum_j B_ij x_j and, for shells, the bending strain de_i and the central triangle's unit normal n
// with 1/|d_1 x d_2|.
template <typename R, bool SHELL>
__device__ __forceinline__ void tri_force(const V3<R> (&d)[6], const V3<R> (&C)[3], const R (&B)[3][6],
                                          const R (&de)[3], V3<R> n, R ilu, R kb, R nu, V3<R> (&f)[6],
                                          R& energy) {
    const R t = R(0.5) * (R(1) - nu);
    if constexpr (!SHELL) {
        V3<R> DC[3];
        DC[0] = kb * (C[0] + nu * C[1]);
        DC[1] = kb * (nu * C[0] + C[1]);
        DC[2] = (kb * t) * C[2];
        energy = R(0.5) * (dot(C[0], DC[0]) + dot(C[1], DC[1]) + dot(C[2], DC[2]));
#pragma unroll
        for (int j = 0; j < 6; ++j) {
            V3<R> fj = (-B[0][j]) * DC[0];
            fma3(fj, -B[1][j], DC[1]);
            fma3(fj, -B[2][j], DC[2]);
            f[j] = fj;
        }
    } else {
        const R g0 = kb * (de[0] + nu * de[1]), g1 = kb * (nu * de[0] + de[1]), g2 = kb * t * de[2];
        energy = R(0.5) * (de[0] * g0 + de[1] * g1 + de[2] * g2);
        V3<R> Cg = g0 * C[0];
        fma3(Cg, g1, C[1]);
        fma3(Cg, g2, C[2]);
        const V3<R> w = ilu * (Cg - dot(Cg, n) * n);
#pragma unroll
        for (int j = 0; j < 6; ++j) {
            const R bj = g0 * B[0][j] + g1 * B[1][j] + g2 * B[2][j];
            f[j] = (-bj) * n;
        }
        // (du/dx1)^T w = w x (x3 - x2), (du/dx2)^T w = w x (x1 - x3), (du/dx3)^T w = w x (x2 - x1)
        f[0] = f[0] - cross(w, d[2] - d[1]);
        f[1] = f[1] - cross(d[2], w);
        f[2] = f[2] - cross(w, d[1]);
    }
}

// Coefficients (a, b) of the projection of v on the plane of e1, e2: v ~ a e1 + b e2 (float64 normal
// equations of the 2 x 2 Gram system).
struct Plane2 {
    double g11, g12, g22, idet;
    __device__ __forceinline__ Plane2(V3<double> e1, V3<double> e2) {
        g11 = dot(e1, e1);
        g12 = dot(e1, e2);
        g22 = dot(e2, e2);
        idet = inv_fast(g11 * g22 - g12 * g12);
    }
    __device__ __forceinline__ void coords(V3<double> e1, V3<double> e2, V3<double> v, double& a, double& b) const {
        const double r1 = dot(e1, v), r2 = dot(e2, v);
        a = (g22 * r1 - g12 * r2) * idet;
        b = (g11 * r2 - g12 * r1) * idet;
    }
};

// 16-byte stream chunks (clang vector types, which load through address-space pointers in one
// instruction).  The streams are read with non-temporal loads, which keep them from displacing the
// gathered positions from L2 (measured 2-5% faster than plain loads for the float record).
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef int i32x4 __attribute__((ext_vector_type(4)));
typedef double f64x2 __attribute__((ext_vector_type(2)));

// a stencil's force on an owned vertex into the tile's order-independent accumulator (both precisions)
// A stencil's forces on the tile's own vertices into its order-independent accumulator (both
// precisions).  HOIST: one range test for the whole stencil; when its largest component is below 2^51
// counts (nearly always), each component is rounded by the accumulator's one-addition path, else by the
// general one, which also flags values out of range.  Otherwise each component is tested on its own
// (the triangle shells: the second copy of the loop costs them registers and is slower there).
template <bool HOIST, int K, typename R, typename Acc>
__device__ __forceinline__ void lds_add_stencil(Acc& acc, const int (&vid)[K], long base, int nown,
                                                const V3<R> (&f)[K], double counts_per_unit) {
    if constexpr (!HOIST) {
#pragma unroll
        for (int j = 0; j < K; ++j) {
            const unsigned slot = unsigned(vid[j] - base);
            if (slot < unsigned(nown)) {
                acc.add_counts(3 * int(slot) + 0, double(f[j].x) * counts_per_unit);
                acc.add_counts(3 * int(slot) + 1, double(f[j].y) * counts_per_unit);
                acc.add_counts(3 * int(slot) + 2, double(f[j].z) * counts_per_unit);
            }
        }
        return;
    }
    R m = R(0);
#pragma unroll
    for (int j = 0; j < K; ++j) m = fmax(m, fmax(fabs(f[j].x), fmax(fabs(f[j].y), fabs(f[j].z))));
    if (double(m) * counts_per_unit < 0x1p51) {
#pragma unroll
        for (int j = 0; j < K; ++j) {
            const unsigned slot = unsigned(vid[j] - base);
            if (slot < unsigned(nown)) {
                acc.add_counts_small(3 * int(slot) + 0, double(f[j].x) * counts_per_unit);
                acc.add_counts_small(3 * int(slot) + 1, double(f[j].y) * counts_per_unit);
                acc.add_counts_small(3 * int(slot) + 2, double(f[j].z) * counts_per_unit);
            }
        }
    } else {
#pragma unroll
        for (int j = 0; j < K; ++j) {
            const unsigned slot = unsigned(vid[j] - base);
            if (slot < unsigned(nown)) {
                acc.add_counts(3 * int(slot) + 0, double(f[j].x) * counts_per_unit);
                acc.add_counts(3 * int(slot) + 1, double(f[j].y) * counts_per_unit);
                acc.add_counts(3 * int(slot) + 2, double(f[j].z) * counts_per_unit);
            }
        }
    }
}

// Largest force work-group; the kernels are compiled for it, so any size up to it can be launched.
constexpr int kMaxForceThreads = 1024;

// One work-group per (mesh, vertex tile) work item.  K = 4 (edge) or 6 (triangle) vertices per stencil.
template <int MODEL, typename R>
__global__ __launch_bounds__(kMaxForceThreads) void force_tiles(const ForceDesc* __restrict__ descs,
                                                   const WorkItem* __restrict__ items, long nitems) {
    constexpr bool EDGE = (MODEL == SHELL_EP || MODEL == SHELL_ES);
    constexpr bool SHELL = (MODEL == SHELL_ES || MODEL == SHELL_FS || MODEL == SHELL_SS);
    constexpr int K = EDGE ? 4 : 6;
    constexpr int O = EDGE ? 1 : 0;                 // origin of the differences
    constexpr bool MIX = sizeof(R) == 4;
    constexpr bool REST = MIX && !SHELL && !EDGE;   // mixed triangle plates also gather the rest positions
    extern __shared__ unsigned char smem_raw[];
    long it = xcd_logical(blockIdx.x, gridDim.x);
    if (it >= nitems) return;
    const WorkItem wi = items[it];
    const ForceDesc& d = descs[wi.mesh];
    // global-address views of the descriptor's pointers: global loads wait on the vector-memory counter
    // only, so the LDS accumulation does not stall behind loads in flight
    const gbl<const double>* x = G(d.x);
    const gbl<const double>* X = G(d.X);
    const R kb = R(d.kb), nu = R(d.nu);
    const long blk = wi.unit;
    const long base = blk * long(d.T);
    const int nown = int(min(long(d.T), d.nv - base));
    // float32 results take the one-part accumulator
    TileAccT<MIX ? 1 : 2> acc(smem_raw, d.T);
    acc.clear(3 * nown);
    const double inv_scale = acc.kUnit / d.fscale;  // counts per force unit, a power of two: exact
    // The triangle models' forces are linear in kb: scaled by inv_scale (exactly: a power of two) it gives
    // their forces, and energies, in counts directly, the same values without a multiply per component.
    const R kbt = EDGE ? kb : R(d.kb * inv_scale);
    const double count_unit = EDGE ? inv_scale : 1.0;    // counts per unit of the stencil forces below
    const double en_unit = EDGE ? 1.0 : 1.0 / inv_scale;  // energy units per unit of their energies
    __syncthreads();
    double e_own = 0.0;
    // a tile's list starts on a 64-stencil block and the work-group's stride is a whole number of
    // blocks, so each wave reads whole blocks: every field of its 64 stencils is one contiguous run
    constexpr int R_ = EDGE ? 1 : 3;                // curvature components
    constexpr int NB = R_ * K;                      // FP64: operator entries per stencil
    constexpr int NK = R_;                          // FP64: rest-curvature slots (zero for plates)
    constexpr int NBM = R_ * (K - 1);               // mixed: operator entries without the origin column
    constexpr int NV = MIX ? NBM : NB + NK;         // float values per stencil (mixed shells: then the
                                                    // rest curvatures as float64)
    constexpr int NCH32 = stream_chunks(rec32_fields(K, R_, SHELL), 4);
    constexpr int NCHI = stream_chunks(K, 4);
    constexpr int NCHV = stream_chunks(rec64_fields(K, R_), 2);
    struct In {
        int vid[K];
        bool clamp;           // mixed plates: a stencil with a clamped edge (rest-relative curvature)
        double ab[2];         // mixed edge plates: the tip's rest-plane coordinates (alpha, beta)
        double k0[SHELL ? R_ : 1];  // mixed shells: the rest curvatures of the rounded operator
        V3<double> pg[K];     // positions
        V3<double> pr[REST ? K : 1];  // mixed plates: rest positions
        R ob[NV];
    };
    auto load = [&](long e, In& in) {
        const long first = (e / kStreamBlock) * kStreamBlock, lane = e % kStreamBlock;
        if constexpr (MIX) {
            const gbl<const f32x4>* rec = G(static_cast<const f32x4*>(d.trec)) + first * NCH32 + lane;
            float f[4 * NCH32];
#pragma unroll
            for (int c = 0; c < NCH32; ++c) {
                const f32x4 v = __builtin_nontemporal_load(rec + c * kStreamBlock);
                f[4 * c] = v.x;
                f[4 * c + 1] = v.y;
                f[4 * c + 2] = v.z;
                f[4 * c + 3] = v.w;
            }
            const uint32_t id0 = __float_as_uint(f[0]);
            in.clamp = (id0 & kRecClampBit) != 0;
            in.vid[0] = int(id0 & kRecIdMask);
#pragma unroll
            for (int j = 1; j < K; ++j) in.vid[j] = __float_as_int(f[j]);
#pragma unroll
            for (int q = 0; q < NV; ++q) in.ob[q] = f[K + q];
            auto f64 = [&](int at) {
                return __longlong_as_double((long long)((unsigned long long)__float_as_uint(f[at]) |
                                                        ((unsigned long long)__float_as_uint(f[at + 1]) << 32)));
            };
            if constexpr (EDGE && !SHELL) {
#pragma unroll
                for (int q = 0; q < 2; ++q) in.ab[q] = f64(kRecEdgeAffine + 2 * q);
            }
            if constexpr (SHELL) {
#pragma unroll
                for (int q = 0; q < R_; ++q) in.k0[q] = f64(K + NBM + 2 * q);
            }
        } else {
            const gbl<const i32x4>* ti = G(reinterpret_cast<const i32x4*>(d.tidx)) + first * NCHI + lane;
            const gbl<const f64x2>* tv = G(static_cast<const f64x2*>(d.trec)) + first * NCHV + lane;
            int fi[4 * NCHI];
            double fv[2 * NCHV];
#pragma unroll
            for (int c = 0; c < NCHI; ++c) {
                const i32x4 v = __builtin_nontemporal_load(ti + c * kStreamBlock);
                fi[4 * c] = v.x;
                fi[4 * c + 1] = v.y;
                fi[4 * c + 2] = v.z;
                fi[4 * c + 3] = v.w;
            }
#pragma unroll
            for (int c = 0; c < NCHV; ++c) {
                const f64x2 v = __builtin_nontemporal_load(tv + c * kStreamBlock);
                fv[2 * c] = v.x;
                fv[2 * c + 1] = v.y;
            }
#pragma unroll
            for (int j = 0; j < K; ++j) in.vid[j] = fi[j];
            in.clamp = false;
#pragma unroll
            for (int q = 0; q < NV; ++q) in.ob[q] = R(fv[q]);
        }
#pragma unroll
        for (int j = 0; j < K; ++j)
            in.pg[j] = {x[3L * in.vid[j]], x[3L * in.vid[j] + 1], x[3L * in.vid[j] + 2]};
        if constexpr (REST) {
#pragma unroll
            for (int j = 0; j < K; ++j)
                in.pr[j] = {X[3L * in.vid[j]], X[3L * in.vid[j] + 1], X[3L * in.vid[j] + 2]};
        }
    };
    auto compute = [&](const In& in) {
        V3<R> fs[K];
        R en;
        // float64 differences from the origin
        V3<double> dv[K];
#pragma unroll
        for (int j = 0; j < K; ++j) dv[j] = in.pg[j] - in.pg[O];
        if constexpr (EDGE) {
            R L[4];
            if constexpr (MIX) {
                L[0] = in.ob[0];
                L[2] = in.ob[1];
                L[3] = in.ob[2];
                L[1] = -(L[0] + L[2] + L[3]);
            } else {
#pragma unroll
                for (int j = 0; j < 4; ++j) L[j] = in.ob[j];
            }
            const V3<R> a = cvt<R>(dv[0]), c = cvt<R>(dv[2]), b = cvt<R>(dv[3]);
            V3<R> C;
            R delta = R(0);
            EdgeFrame<R> fr{};
            if constexpr (SHELL) {
                fr = edge_frame<R>(a, c, b);
                C = L[0] * a;
                fma3(C, L[2], c);
                fma3(C, L[3], b);
                if constexpr (MIX) {
                    // the float32 normal renormalised in float64: its length error would otherwise
                    // enter the heights along n, as kappa0 times eps_32
                    V3<double> nd = cvt<double>(fr.n);
                    nd = inv_norm<1>(nd) * nd;
                    double dl = -in.k0[0];
                    dl = fma(double(L[0]), dot(dv[0], nd), dl);
                    dl = fma(double(L[2]), dot(dv[2], nd), dl);
                    dl = fma(double(L[3]), dot(dv[3], nd), dl);
                    delta = R(dl);
                } else {
                    delta = dot(fr.n, C) - in.ob[4];
                }
            } else if constexpr (MIX) {
                if (in.clamp) {
                    // rest-relative (a boundary stencil): the rest positions are gathered here only
                    C = mk(R(0), R(0), R(0));
                    const V3<double> Xo = {X[3L * in.vid[O]], X[3L * in.vid[O] + 1], X[3L * in.vid[O] + 2]};
#pragma unroll
                    for (int j = 0; j < 4; ++j)
                        if (j != O) {
                            const V3<double> Xj = {X[3L * in.vid[j]], X[3L * in.vid[j] + 1], X[3L * in.vid[j] + 2]};
                            fma3(C, L[j], cvt<R>(dv[j] - (Xj - Xo)));
                        }
                } else {
                    // the tip's deviation from the affine map of the first hinge triangle
                    V3<double> w = dv[3];
                    fma3(w, -in.ab[0], dv[0]);
                    fma3(w, -in.ab[1], dv[2]);
                    C = L[3] * cvt<R>(w);
                }
            } else {
                C = L[0] * a;
                fma3(C, L[2], c);
                fma3(C, L[3], b);
            }
            edge_force<R, SHELL>(a, c, b, C, L, fr, delta, fs, en);
        } else {
            R Bm[3][6];
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                if constexpr (MIX) {
                    R s0 = R(0);
#pragma unroll
                    for (int j = 1; j < 6; ++j) {
                        Bm[i][j] = in.ob[5 * i + j - 1];
                        s0 += Bm[i][j];
                    }
                    Bm[i][0] = -s0;
                } else {
#pragma unroll
                    for (int j = 0; j < 6; ++j) Bm[i][j] = in.ob[6 * i + j];
                }
            }
            V3<R> dd[6], C[3];
#pragma unroll
            for (int j = 0; j < 6; ++j) dd[j] = cvt<R>(dv[j]);
            R de[3] = {R(0), R(0), R(0)};
            V3<R> n = mk(R(0), R(0), R(0));
            R ilu = R(0);
            if constexpr (SHELL) {
                const V3<R> u = cross(dd[1], dd[2]);
                ilu = inv_norm(u);
                n = ilu * u;
            }
            if constexpr (MIX && !SHELL) {
#pragma unroll
                for (int i = 0; i < 3; ++i) C[i] = mk(R(0), R(0), R(0));
                if (in.clamp) {
#pragma unroll
                    for (int j = 1; j < 6; ++j) {
                        const V3<R> du = cvt<R>(dv[j] - (in.pr[j] - in.pr[0]));
#pragma unroll
                        for (int i = 0; i < 3; ++i) fma3(C[i], Bm[i][j], du);
                    }
                } else {
                    // the flaps' deviation from the affine map of the central triangle
                    const V3<double> e1 = in.pr[1] - in.pr[0], e2 = in.pr[2] - in.pr[0];
                    const Plane2 pl(e1, e2);
#pragma unroll
                    for (int j = 3; j < 6; ++j) {
                        double a, b;
                        pl.coords(e1, e2, in.pr[j] - in.pr[0], a, b);
                        V3<double> w = dv[j];
                        fma3(w, -a, dv[1]);
                        fma3(w, -b, dv[2]);
                        const V3<R> wr = cvt<R>(w);
#pragma unroll
                        for (int i = 0; i < 3; ++i) fma3(C[i], Bm[i][j], wr);
                    }
                }
            } else {
#pragma unroll
                for (int i = 0; i < 3; ++i) {
                    C[i] = mk(R(0), R(0), R(0));
#pragma unroll
                    for (int j = 1; j < 6; ++j) fma3(C[i], Bm[i][j], dd[j]);
                }
                if constexpr (SHELL) {
                    if constexpr (MIX) {
                        // the float32 normal renormalised in float64 (its length error would otherwise
                        // enter the heights along n, as kappa0 times eps_32)
                        V3<double> nd = cvt<double>(n);
                        nd = inv_norm<1>(nd) * nd;
                        double h[6];
#pragma unroll
                        for (int j = 1; j < 6; ++j) h[j] = dot(dv[j], nd);
#pragma unroll
                        for (int i = 0; i < 3; ++i) {
                            double s0 = -in.k0[i];
#pragma unroll
                            for (int j = 1; j < 6; ++j) s0 = fma(double(Bm[i][j]), h[j], s0);
                            de[i] = R(s0);
                        }
                    } else {
#pragma unroll
                        for (int i = 0; i < 3; ++i) de[i] = dot(n, C[i]) - in.ob[NB + i];
                    }
                }
            }
            tri_force<R, SHELL>(dd, C, Bm, de, n, ilu, kbt, nu, fs, en);
        }
        // the tile that owns vertex 1 of the stencil counts its energy
        if (unsigned(in.vid[0] - base) < unsigned(nown)) e_own += double(en) * en_unit;
        lds_add_stencil<!(SHELL && !EDGE), K>(acc, in.vid, base, nown, fs, count_unit);
    };
    const long e0 = d.boff[2 * blk], e1 = d.boff[2 * blk + 1];
    for (long e = e0 + threadIdx.x; e < e1; e += blockDim.x) {
        In a;
        load(e, a);
        compute(a);
    }
    __syncthreads();
    gbl<R>* out = G(static_cast<R*>(d.f)) + 3 * base;
    const double sc = d.fscale;
    if constexpr (!MIX) {
        if (d.bias) {
            // plates with clamped edges: the constant force and energy terms that make the clamped
            // stencils rest-relative, f + F0 and E - F0 . x (+ E0 once, when the partials are summed)
            const gbl<const double>* b = G(d.bias) + 3 * base;
            for (int i = threadIdx.x; i < 3 * nown; i += blockDim.x) {
                const double bi = b[i];
                out[i] = acc.get(i) * sc + bi;
                e_own -= bi * x[3 * base + i];
            }
        } else {
            for (int i = threadIdx.x; i < 3 * nown; i += blockDim.x) out[i] = R(acc.get(i) * sc);
        }
    } else {
        for (int i = threadIdx.x; i < 3 * nown; i += blockDim.x) out[i] = R(acc.get(i) * sc);
    }
    if (d.epart) {
        __shared__ double sh[kMaxForceThreads / 64];
        double v[1] = {e_own};
        block_sum<1>(v, sh);
        if (threadIdx.x == 0) d.epart[blk] = v[0];
    }
}

// Work-group size of a force kernel.  A launch has one work-group per tile (512 on a 1M-vertex mesh, two
// per CU), so the waves in flight, which hide the latency of the stencil stream and of the position
// gathers, come from the work-group size.  It is the largest multiple of 256 threads (one wave per
// SIMD; uneven multiples leave a SIMD short of room for the second work-group) whose two work-groups
// per CU fit the waves per SIMD that the kernel's VGPR count allows (512 VGPRs per SIMD lane, allocated
// in granules of 8, at most 8 waves).  Edge kernels (46-86 VGPRs) get 512-1024 threads, triangle kernels
// 512-768.  (Measured against a fixed 256 threads with two stencils per thread and pass: edge models
// 9-15% faster, float shells 5%, the rest equal or up to 4% faster.)
template <typename Kernel>
int force_threads(Kernel kernel) {
    hipFuncAttributes a{};
    SHELL_HIP(hipFuncGetAttributes(&a, reinterpret_cast<const void*>(kernel)));
    const int vgprs = std::max(8, (a.numRegs + 7) / 8 * 8);
    const int waves = std::min(8, 512 / vgprs);  // per SIMD
    return std::min(kMaxForceThreads, 256 * std::max(1, waves / 2));
}

template <int MODEL>
void launch_model(int precision, const ForceDesc* descs, const WorkItem* items, long nitems, int lds_T,
                  hipStream_t s, hipEvent_t start, hipEvent_t stop) {
    static const int threads_d = force_threads(force_tiles<MODEL, double>);
    static const int threads_f = force_threads(force_tiles<MODEL, float>);
    const dim3 grid(unsigned(xcd_grid(nitems)));
    // start/stop (may be null) receive the dispatch's own begin and end times
    if (precision == SHELL_PREC_FP64)
        hipExtLaunchKernelGGL(force_tiles<MODEL, double>, grid, dim3(threads_d), uint32_t(TileAccT<2>::bytes(lds_T)),
                              s, start, stop, 0, descs, items, nitems);
    else
        hipExtLaunchKernelGGL(force_tiles<MODEL, float>, grid, dim3(threads_f), uint32_t(TileAccT<1>::bytes(lds_T)),
                              s, start, stop, 0, descs, items, nitems);
    SHELL_HIP(hipGetLastError());
}

__global__ void energy_finalize(const double* __restrict__ part, long n, double add, const double* __restrict__ extra,
                                long m, double* __restrict__ out) {
    __shared__ double sh[16];
    double acc = 0.0;
    for (long i = threadIdx.x; i < n; i += blockDim.x) acc += part[i];
    for (long i = threadIdx.x; i < m; i += blockDim.x) acc += extra[i];
    double v[1] = {acc};
    block_sum<1>(v, sh);
    if (threadIdx.x == 0) *out = v[0] + add;
}

__global__ void write_force_desc(ForceDesc d, ForceDesc* __restrict__ dst, WorkItem* __restrict__ items, long n) {
    const long t = blockIdx.x * long(blockDim.x) + threadIdx.x;
    if (t == 0) *dst = d;
    if (t < n) items[t] = WorkItem{0, int32_t(t)};
}

__global__ void gather_rows(const double* __restrict__ src, const int32_t* __restrict__ perm,
                            double* __restrict__ dst, long nv) {
    long i = blockIdx.x * long(blockDim.x) + threadIdx.x;
    if (i >= nv) return;
    long u = perm[i];
    dst[3 * i] = src[3 * u];
    dst[3 * i + 1] = src[3 * u + 1];
    dst[3 * i + 2] = src[3 * u + 2];
}

template <typename T>
__global__ void scatter_rows(const T* __restrict__ src, const int32_t* __restrict__ perm, T* __restrict__ dst,
                             long nv) {
    long i = blockIdx.x * long(blockDim.x) + threadIdx.x;
    if (i >= nv) return;
    long u = perm[i];
    dst[3 * u] = src[3 * i];
    dst[3 * u + 1] = src[3 * i + 1];
    dst[3 * u + 2] = src[3 * i + 2];
}

}  // namespace

void launch_force_items(int model, int precision, const ForceDesc* descs, const WorkItem* items, long nitems,
                        int lds_T, hipStream_t s, hipEvent_t start, hipEvent_t stop) {
    if (nitems <= 0) return;
    switch (model) {
        case SHELL_EP: launch_model<SHELL_EP>(precision, descs, items, nitems, lds_T, s, start, stop); break;
        case SHELL_ES: launch_model<SHELL_ES>(precision, descs, items, nitems, lds_T, s, start, stop); break;
        case SHELL_FP: launch_model<SHELL_FP>(precision, descs, items, nitems, lds_T, s, start, stop); break;
        case SHELL_FS: launch_model<SHELL_FS>(precision, descs, items, nitems, lds_T, s, start, stop); break;
        case SHELL_SP: launch_model<SHELL_SP>(precision, descs, items, nitems, lds_T, s, start, stop); break;
        case SHELL_SS: launch_model<SHELL_SS>(precision, descs, items, nitems, lds_T, s, start, stop); break;
        default: throw Error(SHELL_E_INVALID_ARG, "unknown model");
    }
}

void launch_write_force_desc(const ForceDesc& d, ForceDesc* dst, WorkItem* items, int64_t ntiles, hipStream_t s) {
    write_force_desc<<<unsigned((std::max<int64_t>(ntiles, 1) + 255) / 256), 256, 0, s>>>(d, dst, items, ntiles);
    SHELL_HIP(hipGetLastError());
}

void launch_energy_finalize(const double* epart, int64_t n, double add, double* energy, hipStream_t s,
                            const double* extra, int64_t m) {
    energy_finalize<<<1, 256, 0, s>>>(epart, n, add, extra, m, energy);
    SHELL_HIP(hipGetLastError());
}

void launch_gather_rows(const double* src, const int32_t* perm, double* dst, int64_t nv, hipStream_t s) {
    if (!nv) return;
    gather_rows<<<(nv + 255) / 256, 256, 0, s>>>(src, perm, dst, nv);
    SHELL_HIP(hipGetLastError());
}

void launch_scatter_rows(const void* src, const int32_t* perm, void* dst, int64_t nv, bool f32, hipStream_t s) {
    if (!nv) return;
    if (f32)
        scatter_rows<float><<<(nv + 255) / 256, 256, 0, s>>>(static_cast<const float*>(src), perm,
                                                             static_cast<float*>(dst), nv);
    else
        scatter_rows<double><<<(nv + 255) / 256, 256, 0, s>>>(static_cast<const double*>(src), perm,
                                                              static_cast<double*>(dst), nv);
    SHELL_HIP(hipGetLastError());
}

}  // namespace shell
