// Membrane (Sec. 3, eq 1) on constant strain triangles with the Saint Venant-Kirchhoff model, float64.
//
// Rest data per triangle (membrane_rest): the rest frame e1 along X1 - X0, e2 = n x e1; Dm the 2x2 matrix
// of the rest edge vectors in that frame; G = Dm^-1 and the area A.  Force (membrane_tiles): with Ds the
// current edge vectors x1 - x0, x2 - x0, F = Ds G (3x2), Green strain E = (F^T F - I)/2 in Voigt form
// [E11, E22, 2 E12], stress sigma = D_m eps with D_m = h E_el (plane stress), energy A/2 eps . sigma;
// dPsi/dDs = A F S G^T (S the stress as a 2x2 tensor), so f1 and f2 are minus its columns and f0 their
// sum.  The triangles are grouped by the same vertex tiles as the bending stencils (halo triangles
// repeat): each work-group accumulates the forces of its own vertices in LDS and adds them to the force
// the bending kernel stored, one read and one write per vertex and no global atomics (the LDS sums are
// exact fixed-point parts, so they do not depend on the order of the additions).  Both precisions
// compute in float64 from float64 positions (the Green strain F^T F - I cancels to the strain's size);
// mixed precision stores the sum as float32.
#include <algorithm>
#include <cmath>
#include <coroutine>
#include <exception>
#include <thread>
#include <utility>

#include "devmath.hpp"
#include "internal.hpp"

namespace shell {

namespace {

__global__ void membrane_rest(const double* __restrict__ X, const int32_t* __restrict__ tris, long nt,
                              double* __restrict__ rest, int32_t* __restrict__ bad) {
    long t = blockIdx.x * long(blockDim.x) + threadIdx.x;
    if (t >= nt) return;
    V3<double> x0 = load3(X, tris[3 * t]), x1 = load3(X, tris[3 * t + 1]), x2 = load3(X, tris[3 * t + 2]);
    V3<double> a = x1 - x0, b = x2 - x0;
    V3<double> n = cross(a, b);
    double twoA = norm(n);
    double la = norm(a);
    if (!(twoA > 0.0) || !(la > 0.0)) {
        *bad = 1;
        for (int k = 0; k < 5; ++k) rest[5 * t + k] = 0.0;
        return;
    }
    V3<double> e1 = (1.0 / la) * a;
    V3<double> e2 = cross((1.0 / twoA) * n, e1);
    double d00 = dot(a, e1), d01 = dot(b, e1), d10 = dot(a, e2), d11 = dot(b, e2);
    double det = d00 * d11 - d01 * d10;
    rest[5 * t + 0] = d11 / det;
    rest[5 * t + 1] = -d01 / det;
    rest[5 * t + 2] = -d10 / det;
    rest[5 * t + 3] = d00 / det;
    rest[5 * t + 4] = 0.5 * twoA;
}

// tiled record of the membrane: ids [n][4] (int32, last unused) and rest data [n][6] (G, A, 0)
__global__ void membrane_tile_copy(const int32_t* __restrict__ src, long n, const int32_t* __restrict__ tris,
                                   const double* __restrict__ rest, int32_t* __restrict__ tid,
                                   double* __restrict__ trest) {
    long e = blockIdx.x * long(blockDim.x) + threadIdx.x;
    if (e >= n) return;
    const long t = src[e];  // -1: alignment padding (never read)
    for (int j = 0; j < 3; ++j) tid[4 * e + j] = t < 0 ? 0 : tris[3 * t + j];
    tid[4 * e + 3] = 0;
    for (int k = 0; k < 5; ++k) trest[6 * e + k] = t < 0 ? 0.0 : rest[5 * t + k];
    trest[6 * e + 5] = 0.0;
}

constexpr int kMembThreads = 512;

template <typename R>
__global__ __launch_bounds__(kMembThreads) void membrane_tiles(const double* __restrict__ pos,
                                                               const int32_t* __restrict__ tid,
                                                               const double* __restrict__ trest,
                                                               const int64_t* __restrict__ boff, long nv, int T,
                                                               double c, double nu, double scale,
                                                               R* __restrict__ f, double* __restrict__ epart) {
    extern __shared__ unsigned char smem_raw[];
    const long blk = blockIdx.x;
    const long base = blk * long(T);
    const int nown = int(min(long(T), nv - base));
    TileAccT<sizeof(R) == 4 ? 1 : 2> acc(smem_raw, T);  // float32 results take the one-part accumulator
    acc.clear(3 * nown);
    const double inv_scale = acc.kUnit / scale;  // counts per force unit, a power of two: exact
    __syncthreads();
    double en[1] = {0.0};
    const long e0 = boff[2 * blk], e1 = boff[2 * blk + 1];
    for (long e = e0 + threadIdx.x; e < e1; e += blockDim.x) {
        const long v[3] = {tid[4 * e], tid[4 * e + 1], tid[4 * e + 2]};
        double d1[3], d2[3];
        for (int i = 0; i < 3; ++i) {
            d1[i] = pos[3 * v[1] + i] - pos[3 * v[0] + i];
            d2[i] = pos[3 * v[2] + i] - pos[3 * v[0] + i];
        }
        const double G[2][2] = {{trest[6 * e], trest[6 * e + 1]}, {trest[6 * e + 2], trest[6 * e + 3]}};
        const double A = trest[6 * e + 4];
        double F[3][2];
        for (int i = 0; i < 3; ++i)
            for (int b = 0; b < 2; ++b) F[i][b] = d1[i] * G[0][b] + d2[i] * G[1][b];
        const double C00 = F[0][0] * F[0][0] + F[1][0] * F[1][0] + F[2][0] * F[2][0];
        const double C11 = F[0][1] * F[0][1] + F[1][1] * F[1][1] + F[2][1] * F[2][1];
        const double C01 = F[0][0] * F[0][1] + F[1][0] * F[1][1] + F[2][0] * F[2][1];
        const double s0e = 0.5 * (C00 - 1.0), s1e = 0.5 * (C11 - 1.0), s2e = C01;
        const double s0 = c * (s0e + nu * s1e), s1 = c * (nu * s0e + s1e), s2 = c * 0.5 * (1.0 - nu) * s2e;
        const unsigned o0 = unsigned(v[0] - base), o1 = unsigned(v[1] - base), o2 = unsigned(v[2] - base);
        if (o0 < unsigned(nown)) en[0] += 0.5 * A * (s0e * s0 + s1e * s1 + s2e * s2);
        for (int i = 0; i < 3; ++i) {
            const double P0 = A * (F[i][0] * s0 + F[i][1] * s2), P1 = A * (F[i][0] * s2 + F[i][1] * s1);
            const double h0 = P0 * G[0][0] + P1 * G[0][1], h1 = P0 * G[1][0] + P1 * G[1][1];
            if (o1 < unsigned(nown)) acc.add_counts(3 * o1 + i, -h0 * inv_scale);
            if (o2 < unsigned(nown)) acc.add_counts(3 * o2 + i, -h1 * inv_scale);
            if (o0 < unsigned(nown)) acc.add_counts(3 * o0 + i, (h0 + h1) * inv_scale);
        }
    }
    __syncthreads();
    R* out = f + 3 * base;
    const double sc = scale;
    for (int i = threadIdx.x; i < 3 * nown; i += blockDim.x) out[i] = R(double(out[i]) + acc.get(i) * sc);
    __shared__ double sh[kMembThreads / 64];
    block_sum<1>(en, sh);
    if (threadIdx.x == 0) epart[blk] = en[0];
}

// ---------------------------------------------------------------- implicit step with the membrane
//
// Sec. 5's step (eq 62) with the membrane of Sec. 3 added to the bending energy.  Each Newton iteration:
// g = M (x - x_hat) - dt^2 f (held coordinates' rows zero); the matrix M + dt^2 (K_s (x) I3 + K_m(x)) with
// K_m the membrane tangent per triangle: the Gauss-Newton part A B(F)^T D_m B(F) (B(F) the linearised
// Green strain, rows g_j0 F0^T, g_j1 F1^T, g_j1 F0^T + g_j0 F1^T) plus the stress part A (g_a^T S+ g_b) I3
// with S+ the positive semi-definite part of the 2x2 stress (the exact Hessian under tension, Gauss-Newton
// under compression, PSD always), assembled into 3x3 blocks on the triangle adjacency; one
// Jacobi-PCG over all coordinates (1/(m + dt^2 (K_s,ii + tr(K_m,ii)/3)) per vertex); then x += 2^-h y
// with h the fewest halvings (at most 6) meeting Armijo's condition E(x + a y) <= E(x) + 1e-4 a g.y on the
// incremental potential E = 1/2 (x - x_hat)^T M (x - x_hat) + dt^2 (Psi_b + Psi_m).  Sums are per
// 256-thread block, then in a fixed order by one block, so they do not depend on scheduling.

constexpr int kMsBlk = 256;
// device scalars
enum : int { S_RZ, S_RZN, S_PQ, S_RR, S_RR0, S_TOL2, S_ALPHA, S_BETA, S_GSQ, S_SLOPE, S_E, S_IT, S_TARGET,
             S_ACTIVE, S_REPLAY, S_BUDGET, S_YMAX, S_FRESH, S_COUNT };
// The coupled PCG's state lives in two sets of these scalars (set k at scal + k S_COUNT) that alternate
// with the direction buffers: a product reads its iteration's state from one set and stores the next into
// the other, which no work-group of the same launch reads.  The solve's constants (S_TOL2, S_TARGET,
// S_REPLAY, S_RR0) and the step's other scalars stay in set 0; the one-work-group solver uses set 0 only.

template <int NQ>
__device__ __forceinline__ void ms_partials(double (&v)[NQ], double* part, long ngroups) {
    __shared__ double sh[NQ * (kMsBlk / 64)];
    block_sum<NQ>(v, sh);
    if (threadIdx.x == 0)
        for (int q = 0; q < NQ; ++q) part[q * ngroups + blockIdx.x] = v[q];
}

// totals of NQ partial arrays, valid in thread 0 of a single block
template <int NQ>
__device__ __forceinline__ void ms_totals(const double* part, long ngroups, double (&out)[NQ]) {
    for (int q = 0; q < NQ; ++q) out[q] = 0.0;
    for (long b = threadIdx.x; b < ngroups; b += blockDim.x)
        for (int q = 0; q < NQ; ++q) out[q] += part[q * ngroups + b];
    __shared__ double sh[NQ * (kMsBlk / 64)];
    block_sum<NQ>(out, sh);
}

__global__ void ms_predictor(double* __restrict__ x, const double* __restrict__ v, double* __restrict__ xt,
                             double* __restrict__ xhat, const uint8_t* __restrict__ pinned, long nv, double dt,
                             double gx, double gy, double gz) {
    long i = blockIdx.x * long(blockDim.x) + threadIdx.x;
    if (i >= nv) return;
    const double gr[3] = {gx, gy, gz};
    for (int c = 0; c < 3; ++c) {
        const double xi = x[3 * i + c];
        const double xh = (pinned[i] >> c & 1u) ? xi : xi + dt * v[3 * i + c] + dt * dt * gr[c];
        xt[3 * i + c] = xi;
        xhat[3 * i + c] = xh;
        x[3 * i + c] = xh;
    }
}

__global__ void ms_axpy(const double* __restrict__ x, const double* __restrict__ y, double a, double* __restrict__ out,
                        long n) {
    long i = blockIdx.x * long(blockDim.x) + threadIdx.x;
    if (i < n) out[i] = x[i] + a * y[i];
}

__global__ void ms_velocity(const double* __restrict__ x, const double* __restrict__ xt, double* __restrict__ v,
                            long n, double dt) {
    long i = blockIdx.x * long(blockDim.x) + threadIdx.x;
    if (i < n) v[i] = (x[i] - xt[i]) / dt;
}

// partials of the inertia term 1/2 m |x - x_hat|^2
__global__ __launch_bounds__(kMsBlk) void ms_inertia(const double* __restrict__ x, const double* __restrict__ xhat,
                                                     const double* __restrict__ mass, long nv,
                                                     double* __restrict__ part, long ngroups) {
    long i = blockIdx.x * long(blockDim.x) + threadIdx.x;
    double v[1] = {0.0};
    if (i < nv)
        for (int c = 0; c < 3; ++c) {
            const double u = x[3 * i + c] - xhat[3 * i + c];
            v[0] += 0.5 * mass[i] * u * u;
        }
    ms_partials<1>(v, part, ngroups);
}

// E = inertia + dt^2 (bending + membrane) into the scalars
__global__ __launch_bounds__(kMsBlk) void ms_energy(const double* __restrict__ eb, long nb,
                                                    const double* __restrict__ em, long nm, double add,
                                                    const double* __restrict__ part, long ngroups, double dt2,
                                                    double* __restrict__ scal) {
    double t[1];
    ms_totals<1>(part, ngroups, t);
    double b = 0.0;
    for (long k = threadIdx.x; k < nb; k += blockDim.x) b += eb[k];
    for (long k = threadIdx.x; k < nm; k += blockDim.x) b += em[k];
    double v[1] = {b};
    __shared__ double sh[kMsBlk / 64];
    block_sum<1>(v, sh);
    if (threadIdx.x == 0) scal[S_E] = t[0] + dt2 * (v[0] + add);
}

// g = M (x - x_hat) - dt^2 f, fixed rows zero; partial |g|^2
__global__ __launch_bounds__(kMsBlk) void ms_grad(const double* __restrict__ x, const double* __restrict__ xhat,
                                                  const double* __restrict__ mass, const double* __restrict__ f,
                                                  const uint8_t* __restrict__ pinned, long nv, double dt2,
                                                  double* __restrict__ g, double* __restrict__ part, long ngroups) {
    long i = blockIdx.x * long(blockDim.x) + threadIdx.x;
    double v[1] = {0.0};
    if (i < nv)
        for (int c = 0; c < 3; ++c) {
            const double gi = (pinned[i] >> c & 1u) ? 0.0 : mass[i] * (x[3 * i + c] - xhat[3 * i + c]) - dt2 * f[3 * i + c];
            g[3 * i + c] = gi;
            v[0] += gi * gi;
        }
    ms_partials<1>(v, part, ngroups);
}

__global__ __launch_bounds__(kMsBlk) void ms_dot(const double* __restrict__ a, const double* __restrict__ b, long n,
                                                 double* __restrict__ part, long ngroups) {
    double v[1] = {0.0};
    for (long i = blockIdx.x * long(blockDim.x) + threadIdx.x; i < n; i += long(gridDim.x) * blockDim.x)
        v[0] += a[i] * b[i];
    ms_partials<1>(v, part, ngroups);
}

__global__ __launch_bounds__(kMsBlk) void ms_fin1(const double* __restrict__ part, long ngroups,
                                                  double* __restrict__ scal, int slot) {
    double t[1];
    ms_totals<1>(part, ngroups, t);
    if (threadIdx.x == 0) scal[slot] = t[0];
}

// The membrane tangent into the 3x3 blocks, one thread per stored block (i, j): the thread sums, in
// ascending order, the contributions of the triangles holding both vertices (the one or two triangles
// of edge ij; every triangle of i when j = i) in registers and writes the block once, so every block
// takes the same sums in every run (no atomics, no read-modify-write).  Per triangle, with a and b the
// corners of i and j: the Gauss-Newton part A B_a^T D_m B_b (B_c the linearised Green strain of corner
// c: rows g_c0 F0^T, g_c1 F1^T, g_c1 F0^T + g_c0 F1^T) and the stress part A (g_a^T S+ g_b) I3.
// Component (a, b) of CSR block e is mval[mbase[e] + (3 a + b) mstride].  With s2e (the staged layout)
// thread t takes SELL slot t, s2e[t] its CSR block (-1 on padding, which stays zero), so that the
// lanes of a wave write consecutive slots; otherwise thread t takes CSR block t.  Mixed precision
// (mvalf not null) also writes the float32 copy the product reads.
__global__ void ms_tangent(const double* __restrict__ rest, const int32_t* __restrict__ tris,
                           const int32_t* __restrict__ brow, const int32_t* __restrict__ mcol,
                           const int64_t* __restrict__ btptr, const int32_t* __restrict__ bttri,
                           const int64_t* __restrict__ s2e, long nthreads, const double* __restrict__ x, double c,
                           double nu, const int64_t* __restrict__ mbase, long mstride, double* __restrict__ mval,
                           float* __restrict__ mvalf) {
    const long tid = blockIdx.x * long(blockDim.x) + threadIdx.x;
    if (tid >= nthreads) return;
    const long e = s2e ? s2e[tid] : tid;
    if (e < 0) return;
    const int32_t r = brow[e], jc = mcol[e];
    double acc[9];
    for (int k = 0; k < 9; ++k) acc[k] = 0.0;
    for (long q = btptr[e]; q < btptr[e + 1]; ++q) {
        const long t = bttri[q];
        const int32_t v[3] = {tris[3 * t], tris[3 * t + 1], tris[3 * t + 2]};
        const int a = v[0] == r ? 0 : (v[1] == r ? 1 : 2);
        const int b = v[0] == jc ? 0 : (v[1] == jc ? 1 : 2);
        const double G[2][2] = {{rest[5 * t], rest[5 * t + 1]}, {rest[5 * t + 2], rest[5 * t + 3]}};
        const double A = rest[5 * t + 4];
        double F[3][2];
        for (int i = 0; i < 3; ++i) {
            const double d1 = x[3L * v[1] + i] - x[3L * v[0] + i], d2 = x[3L * v[2] + i] - x[3L * v[0] + i];
            for (int k = 0; k < 2; ++k) F[i][k] = d1 * G[0][k] + d2 * G[1][k];
        }
        const double g[3][2] = {{-G[0][0] - G[1][0], -G[0][1] - G[1][1]}, {G[0][0], G[0][1]}, {G[1][0], G[1][1]}};
        // B rows of corner a (coordinate ca) and D_m B of corner b (coordinate cb),
        // D_m = c [[1, nu, 0], [nu, 1, 0], [0, 0, (1 - nu)/2]]
        double Ba[3][3], DBb[3][3];
        for (int k = 0; k < 3; ++k) {
            Ba[k][0] = g[a][0] * F[k][0];
            Ba[k][1] = g[a][1] * F[k][1];
            Ba[k][2] = g[a][1] * F[k][0] + g[a][0] * F[k][1];
            const double b0 = g[b][0] * F[k][0], b1 = g[b][1] * F[k][1], b2 = g[b][1] * F[k][0] + g[b][0] * F[k][1];
            DBb[k][0] = c * (b0 + nu * b1);
            DBb[k][1] = c * (nu * b0 + b1);
            DBb[k][2] = c * 0.5 * (1.0 - nu) * b2;
        }
        // the stress and its positive semi-definite part from the principal values l1 >= l2
        const double C00 = F[0][0] * F[0][0] + F[1][0] * F[1][0] + F[2][0] * F[2][0];
        const double C11 = F[0][1] * F[0][1] + F[1][1] * F[1][1] + F[2][1] * F[2][1];
        const double C01 = F[0][0] * F[0][1] + F[1][0] * F[1][1] + F[2][0] * F[2][1];
        const double e0 = 0.5 * (C00 - 1.0), e1 = 0.5 * (C11 - 1.0);
        const double s11 = c * (e0 + nu * e1), s22 = c * (nu * e0 + e1), s12 = c * 0.5 * (1.0 - nu) * C01;
        const double mean = 0.5 * (s11 + s22), half = 0.5 * (s11 - s22);
        const double rad = sqrt(half * half + s12 * s12);
        const double l1 = mean + rad, l2 = mean - rad;
        double P00 = s11, P01 = s12, P11 = s22;
        if (l1 <= 0.0) {
            P00 = P01 = P11 = 0.0;
        } else if (l2 < 0.0) {
            const double w = l1 / (l1 - l2);  // l1 v v^T with v v^T = (S - l2 I) / (l1 - l2)
            P00 = w * (s11 - l2);
            P01 = w * s12;
            P11 = w * (s22 - l2);
        }
        for (int ca = 0; ca < 3; ++ca)
            for (int cb = 0; cb < 3; ++cb)
                acc[3 * ca + cb] += A * (Ba[ca][0] * DBb[cb][0] + Ba[ca][1] * DBb[cb][1] + Ba[ca][2] * DBb[cb][2]);
        const double gsg = g[a][0] * (P00 * g[b][0] + P01 * g[b][1]) + g[a][1] * (P01 * g[b][0] + P11 * g[b][1]);
        for (int cc = 0; cc < 3; ++cc) acc[4 * cc] += A * gsg;
    }
    const long base = s2e ? tid : mbase[e];
    for (int k = 0; k < 9; ++k) mval[base + k * mstride] = acc[k];
    if (mvalf)
        for (int k = 0; k < 9; ++k) mvalf[base + k * mstride] = float(acc[k]);
}

__global__ void ms_dinv(const double* __restrict__ kdiag, const double* __restrict__ mval,
                        const int64_t* __restrict__ mdiag, long mstride, const double* __restrict__ mass,
                        const uint8_t* __restrict__ pinned, long nv, double dt2, double* __restrict__ dinv) {
    long i = blockIdx.x * long(blockDim.x) + threadIdx.x;
    if (i >= nv) return;
    const double* b = mval + mdiag[i];
    const double d = mass[i] + dt2 * (kdiag[i] + (b[0] + b[4 * mstride] + b[8 * mstride]) / 3.0);
    dinv[i] = ((pinned[i] & 7u) == 7u || d == 0.0) ? 0.0 : 1.0 / d;
}

// r = -g, y = 0, z = D^-1 r, p = z; partials r.z, r.r
__global__ __launch_bounds__(kMsBlk) void ms_pcg_init(const double* __restrict__ g, const double* __restrict__ dinv,
                                                      double* __restrict__ r, double* __restrict__ z,
                                                      double* __restrict__ p, double* __restrict__ y, long nv,
                                                      double* __restrict__ part, long ngroups) {
    long i = blockIdx.x * long(blockDim.x) + threadIdx.x;
    double v[2] = {0.0, 0.0};
    if (i < nv)
        for (int c = 0; c < 3; ++c) {
            const double ri = -g[3 * i + c], zi = dinv[i] * ri;
            r[3 * i + c] = ri;
            z[3 * i + c] = zi;
            p[3 * i + c] = zi;
            y[3 * i + c] = 0.0;
            v[0] += ri * zi;
            v[1] += ri * ri;
        }
    ms_partials<2>(v, part, ngroups);
}

__global__ __launch_bounds__(kMsBlk) void ms_fin_init(const double* __restrict__ part, long ngroups,
                                                      double* __restrict__ scal, double rtol2, int target,
                                                      int replay) {
    double t[2];
    ms_totals<2>(part, ngroups, t);
    if (threadIdx.x == 0) {
        scal[S_RZ] = t[0];
        scal[S_RR0] = t[1];
        scal[S_RR] = t[1];
        scal[S_TOL2] = rtol2 * t[1];
        scal[S_IT] = 0.0;
        scal[S_TARGET] = double(target);
        scal[S_REPLAY] = double(replay);
        scal[S_BUDGET] = 0.0;
        scal[S_BETA] = 0.0;
        scal[S_ACTIVE] = (0 < target && (replay || t[1] > rtol2 * t[1])) ? 1.0 : 0.0;
        scal[S_FRESH] = 1.0;
    }
}

// The coupled PCG iteration in two kernels, none with cross-block synchronisation inside it: the product
// first finishes the previous update (r.z, r.r, beta, the count and the stop test from the update's
// partials, summed by every work-group alike in one fixed order) and writes per-work-group partials of
// p.q; the update sums those (or, with many, one work-group does, into alpha) and writes its own partials.
// A chunk of iterations ends with a one-work-group kernel that finishes the last update, so that the host
// reads the exact state; on large meshes (many update partials) that kernel runs after every iteration
// and the product finds the state settled.  The product and the update stride over the rows with at most
// kMsPartMax work-groups.

// Totals of the update's two partial arrays (ung entries each) in one fixed order whatever the work-group
// size: lane l of the first wave adds entries l, l + 64, ... in turn, then the wave sum; valid in thread 0.
// No barrier.  U entries per lane are loaded before they are added, so that their loads are in flight
// together (the order of the additions is that of the plain loop).
template <int U>
__device__ __forceinline__ void ms_update_totals(const double* __restrict__ upart, long ung, double (&t)[2]) {
    t[0] = t[1] = 0.0;
    if (threadIdx.x < 64) {
        for (long b0 = threadIdx.x; b0 < ung; b0 += 64L * U) {
            double a[U], c[U];
#pragma unroll
            for (int k = 0; k < U; ++k) {
                const long b = b0 + 64L * k;
                a[k] = b < ung ? upart[b] : 0.0;
                c[k] = b < ung ? upart[ung + b] : 0.0;
            }
#pragma unroll
            for (int k = 0; k < U; ++k) {
                t[0] += a[k];
                t[1] += c[k];
            }
        }
        t[0] = wave_sum(t[0]);
        t[1] = wave_sum(t[1]);
    }
}

// One thread: the state that follows `sin` once the update with partial totals t has run (beta, r.z, r.r,
// the count, the budget and the activity), into `out` (which may be sin); the constants from `cst`.
__device__ __forceinline__ void ms_finish_to(const double* cst, const double* sin, const double (&t)[2], double* out) {
    const double rz = sin[S_RZ], it = sin[S_IT] + 1.0, target = cst[S_TARGET];
    double budget = sin[S_BUDGET];
    const bool replay = cst[S_REPLAY] != 0.0;
    const bool more = replay || t[1] > cst[S_TOL2];
    if (!replay && it >= target && more) budget = 1.0;
    if (!isfinite(t[1])) budget = 2.0;
    out[S_BETA] = rz != 0.0 ? t[0] / rz : 0.0;
    out[S_RZ] = t[0];
    out[S_RR] = t[1];
    out[S_IT] = it;
    out[S_BUDGET] = budget;
    out[S_ACTIVE] = (it < target && more && isfinite(t[1])) ? 1.0 : 0.0;
}

// The state a product's iteration starts from, alike in every work-group: set `sin` as the previous product
// left it, finished here from the previous update's partials unless it is settled (S_FRESH: the solve's
// first iteration, or the first of a chunk after ms_iter_settle) or stopped.  Work-group 0 stores it,
// unsettled, into `sout` for the update and the next product.  Returns false when the solve has stopped;
// beta otherwise.
__device__ __forceinline__ bool ms_iteration_state(const double* cst, const double* __restrict__ sin,
                                                   double* __restrict__ sout, const double* __restrict__ upart,
                                                   long ung, double& beta) {
    __shared__ double res[2];
    const bool settled = sin[S_FRESH] != 0.0, running = sin[S_ACTIVE] != 0.0;  // the same in every thread
    double t[2] = {0.0, 0.0};
    if (!settled && running) ms_update_totals<4>(upart, ung, t);  // fused only up to 1024 partials
    if (threadIdx.x == 0) {
        double o[S_COUNT];
        o[S_RZ] = sin[S_RZ];
        o[S_RR] = sin[S_RR];
        o[S_IT] = sin[S_IT];
        o[S_BUDGET] = sin[S_BUDGET];
        o[S_ACTIVE] = sin[S_ACTIVE];
        o[S_BETA] = sin[S_BETA];
        if (!settled && running) ms_finish_to(cst, sin, t, o);
        if (blockIdx.x == 0) {
            sout[S_RZ] = o[S_RZ];
            sout[S_RR] = o[S_RR];
            sout[S_IT] = o[S_IT];
            sout[S_BUDGET] = o[S_BUDGET];
            sout[S_ACTIVE] = o[S_ACTIVE];
            sout[S_BETA] = o[S_BETA];
            sout[S_FRESH] = 0.0;
        }
        res[0] = o[S_BETA];
        res[1] = o[S_ACTIVE];
    }
    __syncthreads();
    beta = res[0];
    return res[1] != 0.0;
}

// p_new = z + beta p_old (row i, stored) and q = M p_new + dt^2 (K_s (x) I3 + K_m) p_new, the neighbours'
// p_new formed on the fly from their z and p_old; fixed rows zero; partial p.q.  LANES lanes share a row:
// they take its K_s entries and its 3x3 blocks in turn (consecutive lanes read consecutive entries) and
// combine their sums by shuffles; the row's first lane stores.  Measured at 1M vertices: 8 lanes for
// float64 entries (315 us, against 384 with 16 and 328 with 4), 4 for float32 entries (252 us, against
// 445 with 16, 291 with 8 and 340 with 2): fewer lanes give each more entries in flight and fewer
// shuffles, until too few rows share a wave's loads.
constexpr int kMsLanesF64 = 8;
constexpr int kMsLanesF32 = 4;
// The staged product (below) from this many rows up; on smaller meshes its latency floor exceeds the CSR
// product's.  Measured with 512-row groups on SS cylinders, staged against CSR product, FP64: 10.1 / 5.3 us
// at 4K rows, 14.4 / 10.2 at 33K, 15.0 / 14.1 at 48K, 15.5 / 18.1 at 65K, 20.2 / 32.9 at 131K, 144 / 317 at
// 1M.  With the smaller groups of mid-size meshes (ms_group_rows), whole steps, staged against CSR, FP64 and
// mixed: 12.0 / 10.3 and 11.3 / 10.4 ms at 16K rows, 9.9 / 10.9 and 10.0 / 9.4 at 33K, 12.5 / 14.4 and
// 12.1 / 12.5 at 48K.
#ifndef SHELL_MS_STAGED_MIN_ROWS
#define SHELL_MS_STAGED_MIN_ROWS 32768
#endif
constexpr long kMsStagedMinRows = SHELL_MS_STAGED_MIN_ROWS;
// The product and the update stride over the rows with at most kMsPartMax work-groups, so that one
// work-group sums their partials in a fixed order in a few microseconds at any mesh size.
constexpr long kMsPartMax = 2048;
inline unsigned ms_product_grid(long nv, int lanes) {
    const long rows = kMsBlk / lanes;
    return unsigned(std::min(kMsPartMax, std::max(1L, (nv + rows - 1) / rows)));
}
inline unsigned ms_update_grid(long nv) {
    return unsigned(std::min(kMsPartMax, std::max(1L, (nv + kMsBlk - 1) / kMsBlk)));
}

// VT: the type of the stored K_s entries and blocks.  Float32 entries (mixed precision) are applied in
// difference form, q_i = m_i p_i + dt^2 sum_j (K_s,ij I + K_m,ij)(p_j - p_i): K_s and the tangent both
// annihilate translations (their rows of 3x3 blocks sum to zero), and this form keeps that exactly
// whatever the rounding of the entries, as the bending product's mixed form does.
template <typename VT, int LANES>
__global__ __launch_bounds__(kMsBlk) void ms_iter_product(const double* cst, const double* __restrict__ sin,
                                                          double* __restrict__ sout, const double* __restrict__ upart,
                                                          long ung, const int64_t* __restrict__ srow,
                                                          const int32_t* __restrict__ scol, const VT* __restrict__ sval,
                                                          const int64_t* __restrict__ mrow, const int32_t* __restrict__ mcol,
                                                          const VT* __restrict__ mval, const double* __restrict__ mass,
                                                          const uint8_t* __restrict__ pinned, const double* __restrict__ z,
                                                          const double* __restrict__ pold, double* __restrict__ pnew,
                                                          double* __restrict__ q, long nv, double dt2,
                                                          double* __restrict__ ppart, long npart) {
    double be;
    if (!ms_iteration_state(cst, sin, sout, upart, ung, be)) return;
    constexpr int ROWS = kMsBlk / LANES;
    const int lane = threadIdx.x % LANES;
    double v[1] = {0.0};
    for (long i = blockIdx.x * long(ROWS) + threadIdx.x / LANES; i - threadIdx.x / LANES < nv;
         i += long(gridDim.x) * ROWS) {
    constexpr bool DIFF = sizeof(VT) == 4;
    double a[3] = {0.0, 0.0, 0.0};
    if (i < nv) {
        double po[3] = {0.0, 0.0, 0.0};  // the row's own direction (difference form)
        if constexpr (DIFF)
            for (int c = 0; c < 3; ++c) po[c] = z[3 * i + c] + be * pold[3 * i + c];
        for (long e = srow[i] + lane; e < srow[i + 1]; e += LANES) {
            const long j = scol[e];
            const double k = double(sval[e]);
            for (int c = 0; c < 3; ++c) a[c] += k * (z[3 * j + c] + be * pold[3 * j + c] - po[c]);
        }
        for (long e = mrow[i] + lane; e < mrow[i + 1]; e += LANES) {
            const long j = mcol[e];
            const VT* b = mval + 9 * e;
            const double pj[3] = {z[3 * j] + be * pold[3 * j] - po[0], z[3 * j + 1] + be * pold[3 * j + 1] - po[1],
                                  z[3 * j + 2] + be * pold[3 * j + 2] - po[2]};
            for (int c = 0; c < 3; ++c)
                a[c] += double(b[3 * c]) * pj[0] + double(b[3 * c + 1]) * pj[1] + double(b[3 * c + 2]) * pj[2];
        }
    }
    for (int off = LANES / 2; off > 0; off >>= 1)
        for (int c = 0; c < 3; ++c) a[c] += __shfl_xor(a[c], off, LANES);
    if (i < nv && lane == 0)
        for (int c = 0; c < 3; ++c) {
            const double pi = z[3 * i + c] + be * pold[3 * i + c];
            pnew[3 * i + c] = pi;
            const double qi = (pinned[i] >> c & 1u) ? 0.0 : mass[i] * pi + dt2 * a[c];
            q[3 * i + c] = qi;
            v[0] += pi * qi;
        }
    }
    ms_partials<1>(v, ppart, npart);
}

// The same product over SELL-64 slices with the rows in groups of G (ms_group_rows), one work-group per group
// (striding over the groups with at most kMsPartMax work-groups): the group's new directions
// p_new = z + beta p_old at its distinct columns are formed once into LDS, then each lane takes one row
// through K_s (the bending Hessian's slots) and through the blocks' nine component arrays.  A slice's
// width and offset are the same in every lane of its wave, and consecutive lanes read consecutive slots,
// so every load of ids and values is coalesced; padding slots hold zero values.  Rows past nv in the last
// slice run the loops on their padding and store nothing.  The matrix values, read once per product, are
// loaded non-temporally so that they do not displace the staged directions' sources and the vectors the
// update reads next from the caches (measured at 1M vertices: 173 -> 144 us FP64, 112 -> 92 us mixed).
template <typename VT, int G>
__global__ __launch_bounds__(G) void ms_iter_product_staged(
    const double* cst, const double* __restrict__ sin, double* __restrict__ sout, const double* __restrict__ upart,
    long ung, const int64_t* __restrict__ sptr, const int32_t* __restrict__ swidth,
    const uint16_t* __restrict__ slcol, const VT* __restrict__ sval, const int64_t* __restrict__ mptr,
    const int32_t* __restrict__ mwidth, const uint16_t* __restrict__ mlcol, const VT* __restrict__ mval, long mstride,
    const int32_t* __restrict__ gptr, const int32_t* __restrict__ gcols, const int32_t* __restrict__ gself,
    const double* __restrict__ mass, const uint8_t* __restrict__ pinned, const double* __restrict__ z,
    const double* __restrict__ pold, double* __restrict__ pnew, double* __restrict__ q, long nv, double dt2,
    double* __restrict__ ppart) {
    extern __shared__ double ps[];
    __shared__ double red[G / 64];
    double be;
    if (!ms_iteration_state(cst, sin, sout, upart, ung, be)) return;
    constexpr bool DIFF = sizeof(VT) == 4;
    const long ngroups = (nv + G - 1) / G, nslices = (nv + 63) / 64;
    double v = 0.0;
    for (long g = blockIdx.x; g < ngroups; g += gridDim.x) {
        const int a0 = gptr[g], n = gptr[g + 1] - a0;
        __syncthreads();  // the previous group's rows have read ps
        for (int k = threadIdx.x; k < n; k += blockDim.x) {
            const long j = gcols[a0 + k];
            for (int c = 0; c < 3; ++c) ps[3 * k + c] = z[3 * j + c] + be * pold[3 * j + c];
        }
        __syncthreads();
        const long i = g * G + threadIdx.x;
        const long slice = i >> 6;
        if (slice >= nslices) continue;  // whole waves past the last slice
        double po[3] = {0.0, 0.0, 0.0};
        if (i < nv)
            for (int c = 0; c < 3; ++c) po[c] = ps[3 * (gself[g] + threadIdx.x) + c];
        double a[3] = {0.0, 0.0, 0.0};
        {
            const int w = __builtin_amdgcn_readfirstlane(swidth[slice]);
            const long s0 = uniform64(sptr[slice]) + (i & 63);
            for (int k = 0; k < w; ++k) {
                const long o = s0 + 64L * k;
                const double kv = double(__builtin_nontemporal_load(sval + o));
                const double* pc = ps + 3 * int(slcol[o]);
                for (int c = 0; c < 3; ++c) a[c] = fma(kv, DIFF ? pc[c] - po[c] : pc[c], a[c]);
            }
        }
        {
            const int w = __builtin_amdgcn_readfirstlane(mwidth[slice]);
            const long m0 = uniform64(mptr[slice]) + (i & 63);
            for (int k = 0; k < w; ++k) {
                const long o = m0 + 64L * k;
                const double* pc = ps + 3 * int(mlcol[o]);
                const double d[3] = {DIFF ? pc[0] - po[0] : pc[0], DIFF ? pc[1] - po[1] : pc[1],
                                     DIFF ? pc[2] - po[2] : pc[2]};
                for (int r = 0; r < 3; ++r)
                    a[r] += double(__builtin_nontemporal_load(mval + o + (3 * r) * mstride)) * d[0] +
                            double(__builtin_nontemporal_load(mval + o + (3 * r + 1) * mstride)) * d[1] +
                            double(__builtin_nontemporal_load(mval + o + (3 * r + 2) * mstride)) * d[2];
            }
        }
        if (i < nv)
            for (int c = 0; c < 3; ++c) {
                const double pi = po[c];
                pnew[3 * i + c] = pi;
                const double qi = (pinned[i] >> c & 1u) ? 0.0 : mass[i] * pi + dt2 * a[c];
                q[3 * i + c] = qi;
                v += pi * qi;
            }
    }
    v = wave_sum(v);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int w = 0; w < G / 64; ++w) t += red[w];
        ppart[blockIdx.x] = t;
    }
}

// The update sums the product's partials itself (FUSED) up to this many partials, and the product the
// update's (finishing the previous iteration) up to this many.
// (every update work-group summing the product's 2048 partials at 1M vertices, against ms_iter_alpha:
// 31.2 against 31.6 ms per FP64 step, 23.2 against 23.4 mixed; so every product partial count, at most
// kMsPartMax, is summed in the update, and ms_iter_alpha serves a lower setting of this limit)
#ifndef SHELL_MS_FUSE_ALPHA_MAX
#define SHELL_MS_FUSE_ALPHA_MAX 2048
#endif
constexpr long kMsFuseAlphaMax = SHELL_MS_FUSE_ALPHA_MAX;
// (finishing the previous update in every product work-group, against a settle kernel after every
// iteration, measured on SS cylinders: 131K vertices, 512 update partials, 9.7 against 10.4 ms per FP64
// step and 8.5 against 9.2 mixed; 262K, 1024 partials, 14.2 against 14.8 and 11.5 against 11.9; at 1M
// vertices, 2048 partials, 151 against 144 us per product and slower steps)
#ifndef SHELL_MS_FUSE_FINISH_MAX
#define SHELL_MS_FUSE_FINISH_MAX 1024
#endif
constexpr long kMsFuseFinishMax = SHELL_MS_FUSE_FINISH_MAX;

// p.q from the product's partials (one work-group, fixed order), then alpha = r.z / p.q, in the state set
// `st` that the product wrote
__global__ __launch_bounds__(kMsBlk) void ms_iter_alpha(const double* __restrict__ ppart, long npart,
                                                        double* __restrict__ st) {
    if (st[S_ACTIVE] == 0.0) return;
    double pq[1];
    ms_totals<1>(ppart, npart, pq);
    if (threadIdx.x == 0) {
        st[S_PQ] = pq[0];
        st[S_ALPHA] = pq[0] != 0.0 ? st[S_RZ] / pq[0] : 0.0;
    }
}

// y += alpha p, r -= alpha q, z = D^-1 r; partials r.z and r.r.  alpha from ms_iter_alpha, or, with FUSED
// (few product partials), summed by every work-group itself from the product's partials in the same fixed
// order as ms_iter_alpha sums them (the same bits), which saves that launch on small meshes.  `st`: the
// state set the product wrote.
template <bool FUSED>
__global__ __launch_bounds__(kMsBlk) void ms_iter_update(const double* __restrict__ st, const double* __restrict__ p,
                                                         const double* __restrict__ q, const double* __restrict__ dinv,
                                                         double* __restrict__ y, double* __restrict__ r,
                                                         double* __restrict__ z, long nv, double* __restrict__ part,
                                                         long ngroups, const double* __restrict__ ppart, long npart) {
    if (st[S_ACTIVE] == 0.0) return;
    double al;
    if constexpr (FUSED) {
        __shared__ double al_sh;
        double pq[1];
        ms_totals<1>(ppart, npart, pq);
        if (threadIdx.x == 0) al_sh = pq[0] != 0.0 ? st[S_RZ] / pq[0] : 0.0;
        __syncthreads();
        al = al_sh;
    } else {
        al = st[S_ALPHA];
    }
    double v[2] = {0.0, 0.0};
    for (long i = blockIdx.x * long(blockDim.x) + threadIdx.x; i < nv; i += long(gridDim.x) * blockDim.x)
        for (int c = 0; c < 3; ++c) {
            y[3 * i + c] += al * p[3 * i + c];
            const double ri = r[3 * i + c] - al * q[3 * i + c], zi = dinv[i] * ri;
            r[3 * i + c] = ri;
            z[3 * i + c] = zi;
            v[0] += ri * zi;
            v[1] += ri * ri;
        }
    ms_partials<2>(v, part, ngroups);
}

// Small meshes (at most kMsSmallRows vertices): the whole PCG iteration in one work-group, up to `count`
// iterations per launch, work-group barriers in place of the kernel boundaries of the chain above (whose
// launches, some microseconds each, dominate at these sizes).  The direction p and the product q live in
// LDS for the launch (p is read from and written back to m.p at its ends); LANES lanes share a row's
// entries (consecutive lanes, consecutive entries) and combine their sums by shuffles.  The same
// recurrence and stop test: p = z + beta p, q with held coordinates zero, alpha = r.z / p.q, y, r, z
// updated, then beta, the count, the budget and the activity from r.z and r.r exactly as ms_finish_to
// takes them (in state set 0).  Sums are per wave, then over the waves in a fixed order, so a run is reproducible; VT as
// in ms_iter_product (float32 entries in difference form).  Measured: one thread per row of a
// 1088-vertex mesh took 38 us per iteration (each row's gathers one after another), three times the
// kernel chain; with p in LDS and several lanes per row the one-work-group solver wins up to some
// hundreds of vertices.
constexpr int kMsSmallThreads = 1024;
constexpr long kMsSmallRows = 512;
constexpr int kMsSmallChunk = 4096;  // iterations per launch at most (the host loop launches again)

template <int NQ>
__device__ __forceinline__ void ms_small_sum(double (&v)[NQ], double* sh) {
    constexpr int NW = kMsSmallThreads / 64;
    for (int q = 0; q < NQ; ++q) v[q] = wave_sum(v[q]);
    __syncthreads();  // the previous sum's readers are done with sh
    if ((threadIdx.x & 63) == 0)
        for (int q = 0; q < NQ; ++q) sh[q * NW + (threadIdx.x >> 6)] = v[q];
    __syncthreads();
    for (int q = 0; q < NQ; ++q) {
        double t = 0.0;
        for (int w = 0; w < NW; ++w) t += sh[q * NW + w];
        v[q] = t;  // every thread, the same order
    }
}

template <typename VT, int LANES>
__global__ __launch_bounds__(kMsSmallThreads) void ms_pcg_small(
    double* __restrict__ scal, const int64_t* __restrict__ srow, const int32_t* __restrict__ scol,
    const VT* __restrict__ sval, const int64_t* __restrict__ mrow, const int32_t* __restrict__ mcol,
    const VT* __restrict__ mval, const double* __restrict__ mass, const uint8_t* __restrict__ pinned,
    const double* __restrict__ dinv, double* __restrict__ z, double* __restrict__ pg, double* __restrict__ y,
    double* __restrict__ r, long nv, double dt2, int count) {
    __shared__ double sh[2 * (kMsSmallThreads / 64)];
    __shared__ double ps[3 * kMsSmallRows], qs[3 * kMsSmallRows];
    constexpr bool DIFF = sizeof(VT) == 4;
    constexpr int ROWS = kMsSmallThreads / LANES;
    const int lane = threadIdx.x % LANES;
    for (long i = threadIdx.x; i < 3 * nv; i += blockDim.x) ps[i] = pg[i];
    __syncthreads();
    for (int k = 0; k < count; ++k) {
        if (scal[S_ACTIVE] == 0.0) break;  // every thread reads it after the same barrier
        const double be = scal[S_BETA];
        for (long i = threadIdx.x; i < 3 * nv; i += blockDim.x) ps[i] = z[i] + be * ps[i];
        __syncthreads();
        double pq[1] = {0.0};
        for (long i0 = 0; i0 < nv; i0 += ROWS) {  // every lane of a row group takes part in the shuffles
            const long i = i0 + threadIdx.x / LANES;
            double a[3] = {0.0, 0.0, 0.0};
            double po[3] = {0.0, 0.0, 0.0};
            if (i < nv) {
                if constexpr (DIFF)
                    for (int c = 0; c < 3; ++c) po[c] = ps[3 * i + c];
                for (long e = srow[i] + lane; e < srow[i + 1]; e += LANES) {
                    const long j = scol[e];
                    const double kv = double(sval[e]);
                    for (int c = 0; c < 3; ++c) a[c] += kv * (ps[3 * j + c] - po[c]);
                }
                for (long e = mrow[i] + lane; e < mrow[i + 1]; e += LANES) {
                    const long j = mcol[e];
                    const VT* b = mval + 9 * e;
                    const double pj[3] = {ps[3 * j] - po[0], ps[3 * j + 1] - po[1], ps[3 * j + 2] - po[2]};
                    for (int c = 0; c < 3; ++c)
                        a[c] += double(b[3 * c]) * pj[0] + double(b[3 * c + 1]) * pj[1] + double(b[3 * c + 2]) * pj[2];
                }
            }
            for (int off = LANES / 2; off > 0; off >>= 1)
                for (int c = 0; c < 3; ++c) a[c] += __shfl_xor(a[c], off, LANES);
            if (i < nv && lane == 0)
                for (int c = 0; c < 3; ++c) {
                    const double pi = ps[3 * i + c];
                    const double qi = (pinned[i] >> c & 1u) ? 0.0 : mass[i] * pi + dt2 * a[c];
                    qs[3 * i + c] = qi;
                    pq[0] += pi * qi;
                }
        }
        ms_small_sum<1>(pq, sh);
        const double al = pq[0] != 0.0 ? scal[S_RZ] / pq[0] : 0.0;
        double v[2] = {0.0, 0.0};
        for (long i = threadIdx.x; i < 3 * nv; i += blockDim.x) {
            y[i] += al * ps[i];
            const double ri = r[i] - al * qs[i], zi = dinv[i / 3] * ri;
            r[i] = ri;
            z[i] = zi;
            v[0] += ri * zi;
            v[1] += ri * ri;
        }
        ms_small_sum<2>(v, sh);
        if (threadIdx.x == 0) {
            scal[S_PQ] = pq[0];
            scal[S_ALPHA] = al;
            const double rz = scal[S_RZ];
            scal[S_BETA] = rz != 0.0 ? v[0] / rz : 0.0;
            scal[S_RZ] = v[0];
            scal[S_RR] = v[1];
            const double it = scal[S_IT] + 1.0, target = scal[S_TARGET];
            const bool replay = scal[S_REPLAY] != 0.0;
            const bool more = replay || v[1] > scal[S_TOL2];
            if (!replay && it >= target && more) scal[S_BUDGET] = 1.0;
            scal[S_IT] = it;
            scal[S_ACTIVE] = (it < target && more && isfinite(v[1])) ? 1.0 : 0.0;
            if (!isfinite(v[1])) scal[S_BUDGET] = 2.0;
        }
        __syncthreads();  // the scalars and this iteration's vectors are in place for the next
    }
    for (long i = threadIdx.x; i < 3 * nv; i += blockDim.x) pg[i] = ps[i];
}

template <typename VT, int L>
void launch_pcg_small_lanes(MembraneSolve& m, const VT* sval, const VT* mval, const double* mass,
                            const uint8_t* pinned, long nv, double dt2, hipStream_t s) {
    ms_pcg_small<VT, L><<<1, kMsSmallThreads, 0, s>>>(m.scal.p, m.srow.p, m.scol.p, sval, m.mrow.p, m.mcol.p, mval,
                                                      mass, pinned, m.dinv.p, m.z.p, m.p.p, m.y.p, m.r.p, nv, dt2,
                                                      kMsSmallChunk);
}

template <typename VT>
void launch_pcg_small(MembraneSolve& m, const VT* sval, const VT* mval, const double* mass, const uint8_t* pinned,
                      long nv, double dt2, hipStream_t s) {
    // lanes per row: as many as the work-group has to spare, at most 16
    const long spare = kMsSmallThreads / std::max(nv, 1L);
    if (spare >= 16)
        launch_pcg_small_lanes<VT, 16>(m, sval, mval, mass, pinned, nv, dt2, s);
    else if (spare >= 8)
        launch_pcg_small_lanes<VT, 8>(m, sval, mval, mass, pinned, nv, dt2, s);
    else if (spare >= 4)
        launch_pcg_small_lanes<VT, 4>(m, sval, mval, mass, pinned, nv, dt2, s);
    else
        launch_pcg_small_lanes<VT, 2>(m, sval, mval, mass, pinned, nv, dt2, s);
}

// The end of a chunk of iterations (one block): the last update's state finished in place in set `cur`
// and marked settled, so that the host reads the exact state and the next chunk's first product takes it
// as it is.
__global__ __launch_bounds__(kMsBlk) void ms_iter_settle(const double* __restrict__ upart, long ung, double* scal,
                                                         int cur) {
    double* st = scal + S_COUNT * cur;
    if (st[S_FRESH] != 0.0 || st[S_ACTIVE] == 0.0) return;
    double t[2];
    ms_update_totals<32>(upart, ung, t);
    if (threadIdx.x == 0) {
        ms_finish_to(scal, st, t, st);
        st[S_FRESH] = 1.0;
    }
}

// largest |y| entry: per-block maxima, then their maximum
__global__ __launch_bounds__(kMsBlk) void ms_absmax(const double* __restrict__ y, long n, double* __restrict__ part,
                                                    long ngroups) {
    double m = 0.0;
    for (long i = blockIdx.x * long(blockDim.x) + threadIdx.x; i < n; i += long(gridDim.x) * blockDim.x)
        m = fmax(m, fabs(y[i]));
    __shared__ double sh[kMsBlk];
    sh[threadIdx.x] = m;
    __syncthreads();
    for (int w = kMsBlk / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) sh[threadIdx.x] = fmax(sh[threadIdx.x], sh[threadIdx.x + w]);
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

__global__ __launch_bounds__(kMsBlk) void ms_fin_max(const double* __restrict__ part, long ngroups,
                                                     double* __restrict__ scal) {
    double m = 0.0;
    for (long b = threadIdx.x; b < ngroups; b += blockDim.x) m = fmax(m, part[b]);
    __shared__ double sh[kMsBlk];
    sh[threadIdx.x] = m;
    __syncthreads();
    for (int w = kMsBlk / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) sh[threadIdx.x] = fmax(sh[threadIdx.x], sh[threadIdx.x + w]);
        __syncthreads();
    }
    if (threadIdx.x == 0) scal[S_YMAX] = sh[0];
}

}  // namespace

MembraneSolve::~MembraneSolve() {
    RuntimeLock lk(runtime_mutex());
    for (auto& g : graphs) (void)hipGraphExecDestroy(g.ex);
    if (capture) (void)hipStreamDestroy(capture);
    if (lane) (void)hipStreamDestroy(lane);
    if (ready) (void)hipEventDestroy(ready);
    if (hscal) (void)hipHostFree(hscal);
}

void launch_membrane_rest(shell_stencils_s& st, hipStream_t s) {
    const long nt = st.nt;
    DevArray<double> rest(size_t(5 * nt));
    DevArray<int32_t> bad(1);
    SHELL_HIP(hipMemsetAsync(bad.p, 0, sizeof(int32_t), s));
    if (nt > 0) membrane_rest<<<int((nt + 255) / 256), 256, 0, s>>>(st.X.p, st.tris.p, nt, rest.p, bad.p);
    SHELL_HIP(hipGetLastError());
    int32_t h = 0;
    bad.download(&h, 1, s);
    SHELL_HIP(hipStreamSynchronize(s));
    SHELL_CHECK(h == 0, SHELL_E_DEGENERATE, "degenerate triangle (zero area) for the membrane");
    // the triangles in the bending kernel's vertex tiles
    Tiling til = build_tiling(st.h_tris, 3, nt, st.nv, st.T);
    st.mboff.alloc(til.boff.size());
    st.mboff.upload(til.boff.data(), til.boff.size(), s);
    DevArray<int32_t> src(til.src.size());
    src.upload(til.src.data(), til.src.size(), s);
    const long n = long(til.src.size());
    st.mtid.alloc(size_t(4 * n));
    st.mtrest.alloc(size_t(6 * n));
    if (n > 0)
        membrane_tile_copy<<<int((n + 255) / 256), 256, 0, s>>>(src.p, n, st.tris.p, rest.p, st.mtid.p, st.mtrest.p);
    SHELL_HIP(hipGetLastError());
    st.mepart.alloc(size_t(st.nblocks));
    SHELL_HIP(hipStreamSynchronize(s));  // the temporaries are released on return
}

void launch_membrane_forces(shell_stencils_s& st, const double* pos, void* f, hipStream_t s, double* epart) {
    if (st.nv == 0 || st.nblocks == 0) return;
    double* ep = epart ? epart : st.mepart.p;
    const double c = st.young * st.thickness / (1.0 - st.poisson * st.poisson);
    const unsigned grid = unsigned(st.nblocks);
    if (st.precision == SHELL_PREC_MIXED)
        membrane_tiles<float><<<grid, kMembThreads, TileAccT<1>::bytes(st.T), s>>>(pos, st.mtid.p, st.mtrest.p, st.mboff.p,
                                                              st.nv, st.T, c, st.poisson, st.mscale, static_cast<float*>(f),
                                                              ep);
    else
        membrane_tiles<double><<<grid, kMembThreads, TileAccT<2>::bytes(st.T), s>>>(pos, st.mtid.p, st.mtrest.p, st.mboff.p,
                                                               st.nv, st.T, c, st.poisson, st.mscale, static_cast<double*>(f),
                                                               ep);
    SHELL_HIP(hipGetLastError());
}

namespace {

__global__ void ms_gather_csr(const double* __restrict__ val, const int64_t* __restrict__ csr2sell, long nnz,
                              double* __restrict__ out) {
    long e = blockIdx.x * long(blockDim.x) + threadIdx.x;
    if (e < nnz) out[e] = val[csr2sell[e]];
}

__global__ void ms_narrow(const double* __restrict__ src, float* __restrict__ dst, long n) {
    long i = blockIdx.x * long(blockDim.x) + threadIdx.x;
    if (i < n) dst[i] = float(src[i]);
}

__global__ void ms_widen(const float* __restrict__ src, double* __restrict__ dst, long n) {
    long i = blockIdx.x * long(blockDim.x) + threadIdx.x;
    if (i < n) dst[i] = double(src[i]);
}

__global__ void ms_zero(double* __restrict__ p, long n) {
    long i = blockIdx.x * long(blockDim.x) + threadIdx.x;
    if (i < n) p[i] = 0.0;
}

inline unsigned ms_grid(long n) { return unsigned(std::max(1L, (n + kMsBlk - 1) / kMsBlk)); }

// Rows per group of the staged product: the largest of 512 and 256 that still makes at least 256 groups
// (one work-group per CU), else 128, so that mid-size meshes fill the chip; smaller groups stage more
// neighbouring columns per row.  Measured on SS cylinders against at least 512 and 1024 groups: 65K
// vertices (256-row groups) 12.4 ms per FP64 step against 13.6 (128-row) and 13.6; 131K and 262K equal
// within 2%, or 8-13% slower with 1024.
#ifndef SHELL_MS_MIN_GROUPS
#define SHELL_MS_MIN_GROUPS 256
#endif
inline int ms_group_rows(long nv) {
    for (int g : {512, 256})
        if ((nv + g - 1) / g >= SHELL_MS_MIN_GROUPS) return g;
    return 128;
}

}  // namespace

void membrane_sim_init(shell_sim_s& sim, hipStream_t s) {
    shell_stencils_s& st = *sim.st;
    shell_hessian_s& h = *sim.h;
    auto ms = std::make_unique<MembraneSolve>();
    const long nv = st.nv, nt = st.nt, n3 = 3 * nv;
    const SellPattern& pat = h.pat;
    ms->mixed = st.precision == SHELL_PREC_MIXED;
    // membrane block pattern: each vertex, its triangle neighbours and itself, sorted
    std::vector<std::vector<int32_t>> nb(static_cast<size_t>(nv));
    for (long i = 0; i < nv; ++i) nb[size_t(i)].push_back(int32_t(i));
    for (long t = 0; t < nt; ++t)
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b)
                if (a != b) nb[size_t(st.h_tris[size_t(3 * t + a)])].push_back(st.h_tris[size_t(3 * t + b)]);
    std::vector<int64_t> mrow(size_t(nv + 1), 0), mdiag(size_t(nv), 0);
    std::vector<int32_t> mcol;
    for (long i = 0; i < nv; ++i) {
        auto& v = nb[size_t(i)];
        std::sort(v.begin(), v.end());
        v.erase(std::unique(v.begin(), v.end()), v.end());
        for (int32_t j : v) {
            if (j == i) mdiag[size_t(i)] = int64_t(mcol.size());
            mcol.push_back(j);
        }
        mrow[size_t(i + 1)] = int64_t(mcol.size());
    }
    ms->mrow.alloc(mrow.size());
    ms->mrow.upload(mrow.data(), mrow.size(), s);
    ms->mcol.alloc(std::max<size_t>(mcol.size(), 1));
    ms->mcol.upload(mcol.data(), mcol.size(), s);
    // where each block is stored: CSR order (the direct product), or SELL-64 slices for the staged one
    const int64_t nnz_m = int64_t(mcol.size());
    std::vector<int64_t> mbase(size_t(std::max<int64_t>(nnz_m, 1)), 0);
    int64_t nblock_vals = 9 * nnz_m;
    ms->staged = (st.cfg_flags & SHELL_FLAG_DIRECT_PRODUCT) == 0 && nv >= kMsStagedMinRows;
    if (ms->staged) {
        // each row group's distinct columns of K_s and of the blocks, with its own rows
        const int64_t G = ms_group_rows(nv);
        const int64_t ng = (nv + G - 1) / G, nsl = (nv + 63) / 64;
        std::vector<std::vector<int32_t>> gl(static_cast<size_t>(ng));
        for (int64_t g = 0; g < ng; ++g) {
            auto& v = gl[size_t(g)];
            for (int64_t i = g * G; i < std::min<int64_t>(nv, (g + 1) * G); ++i) {
                v.push_back(int32_t(i));
                v.insert(v.end(), pat.col.begin() + pat.rowptr[size_t(i)], pat.col.begin() + pat.rowptr[size_t(i + 1)]);
                v.insert(v.end(), mcol.begin() + mrow[size_t(i)], mcol.begin() + mrow[size_t(i + 1)]);
            }
            std::sort(v.begin(), v.end());
            v.erase(std::unique(v.begin(), v.end()), v.end());
            ms->max_gcols = std::max<int32_t>(ms->max_gcols, int32_t(v.size()));
        }
        ms->staged = ms->max_gcols <= kMaxGroupCols && pat.nslices == nsl;
        if (ms->staged) {
            auto local = [&](int64_t g, int32_t c) {  // index of column c in group g's list (0 if absent)
                const auto& v = gl[size_t(g)];
                auto it = std::lower_bound(v.begin(), v.end(), c);
                return (it != v.end() && *it == c) ? uint16_t(it - v.begin()) : uint16_t(0);
            };
            std::vector<int32_t> gptr(static_cast<size_t>(ng + 1), 0), gcols, gself(static_cast<size_t>(ng));
            for (int64_t g = 0; g < ng; ++g) {
                gptr[size_t(g + 1)] = gptr[size_t(g)] + int32_t(gl[size_t(g)].size());
                gcols.insert(gcols.end(), gl[size_t(g)].begin(), gl[size_t(g)].end());
                gself[size_t(g)] = local(g, int32_t(g * G));
            }
            std::vector<uint16_t> slcol(size_t(pat.nslots));
            for (int64_t sl = 0; sl < nsl; ++sl)
                for (int64_t slot = pat.sptr[size_t(sl)]; slot < pat.sptr[size_t(sl + 1)]; ++slot)
                    slcol[size_t(slot)] = local((64 * sl) / G, pat.scol[size_t(slot)]);
            std::vector<int32_t> mwidth(static_cast<size_t>(nsl));
            std::vector<int64_t> mptr(size_t(nsl + 1), 0);
            for (int64_t sl = 0; sl < nsl; ++sl) {
                int w = 1;
                for (int64_t i = 64 * sl; i < std::min<int64_t>(nv, 64 * sl + 64); ++i)
                    w = std::max(w, int(mrow[size_t(i + 1)] - mrow[size_t(i)]));
                mwidth[size_t(sl)] = w;
                mptr[size_t(sl + 1)] = mptr[size_t(sl)] + 64 * int64_t(w);
            }
            const int64_t mslots = mptr[size_t(nsl)];
            std::vector<uint16_t> mlcol(size_t(mslots), 0);
            std::vector<int64_t> s2e(size_t(mslots), -1);
            for (int64_t sl = 0; sl < nsl; ++sl)
                for (int lane = 0; lane < 64; ++lane) {
                    const int64_t i = 64 * sl + lane, g = i / G;
                    const int64_t len = i < nv ? mrow[size_t(i + 1)] - mrow[size_t(i)] : 0;
                    for (int64_t k = 0; k < mwidth[size_t(sl)]; ++k) {
                        const int64_t slot = mptr[size_t(sl)] + 64 * k + lane;
                        if (k < len) {
                            const int64_t e = mrow[size_t(i)] + k;
                            mbase[size_t(e)] = slot;
                            s2e[size_t(slot)] = e;
                            mlcol[size_t(slot)] = local(g, mcol[size_t(e)]);
                        } else {
                            mlcol[size_t(slot)] = i < nv ? local(g, int32_t(i)) : uint16_t(0);  // zero value
                        }
                    }
                }
            ms->mstride = mslots;
            nblock_vals = 9 * mslots;
            ms->hsptr = h.sptr.p;
            ms->hwidth = h.width.p;
            ms->hval = h.val.p;
            ms->hvalf = h.valf.p;
            SHELL_CHECK(!ms->mixed || ms->hvalf, SHELL_E_INVALID_ARG, "mixed precision needs the float32 K_s");
            ms->gptr.alloc(gptr.size());
            ms->gptr.upload(gptr.data(), gptr.size(), s);
            ms->gcols.alloc(std::max<size_t>(gcols.size(), 1));
            ms->gcols.upload(gcols.data(), gcols.size(), s);
            ms->gself.alloc(gself.size());
            ms->gself.upload(gself.data(), gself.size(), s);
            ms->slcol.alloc(std::max<size_t>(slcol.size(), 1));
            ms->slcol.upload(slcol.data(), slcol.size(), s);
            ms->mwidth.alloc(mwidth.size());
            ms->mwidth.upload(mwidth.data(), mwidth.size(), s);
            ms->mptr.alloc(mptr.size());
            ms->mptr.upload(mptr.data(), mptr.size(), s);
            ms->mlcol.alloc(mlcol.size());
            ms->mlcol.upload(mlcol.data(), mlcol.size(), s);
            ms->s2e.alloc(s2e.size());
            ms->s2e.upload(s2e.data(), s2e.size(), s);
            SHELL_HIP(hipStreamSynchronize(s));  // the host copies are released on leaving the scope
        }
    }
    if (!ms->staged) {
        ms->mstride = 1;
        for (int64_t e = 0; e < nnz_m; ++e) mbase[size_t(e)] = 9 * e;
    }
    DevArray<int64_t> c2s;
    if (!ms->staged) {  // the direct product reads K_s as CSR, gathered from the assembled SELL slots
        ms->srow.alloc(pat.rowptr.size());
        ms->srow.upload(pat.rowptr.data(), pat.rowptr.size(), s);
        ms->scol.alloc(std::max<size_t>(pat.col.size(), 1));
        ms->scol.upload(pat.col.data(), pat.col.size(), s);
        ms->sval.alloc(std::max<size_t>(pat.col.size(), 1));
        c2s.alloc(std::max<size_t>(pat.csr2sell.size(), 1));
        c2s.upload(pat.csr2sell.data(), pat.csr2sell.size(), s);
        if (!pat.col.empty())
            ms_gather_csr<<<ms_grid(long(pat.col.size())), kMsBlk, 0, s>>>(h.val.p, c2s.p, long(pat.col.size()),
                                                                            ms->sval.p);
        if (ms->mixed) {
            ms->svalf.alloc(std::max<size_t>(pat.col.size(), 1));
            if (!pat.col.empty())
                ms_narrow<<<ms_grid(long(pat.col.size())), kMsBlk, 0, s>>>(ms->sval.p, ms->svalf.p,
                                                                            long(pat.col.size()));
        }
    }
    for (long i = 0; i < nv; ++i) mdiag[size_t(i)] = mbase[size_t(mdiag[size_t(i)])];
    ms->mbase.alloc(mbase.size());
    ms->mbase.upload(mbase.data(), mbase.size(), s);
    ms->mdiag.alloc(std::max<size_t>(mdiag.size(), 1));
    ms->mdiag.upload(mdiag.data(), mdiag.size(), s);
    ms->mval.alloc(size_t(std::max<int64_t>(nblock_vals, 1)));
    if (ms->mixed) ms->mvalf.alloc(size_t(std::max<int64_t>(nblock_vals, 1)));
    // each block's row, and the triangles holding both of its vertices, ascending (the tangent assembly's
    // fixed order): every triangle adds to the nine blocks of its corner pairs
    std::vector<int32_t> brow(size_t(std::max<int64_t>(nnz_m, 1)), 0);
    for (long i = 0; i < nv; ++i)
        for (int64_t e = mrow[size_t(i)]; e < mrow[size_t(i + 1)]; ++e) brow[size_t(e)] = int32_t(i);
    auto entry = [&](int32_t i, int32_t j) {
        auto lo = mcol.begin() + mrow[size_t(i)], hi = mcol.begin() + mrow[size_t(i + 1)];
        return int64_t(std::lower_bound(lo, hi, j) - mcol.begin());
    };
    std::vector<int64_t> btptr(size_t(nnz_m + 1), 0);
    for (long t = 0; t < nt; ++t)
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b)
                ++btptr[size_t(entry(st.h_tris[size_t(3 * t + a)], st.h_tris[size_t(3 * t + b)]) + 1)];
    for (int64_t e = 0; e < nnz_m; ++e) btptr[size_t(e + 1)] += btptr[size_t(e)];
    std::vector<int32_t> bttri(size_t(std::max(9 * nt, 1L)));
    {
        std::vector<int64_t> fill(btptr.begin(), btptr.end() - 1);
        for (long t = 0; t < nt; ++t)
            for (int a = 0; a < 3; ++a)
                for (int b = 0; b < 3; ++b)
                    bttri[size_t(fill[size_t(entry(st.h_tris[size_t(3 * t + a)], st.h_tris[size_t(3 * t + b)]))]++)] =
                        int32_t(t);
    }
    ms->brow.alloc(brow.size());
    ms->brow.upload(brow.data(), brow.size(), s);
    ms->btptr.alloc(btptr.size());
    ms->btptr.upload(btptr.data(), btptr.size(), s);
    ms->bttri.alloc(bttri.size());
    ms->bttri.upload(bttri.data(), size_t(9 * nt), s);
    // the blocks' padding slots (staged layout) stay zero: the assembly writes every stored block
    if (ms->mval.n) ms_zero<<<ms_grid(long(ms->mval.n)), kMsBlk, 0, s>>>(ms->mval.p, long(ms->mval.n));
    if (ms->mixed && ms->mval.n)
        ms_narrow<<<ms_grid(long(ms->mval.n)), kMsBlk, 0, s>>>(ms->mval.p, ms->mvalf.p, long(ms->mval.n));
    // per-triangle rest data
    ms->rest.alloc(size_t(std::max(5 * nt, 1L)));
    DevArray<int32_t> bad(1);
    SHELL_HIP(hipMemsetAsync(bad.p, 0, sizeof(int32_t), s));
    if (nt > 0) membrane_rest<<<int((nt + 255) / 256), 256, 0, s>>>(st.X.p, st.tris.p, nt, ms->rest.p, bad.p);
    for (auto* a : {&ms->xtry, &ms->ftry, &ms->z, &ms->p, &ms->p2, &ms->q, &ms->y, &ms->r})
        a->alloc(size_t(std::max(n3, 1L)));
    if (ms->mixed) ms->ff.alloc(size_t(std::max(n3, 1L)));
    ms->dinv.alloc(size_t(std::max(nv, 1L)));
    ms->ngroups = long(ms_grid(nv));
    ms->part.alloc(size_t(2 * ms->ngroups + std::max<int64_t>(st.nblocks, 1)));
    ms->ppart.alloc(size_t(kMsPartMax));
    ms->scal.alloc(2 * S_COUNT);  // two sets of the PCG state
    ms->mepart.alloc(size_t(std::max<int64_t>(st.nblocks, 1)));
    // bending force at xtry into ftry (mixed: into ff, widened into ftry afterwards), with its energy
    // partials after the reduction partials
    ForceDesc d{};
    d.x = ms->xtry.p;
    d.X = st.X.p;
    d.f = ms->mixed ? static_cast<void*>(ms->ff.p) : static_cast<void*>(ms->ftry.p);
    d.epart = ms->part.p + 2 * ms->ngroups;
    d.bias = st.bias.p;
    d.boff = st.boff.p;
    d.tidx = st.tidx.p;
    d.trec = ms->mixed ? static_cast<const void*>(st.trec32.p) : static_cast<const void*>(st.trec64.p);
    d.nst = st.nst_pad;
    d.nv = st.nv;
    d.T = st.T;
    d.model = st.model;
    d.kb = st.kb;
    d.fscale = st.fscale;
    d.nu = st.poisson;
    std::vector<WorkItem> items(size_t(st.nblocks));
    for (int64_t t = 0; t < st.nblocks; ++t) items[size_t(t)] = {0, int32_t(t)};
    ms->fdesc.alloc(1);
    ms->fdesc.upload(&d, 1, s);
    ms->items.alloc(std::max<size_t>(items.size(), 1));
    ms->items.upload(items.data(), items.size(), s);
    int32_t hb = 0;
    bad.download(&hb, 1, s);
    SHELL_HIP(hipStreamSynchronize(s));  // the staging above is released on return
    SHELL_CHECK(hb == 0, SHELL_E_DEGENERATE, "degenerate triangle (zero area) for the membrane");
    sim.ms = std::move(ms);
}

// Bending and membrane force at xtry into ftry (float64; mixed precision computes it in float32 into ff
// and widens it), with the energy partials of both passes.
static void forces_at_try(shell_sim_s& sim, hipStream_t s) {
    shell_stencils_s& st = *sim.st;
    MembraneSolve& m = *sim.ms;
    const long n3 = 3 * sim.nv;
    launch_force_items(st.model, st.precision, m.fdesc.p, m.items.p, st.nblocks, st.T, s);
    if (m.mixed) {
        launch_membrane_forces(st, m.xtry.p, m.ff.p, s, m.mepart.p);
        ms_widen<<<ms_grid(n3), kMsBlk, 0, s>>>(m.ff.p, m.ftry.p, n3);
    } else {
        launch_membrane_forces(st, m.xtry.p, m.ftry.p, s, m.mepart.p);
    }
    SHELL_HIP(hipGetLastError());
}

// The membrane tangent at x into the 3x3 blocks (and their float32 copy in mixed precision), and the
// Jacobi preconditioner of M + dt^2 (K_s (x) I3 + K_m) with the given mass.
static void tangent_at(shell_sim_s& sim, const double* x, const double* mass, double dt2, hipStream_t s) {
    shell_stencils_s& st = *sim.st;
    MembraneSolve& m = *sim.ms;
    const long nv = sim.nv, nt = st.nt;
    const double c = st.young * st.thickness / (1.0 - st.poisson * st.poisson);
    const long nb = long(m.mcol.n), nthreads = m.staged ? long(m.mstride) : nb;
    if (nt > 0 && nb > 0)
        ms_tangent<<<ms_grid(nthreads), kMsBlk, 0, s>>>(m.rest.p, st.tris.p, m.brow.p, m.mcol.p, m.btptr.p, m.bttri.p,
                                                        m.staged ? m.s2e.p : nullptr, nthreads, x, c, st.poisson,
                                                        m.mbase.p, long(m.mstride), m.mval.p,
                                                        m.mixed ? m.mvalf.p : nullptr);
    ms_dinv<<<ms_grid(nv), kMsBlk, 0, s>>>(sim.h->kdiag.p, m.mval.p, m.mdiag.p, long(m.mstride), mass, sim.pinned.p, nv, dt2,
                                           m.dinv.p);
    SHELL_HIP(hipGetLastError());
}

// One PCG iteration: the product kernel forms the new direction into one of the two p buffers from z and
// the other, the update kernel reads it; the buffers alternate.  Once the stop test has cleared the active
// flag all three kernels return at once, so the alternation may run on past the last iteration.
// The coupled product q = (M + dt^2 (K_s (x) I3 + K_m)) p_new with p_new = z + beta p_old written to pnew,
// and its per-work-group partials of p.q in m.ppart, after it has taken the iteration's state from set
// `sin` (finishing the previous update from its partials) and stored it into set `sout`; returns the
// number of partials.
static long launch_product(MembraneSolve& m, const double* mass, const uint8_t* pinned, long nv, double dt2,
                           const double* pold, double* pnew, const double* sin, double* sout, hipStream_t s) {
    const long ung = long(ms_update_grid(nv));
    if (m.staged) {
        const int G = ms_group_rows(nv);
        const unsigned pg = unsigned(std::min(kMsPartMax, (nv + G - 1) / G));
        const size_t lds = size_t(m.max_gcols) * 3 * sizeof(double);
        auto go = [&](auto kernel, const auto* sv, const auto* mv) {
            kernel<<<pg, G, lds, s>>>(m.scal.p, sin, sout, m.part.p, ung, m.hsptr, m.hwidth, m.slcol.p, sv, m.mptr.p,
                                      m.mwidth.p, m.mlcol.p, mv, long(m.mstride), m.gptr.p, m.gcols.p, m.gself.p, mass,
                                      pinned, m.z.p, pold, pnew, m.q.p, nv, dt2, m.ppart.p);
        };
        if (m.mixed) {
            if (G == 512) go(ms_iter_product_staged<float, 512>, m.hvalf, m.mvalf.p);
            else if (G == 256) go(ms_iter_product_staged<float, 256>, m.hvalf, m.mvalf.p);
            else go(ms_iter_product_staged<float, 128>, m.hvalf, m.mvalf.p);
        } else {
            if (G == 512) go(ms_iter_product_staged<double, 512>, m.hval, m.mval.p);
            else if (G == 256) go(ms_iter_product_staged<double, 256>, m.hval, m.mval.p);
            else go(ms_iter_product_staged<double, 128>, m.hval, m.mval.p);
        }
        return long(pg);
    }
    const unsigned pg = ms_product_grid(nv, m.mixed ? kMsLanesF32 : kMsLanesF64);
    if (m.mixed)
        ms_iter_product<float, kMsLanesF32><<<pg, kMsBlk, 0, s>>>(m.scal.p, sin, sout, m.part.p, ung, m.srow.p, m.scol.p, m.svalf.p, m.mrow.p,
                                                                  m.mcol.p, m.mvalf.p, mass, pinned, m.z.p, pold, pnew,
                                                                  m.q.p, nv, dt2, m.ppart.p, long(pg));
    else
        ms_iter_product<double, kMsLanesF64><<<pg, kMsBlk, 0, s>>>(m.scal.p, sin, sout, m.part.p, ung, m.srow.p, m.scol.p, m.sval.p, m.mrow.p,
                                                                   m.mcol.p, m.mval.p, mass, pinned, m.z.p, pold, pnew,
                                                                   m.q.p, nv, dt2, m.ppart.p, long(pg));
    return long(pg);
}

static void pcg_iteration(MembraneSolve& m, const double* mass, const uint8_t* pinned, long nv, double dt2,
                          hipStream_t s) {
    double* pold = m.pswap ? m.p2.p : m.p.p;
    double* pnew = m.pswap ? m.p.p : m.p2.p;
    const double* sin = m.scal.p + (m.pswap ? S_COUNT : 0);
    double* sout = m.scal.p + (m.pswap ? 0 : S_COUNT);
    const long np = launch_product(m, mass, pinned, nv, dt2, pold, pnew, sin, sout, s);
    const unsigned ug = ms_update_grid(nv);
    if (np <= kMsFuseAlphaMax) {
        ms_iter_update<true><<<ug, kMsBlk, 0, s>>>(sout, pnew, m.q.p, m.dinv.p, m.y.p, m.r.p, m.z.p, nv, m.part.p,
                                                   long(ug), m.ppart.p, np);
    } else {
        ms_iter_alpha<<<1, kMsBlk, 0, s>>>(m.ppart.p, np, sout);
        ms_iter_update<false><<<ug, kMsBlk, 0, s>>>(sout, pnew, m.q.p, m.dinv.p, m.y.p, m.r.p, m.z.p, nv,
                                                    m.part.p, long(ug), m.ppart.p, np);
    }
    m.pswap = !m.pswap;
    // with many update partials one work-group settles the state after every iteration instead (every
    // product work-group summing them delays the start of its stream)
    if (ug > kMsFuseFinishMax) ms_iter_settle<<<1, kMsBlk, 0, s>>>(m.part.p, long(ug), m.scal.p, m.pswap ? 1 : 0);
}

constexpr size_t kMsMaxGraphs = 16;

// `count` PCG iterations and the settling of their last update's state (which the host then reads from set
// m.pswap).  With graphs allowed a chunk is captured once on a private stream and replayed (the kernels
// read the scalars and vectors when the graph runs, so one capture serves every solve with the same mass
// array, dt and buffer parity); otherwise the kernels are launched one by one.
static void pcg_chunk(MembraneSolve& m, const double* mass, const uint8_t* pinned, long nv, double dt2, int count,
                      hipStream_t s) {
    for (int it = 0; it < count; ++it) pcg_iteration(m, mass, pinned, nv, dt2, s);
    ms_iter_settle<<<1, kMsBlk, 0, s>>>(m.part.p, long(ms_update_grid(nv)), m.scal.p, m.pswap ? 1 : 0);
}

static void pcg_iterations(MembraneSolve& m, const double* mass, const uint8_t* pinned, long nv, double dt2,
                           int count, bool graphs, hipStream_t s) {
    if (nv <= kMsSmallRows && !m.staged) {  // one work-group runs the iterations (m.p holds the direction)
        if (m.mixed)
            launch_pcg_small<float>(m, m.svalf.p, m.mvalf.p, mass, pinned, nv, dt2, s);
        else
            launch_pcg_small<double>(m, m.sval.p, m.mval.p, mass, pinned, nv, dt2, s);
        SHELL_HIP(hipGetLastError());
        (void)count;
        (void)graphs;
        return;
    }
    if (!graphs) {
        pcg_chunk(m, mass, pinned, nv, dt2, count, s);
        return;
    }
    const bool parity = m.pswap;
    hipGraphExec_t ex = nullptr;
    for (const auto& g : m.graphs)
        if (g.mass == mass && g.dt2 == dt2 && g.count == count && g.parity == parity) ex = g.ex;
    if (!ex) {
        RuntimeLock lk(runtime_mutex());
        if (!m.capture) SHELL_HIP(hipStreamCreateWithFlags(&m.capture, hipStreamNonBlocking));
        hipGraph_t g = nullptr;
        SHELL_HIP(hipStreamBeginCapture(m.capture, hipStreamCaptureModeThreadLocal));
        pcg_chunk(m, mass, pinned, nv, dt2, count, m.capture);
        const hipError_t launched = hipGetLastError();
        const hipError_t ended = hipStreamEndCapture(m.capture, &g);
        m.pswap = parity;
        if (launched != hipSuccess || ended != hipSuccess) {
            if (g) (void)hipGraphDestroy(g);
            SHELL_HIP(launched != hipSuccess ? launched : ended);
        }
        const hipError_t err = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        SHELL_HIP(err);
        if (m.graphs.size() >= kMsMaxGraphs) {
            (void)hipGraphExecDestroy(m.graphs.front().ex);
            m.graphs.erase(m.graphs.begin());
        }
        m.graphs.push_back({mass, dt2, count, parity, ex});
    }
    SHELL_HIP(hipGraphLaunch(ex, s));
    m.pswap = (count & 1) ? !parity : parity;
}

namespace {

// The host side of one simulation's step as a resumable task.  It suspends wherever it needs a value its
// stream has yet to produce, leaving the event that marks the value ready, so that one host thread can
// keep the steps of several simulations in flight on their own streams.
struct StepTask {
    struct promise_type;
    using Handle = std::coroutine_handle<promise_type>;
    struct promise_type {
        shell_status_t rc = SHELL_OK;
        hipEvent_t wait = nullptr;
        std::exception_ptr err;
        StepTask get_return_object() { return StepTask(Handle::from_promise(*this)); }
        std::suspend_always initial_suspend() noexcept { return {}; }
        std::suspend_always final_suspend() noexcept { return {}; }
        void return_value(shell_status_t r) { rc = r; }
        void unhandled_exception() { err = std::current_exception(); }
    };
    Handle h;
    explicit StepTask(Handle x) : h(x) {}
    StepTask(StepTask&& o) noexcept : h(std::exchange(o.h, {})) {}
    StepTask(const StepTask&) = delete;
    StepTask& operator=(const StepTask&) = delete;
    ~StepTask() {
        if (h) h.destroy();
    }
    // runs to the next suspension (rethrowing what the step threw); true once the step has returned
    bool advance() {
        h.resume();
        if (h.promise().err) std::rethrow_exception(h.promise().err);
        return h.done();
    }
    hipEvent_t waiting_on() const { return h.promise().wait; }
    shell_status_t result() const { return h.promise().rc; }
};

// co_await DeviceReady{e}: suspend until the stream has reached event e
struct DeviceReady {
    hipEvent_t ev;
    bool await_ready() const noexcept { return false; }
    void await_suspend(StepTask::Handle h) const noexcept { h.promise().wait = ev; }
    void await_resume() const noexcept {}
};

void ensure_host_side(MembraneSolve& m) {
    if (m.hscal && m.ready) return;
    RuntimeLock lk(runtime_mutex());
    if (!m.hscal) SHELL_HIP(hipHostMalloc(reinterpret_cast<void**>(&m.hscal), 2 * S_COUNT * sizeof(double)));
    if (!m.ready) SHELL_HIP(hipEventCreateWithFlags(&m.ready, hipEventDisableTiming));
}

// One implicit step with the membrane (Sec. 5, eq 62 with the membrane energy of Sec. 3): Newton on the
// incremental potential, each Newton iteration one PCG over all coordinates against the tangent, then
// Armijo backtracking; the same kernels in the same order whichever way the task is driven.
StepTask membrane_step_task(shell_sim_s& sim, shell_step_params_t p, shell_step_stats_t& out, hipStream_t s) {
    shell_stencils_s& st = *sim.st;
    MembraneSolve& m = *sim.ms;
    const bool graphs = (p.flags & SHELL_STEP_NO_GRAPHS) == 0;
    const long nv = sim.nv, n3 = 3 * nv, ng = m.ngroups;
    const double dt = p.dt, dt2 = dt * dt;
    double* part = m.part.p;
    double* eb = m.part.p + 2 * ng;
    out = shell_step_stats_t{};
    ensure_host_side(m);
    const double* hs = m.hscal;
    // the PCG state set the last iterations left (set 0 right after ms_fin_init)
    auto pcg = [&]() { return hs + (m.pswap ? S_COUNT : 0); };
    // the device scalars into the pinned copy; awaiting the result suspends the step until it has landed
    auto fetch = [&]() {
        SHELL_HIP(hipMemcpyAsync(m.hscal, m.scal.p, 2 * S_COUNT * sizeof(double), hipMemcpyDeviceToHost, s));
        SHELL_HIP(hipEventRecord(m.ready, s));
        return DeviceReady{m.ready};
    };
    // energy and force at xtry (force into ftry); the energy lands in hs[S_E] with the next fetch
    auto evaluate = [&]() {
        forces_at_try(sim, s);
        ms_inertia<<<ms_grid(nv), kMsBlk, 0, s>>>(m.xtry.p, sim.xhat.p, sim.mass.p, nv, part, ng);
        ms_energy<<<1, kMsBlk, 0, s>>>(eb, st.nblocks, m.mepart.p, st.nblocks, st.bias_e0, part, ng, dt2,
                                       m.scal.p);
        SHELL_HIP(hipGetLastError());
    };
    ms_predictor<<<ms_grid(nv), kMsBlk, 0, s>>>(sim.x.p, sim.v.p, sim.xt.p, sim.xhat.p, sim.pinned.p, nv, dt,
                                                 p.gravity[0], p.gravity[1], p.gravity[2]);
    SHELL_HIP(hipMemcpyAsync(m.xtry.p, sim.x.p, size_t(n3) * sizeof(double), hipMemcpyDeviceToDevice, s));
    evaluate();
    co_await fetch();
    double E = hs[S_E];
    SHELL_HIP(hipMemcpyAsync(sim.f.p, m.ftry.p, size_t(n3) * sizeof(double), hipMemcpyDeviceToDevice, s));
    const bool replay = p.mode == SHELL_PCG_REPLAY;
    double gn0 = 0.0, gn = 0.0;
    bool budget = false, nonfinite = false;
    for (int k = 0;; ++k) {
        ms_grad<<<ms_grid(nv), kMsBlk, 0, s>>>(sim.x.p, sim.xhat.p, sim.mass.p, sim.f.p, sim.pinned.p, nv, dt2,
                                               sim.g.p, part, ng);
        ms_fin1<<<1, kMsBlk, 0, s>>>(part, ng, m.scal.p, S_GSQ);
        co_await fetch();
        if (!std::isfinite(hs[S_GSQ])) {
            nonfinite = true;
            break;
        }
        gn = std::sqrt(hs[S_GSQ]);
        if (k == 0) gn0 = gn;
        if (gn0 == 0.0 || (k > 0 && gn <= p.newton_rtol * gn0)) break;
        if (k == p.max_newton) {
            out.newton_capped = 1;
            break;
        }
        // the membrane tangent and the Jacobi preconditioner
        tangent_at(sim, sim.x.p, sim.mass.p, dt2, s);
        // one PCG over all coordinates
        const int target = replay ? p.replay_counts[3 * k] : p.max_pcg;
        m.pswap = false;  // ms_pcg_init writes p = z into m.p, the first product's old direction
        ms_pcg_init<<<ms_grid(nv), kMsBlk, 0, s>>>(sim.g.p, m.dinv.p, m.r.p, m.z.p, m.p.p, m.y.p, nv, part, ng);
        ms_fin_init<<<1, kMsBlk, 0, s>>>(part, ng, m.scal.p, p.pcg_rtol * p.pcg_rtol, target, replay ? 1 : 0);
        SHELL_HIP(hipGetLastError());
        co_await fetch();
        int chunk = 16;
        while (pcg()[S_ACTIVE] != 0.0) {
            pcg_iterations(m, sim.mass.p, sim.pinned.p, nv, dt2, chunk, graphs, s);
            SHELL_HIP(hipGetLastError());
            co_await fetch();
            chunk = std::min(2 * chunk, 256);
        }
        if (pcg()[S_BUDGET] == 2.0) {
            nonfinite = true;
            break;
        }
        budget |= pcg()[S_BUDGET] != 0.0;
        const int its = int(pcg()[S_IT]);
        // Armijo backtracking on the incremental potential
        ms_dot<<<unsigned(ng), kMsBlk, 0, s>>>(sim.g.p, m.y.p, n3, part, ng);  // grid-stride: one partial per group
        ms_fin1<<<1, kMsBlk, 0, s>>>(part, ng, m.scal.p, S_SLOPE);
        co_await fetch();
        const double slope = hs[S_SLOPE];
        int halv = 0;
        double a = 1.0, Etry = 0.0;
        for (;;) {
            ms_axpy<<<ms_grid(n3), kMsBlk, 0, s>>>(sim.x.p, m.y.p, a, m.xtry.p, n3);
            evaluate();
            co_await fetch();
            Etry = hs[S_E];
            const bool done = replay ? halv >= p.replay_counts[3 * k + 1] : (Etry <= E + 1e-4 * a * slope || halv == 6);
            if (done) break;
            a *= 0.5;
            ++halv;
        }
        SHELL_HIP(hipMemcpyAsync(sim.x.p, m.xtry.p, size_t(n3) * sizeof(double), hipMemcpyDeviceToDevice, s));
        SHELL_HIP(hipMemcpyAsync(sim.f.p, m.ftry.p, size_t(n3) * sizeof(double), hipMemcpyDeviceToDevice, s));
        E = Etry;
        out.counts[k][0] = its;
        out.counts[k][1] = halv;
        out.pcg_total += its;
        out.newton_iters++;
    }
    ms_velocity<<<ms_grid(n3), kMsBlk, 0, s>>>(sim.x.p, sim.xt.p, sim.v.p, n3, dt);
    SHELL_HIP(hipGetLastError());
    SHELL_HIP(hipEventRecord(m.ready, s));
    co_await DeviceReady{m.ready};
    out.grad_norm0 = gn0;
    out.grad_norm = gn;
    out.status = nonfinite ? SHELL_E_NONFINITE : (budget ? SHELL_E_BUDGET : SHELL_OK);
    sim.stats = out;
    sim.step++;
    sim.last_stream = s;
    co_return shell_status_t(out.status);
}

// Lanes of a membrane batch that are left with work when a member's step throws are drained before the
// error propagates, so that no step is still running when the caller reads or frees the members.
struct LaneDrain {
    const std::vector<hipStream_t>& lanes;
    bool armed = true;
    ~LaneDrain() {
        if (armed)
            for (hipStream_t l : lanes) (void)hipStreamSynchronize(l);
    }
};

}  // namespace

shell_status_t membrane_step(shell_sim_s& sim, const shell_step_params_t& p, shell_step_stats_t& out,
                             hipStream_t s) {
    StepTask t = membrane_step_task(sim, p, out, s);
    while (!t.advance()) SHELL_HIP(hipStreamSynchronize(s));
    return t.result();
}

// A batch of simulations with the membrane.  Every member takes the step it would take alone: the same
// kernels, in the same order, on its own state, so the same result bit for bit.  The members run on
// streams of their own, after the work already on s; one host thread keeps their steps in flight
// together, resuming each whenever the value it waits for has landed (the GPU overlaps one member's
// kernels with another's and with the host's waits and launches).  Every member's work has finished
// when the call returns.
shell_status_t membrane_batch_step(shell_batch_s& b, const shell_step_params_t* p, int nparams,
                                   shell_step_stats_t* stats, hipStream_t s) {
    const size_t n = b.sims.size();
    std::vector<shell_step_stats_t> out(n);
    shell_status_t worst = SHELL_OK;
    auto merge = [&](shell_status_t rc) {
        if (rc == SHELL_E_NONFINITE || (rc == SHELL_E_BUDGET && worst == SHELL_OK)) worst = rc;
    };
    if (n == 1) {
        merge(membrane_step(*b.sims[0], p[0], out[0], s));
    } else if (n > 1) {
        std::vector<hipStream_t> lanes(n);
        hipEvent_t start = nullptr;
        {
            RuntimeLock lk(runtime_mutex());
            for (size_t i = 0; i < n; ++i) {
                MembraneSolve& m = *b.sims[i]->ms;
                if (!m.lane) SHELL_HIP(hipStreamCreateWithFlags(&m.lane, hipStreamNonBlocking));
                lanes[i] = m.lane;
            }
            SHELL_HIP(hipEventCreateWithFlags(&start, hipEventDisableTiming));
        }
        struct EventGuard {
            hipEvent_t e;
            ~EventGuard() { (void)hipEventDestroy(e); }
        } start_guard{start};
        SHELL_HIP(hipEventRecord(start, s));
        for (hipStream_t l : lanes) SHELL_HIP(hipStreamWaitEvent(l, start, 0));
        LaneDrain drain{lanes};
        std::vector<StepTask> tasks;
        tasks.reserve(n);
        for (size_t i = 0; i < n; ++i)
            tasks.push_back(membrane_step_task(*b.sims[i], p[nparams == 1 ? 0 : i], out[i], lanes[i]));
        std::vector<char> done(n, 0);
        size_t left = n;
        while (left > 0) {
            bool moved = false;
            for (size_t i = 0; i < n; ++i) {
                if (done[i]) continue;
                if (hipEvent_t e = tasks[i].waiting_on()) {
                    const hipError_t q = hipEventQuery(e);
                    if (q == hipErrorNotReady) continue;
                    SHELL_HIP(q);
                }
                if (tasks[i].advance()) {
                    done[i] = 1;
                    --left;
                    merge(tasks[i].result());
                }
                moved = true;
            }
            // nothing has landed: poll again (blocking on one member would hold back the others whose
            // values land first; polling measured 4-8% faster on 32 simulations)
            if (!moved) std::this_thread::yield();
        }
        drain.armed = false;
    }
    if (stats)
        for (size_t i = 0; i < n; ++i) stats[i] = out[i];
    return worst;
}

shell_status_t membrane_static(shell_sim_s& sim, const shell_step_params_t& p, const MembraneStatic& qs,
                               shell_step_stats_t& out, hipStream_t s) {
    MembraneSolve& m = *sim.ms;
    const bool graphs = (p.flags & SHELL_STEP_NO_GRAPHS) == 0;
    const long nv = sim.nv, n3 = 3 * nv, ng = m.ngroups;
    double* part = m.part.p;
    out = shell_step_stats_t{};
    if (!sim.zmass.p) {
        sim.zmass.alloc(size_t(nv));
        ms_zero<<<ms_grid(nv), kMsBlk, 0, s>>>(sim.zmass.p, nv);
    }
    double hs[2 * S_COUNT];
    auto read_scal = [&]() {
        SHELL_HIP(hipMemcpyAsync(hs, m.scal.p, sizeof(hs), hipMemcpyDeviceToHost, s));
        SHELL_HIP(hipStreamSynchronize(s));
    };
    // the PCG state set the last iterations left (set 0 right after ms_fin_init)
    auto pcg = [&]() { return hs + (m.pswap ? S_COUNT : 0); };
    // bending plus membrane force at xtry into ftry, then the load added: ftry = f + F
    auto forces_and_load = [&]() {
        forces_at_try(sim, s);
        if (qs.load) ms_axpy<<<ms_grid(n3), kMsBlk, 0, s>>>(m.ftry.p, qs.load, 1.0, m.ftry.p, n3);
        SHELL_HIP(hipGetLastError());
    };
    SHELL_HIP(hipMemcpyAsync(m.xtry.p, sim.x.p, size_t(n3) * sizeof(double), hipMemcpyDeviceToDevice, s));
    forces_and_load();
    const bool replay = p.mode == SHELL_PCG_REPLAY;
    double gn0 = 0.0, gn = 0.0;
    bool budget = false, nonfinite = false;
    for (int k = 0;; ++k) {
        // r = -(f + F) on the free rows: the step's gradient with no mass (x_hat unused)
        ms_grad<<<ms_grid(nv), kMsBlk, 0, s>>>(sim.x.p, sim.x.p, sim.zmass.p, m.ftry.p, sim.pinned.p, nv, 1.0,
                                               sim.g.p, part, ng);
        ms_fin1<<<1, kMsBlk, 0, s>>>(part, ng, m.scal.p, S_GSQ);
        read_scal();
        if (!std::isfinite(hs[S_GSQ])) {
            nonfinite = true;
            break;
        }
        gn = std::sqrt(hs[S_GSQ]);
        if (k == 0) gn0 = gn;
        if (gn == 0.0 || gn < qs.eps_f) break;
        if (k == p.max_newton) {
            out.newton_capped = 1;
            break;
        }
        tangent_at(sim, sim.x.p, sim.zmass.p, 1.0, s);
        const int target = replay ? p.replay_counts[3 * k] : p.max_pcg;
        m.pswap = false;  // ms_pcg_init writes p = z into m.p, the first product's old direction
        ms_pcg_init<<<ms_grid(nv), kMsBlk, 0, s>>>(sim.g.p, m.dinv.p, m.r.p, m.z.p, m.p.p, m.y.p, nv, part, ng);
        ms_fin_init<<<1, kMsBlk, 0, s>>>(part, ng, m.scal.p, p.pcg_rtol * p.pcg_rtol, target, replay ? 1 : 0);
        SHELL_HIP(hipGetLastError());
        read_scal();
        int chunk = 16;
        while (pcg()[S_ACTIVE] != 0.0) {
            pcg_iterations(m, sim.zmass.p, sim.pinned.p, nv, 1.0, chunk, graphs, s);
            SHELL_HIP(hipGetLastError());
            read_scal();
            chunk = std::min(2 * chunk, 256);
        }
        if (pcg()[S_BUDGET] == 2.0) {
            nonfinite = true;
            break;
        }
        budget |= pcg()[S_BUDGET] != 0.0;
        const int its = int(pcg()[S_IT]);
        // incremental displacement limit
        double scale = 1.0;
        if (qs.eps_u > 0.0) {
            ms_absmax<<<unsigned(ng), kMsBlk, 0, s>>>(m.y.p, n3, part, ng);
            ms_fin_max<<<1, kMsBlk, 0, s>>>(part, ng, m.scal.p);
            read_scal();
            if (hs[S_YMAX] > qs.eps_u) scale = qs.eps_u / hs[S_YMAX];
        }
        ms_axpy<<<ms_grid(n3), kMsBlk, 0, s>>>(sim.x.p, m.y.p, scale, m.xtry.p, n3);
        forces_and_load();
        SHELL_HIP(hipMemcpyAsync(sim.x.p, m.xtry.p, size_t(n3) * sizeof(double), hipMemcpyDeviceToDevice, s));
        out.counts[k][0] = its;
        out.pcg_total += its;
        out.newton_iters++;
    }
    SHELL_HIP(hipStreamSynchronize(s));
    out.grad_norm0 = gn0;
    out.grad_norm = gn;
    out.status = nonfinite ? SHELL_E_NONFINITE : (budget ? SHELL_E_BUDGET : SHELL_OK);
    sim.stats = out;
    sim.last_stream = s;
    return shell_status_t(out.status);
}

// Timing harness of the step with the membrane: the force evaluation (bending and membrane tiles), the
// coupled product and the update, each launched `reps` times back to back with HIP events on `s`, on the
// tangent at the current positions and a recurrence started from the force there (every kernel active).
// The positions and velocities are not changed; the solver's work vectors are.
void membrane_time_kernels(shell_sim_s& sim, double dt, int reps, shell_kernel_times_t& out, hipStream_t s) {
    MembraneSolve& m = *sim.ms;
    const long nv = sim.nv, n3 = 3 * nv, ng = m.ngroups;
    const double dt2 = dt * dt;
    hipEvent_t e0, e1;
    SHELL_HIP(hipEventCreate(&e0));
    SHELL_HIP(hipEventCreate(&e1));
    auto elapsed = [&]() {
        SHELL_HIP(hipEventSynchronize(e1));
        float ms = 0.0f;
        SHELL_HIP(hipEventElapsedTime(&ms, e0, e1));
        return double(ms) / reps;
    };
    SHELL_HIP(hipMemcpyAsync(m.xtry.p, sim.x.p, size_t(n3) * sizeof(double), hipMemcpyDeviceToDevice, s));
    SHELL_HIP(hipEventRecord(e0, s));
    for (int k = 0; k < reps; ++k) forces_at_try(sim, s);
    SHELL_HIP(hipEventRecord(e1, s));
    out.force_ms = elapsed();
    tangent_at(sim, sim.x.p, sim.mass.p, dt2, s);
    ms_pcg_init<<<ms_grid(nv), kMsBlk, 0, s>>>(m.ftry.p, m.dinv.p, m.r.p, m.z.p, m.p.p, m.y.p, nv, m.part.p, ng);
    ms_fin_init<<<1, kMsBlk, 0, s>>>(m.part.p, ng, m.scal.p, 0.0, 1 << 30, 1);
    const unsigned ug = ms_update_grid(nv);
    double* set0 = m.scal.p;
    double* set1 = m.scal.p + S_COUNT;
    // one iteration first (state set 0 -> 1, then the update's partials), so that the timed products read
    // an unsettled running state (set 1) and finish it from those partials, as inside a solve
    long np = launch_product(m, sim.mass.p, sim.pinned.p, nv, dt2, m.p.p, m.p2.p, set0, set1, s);
    auto update = [&]() {
        if (np <= kMsFuseAlphaMax) {
            ms_iter_update<true><<<ug, kMsBlk, 0, s>>>(set0, m.p2.p, m.q.p, m.dinv.p, m.y.p, m.r.p, m.z.p, nv,
                                                       m.part.p, long(ug), m.ppart.p, np);
        } else {
            ms_iter_alpha<<<1, kMsBlk, 0, s>>>(m.ppart.p, np, set0);
            ms_iter_update<false><<<ug, kMsBlk, 0, s>>>(set0, m.p2.p, m.q.p, m.dinv.p, m.y.p, m.r.p, m.z.p, nv,
                                                        m.part.p, long(ug), m.ppart.p, np);
        }
    };
    ms_iter_update<true><<<ug, kMsBlk, 0, s>>>(set1, m.p2.p, m.q.p, m.dinv.p, m.y.p, m.r.p, m.z.p, nv, m.part.p,
                                               long(ug), m.ppart.p, np);
    // as in a solve: with many update partials the state is settled before each product
    if (ug > kMsFuseFinishMax) ms_iter_settle<<<1, kMsBlk, 0, s>>>(m.part.p, long(ug), m.scal.p, 1);
    SHELL_HIP(hipEventRecord(e0, s));
    for (int k = 0; k < reps; ++k) np = launch_product(m, sim.mass.p, sim.pinned.p, nv, dt2, m.p.p, m.p2.p, set1, set0, s);
    SHELL_HIP(hipEventRecord(e1, s));
    out.spmv_ms = elapsed();
    if (np > kMsFuseAlphaMax) ms_iter_alpha<<<1, kMsBlk, 0, s>>>(m.ppart.p, np, set0);
    SHELL_HIP(hipEventRecord(e0, s));
    for (int k = 0; k < reps; ++k) update();
    SHELL_HIP(hipEventRecord(e1, s));
    out.update_ms = elapsed();
    SHELL_HIP(hipGetLastError());
    out.reps = reps;
    SHELL_HIP(hipEventDestroy(e0));
    SHELL_HIP(hipEventDestroy(e1));
    m.pswap = false;
}

}  // namespace shell
