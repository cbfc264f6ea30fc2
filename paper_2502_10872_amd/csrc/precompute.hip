// Rest precomputation, one thread per stencil, float64 (done once per mesh).
//
// Edge hinge (Sec. 4.3): rest normal on the bisector of the two triangle normals, stencil projected
// onto its tangent plane (the corotational stencil), signed feet ratios and heights of vertices 1
// and 4 over the hinge 2->3, L_m = 2 L_theta/(h1 + h4) (eqs 7, 9-10), rest curvature
// kappa0 = L_m N0^T X (eq 14).  Scaled by sqrt(k_b A_E), A_E the two rest triangle areas (eq 16).  A
// clamped boundary edge's stencil (L, M, N, L') takes L' as the reflection of L through the edge's
// midpoint, folds L's column onto L (eqs 30-31) and weighs its one real triangle.
//
// Triangle stencil (Secs 4.4-4.5, App. A/C): rest frame at X1 with x along X12 and z the triangle
// normal (eq 65); the six points in that plane; a missing flap replaced by the reflection of its
// tip through the boundary edge's midpoint; L_p = H L_theta row by row (eqs 76-78); FVM: R from the
// in-plane edge normals (eq 38), B = R L_p; smoothed: C_p = [X^2/2, Y^2/2, XY/2] per point (eq 49),
// B = (L_p C_p)^-1 L_p (eq 50); folds on B's columns, free w_L' = w_M + w_N - w_L (eqs 60-61), clamped
// w_L' = w_L (eq 59); FVM free edge: twist dropped in the edge's frame (clamped edges keep it);
// kappa0 = B N0^T X (eqs 43, 51).  Scaled by sqrt(A).
//
// Plate stencils with a clamped edge measure their curvature vectors from the rest shape, the clamped
// fold not annihilating the flat rest coordinates: the mixed record marks them (the kernel then forms
// C = B (x - X)), and FP64 adds the constant force F0 = -f(X) of those stencils (clamp_bias).
#include "devmath.hpp"
#include "internal.hpp"

namespace shell {

namespace {

constexpr int kFlagDegenerate = 1;

__global__ void precompute_edge(const double* __restrict__ X, const int32_t* __restrict__ idx, long ns,
                                double kb, int shell_model, int world_frame, const int32_t* __restrict__ bcm,
                                double* __restrict__ B, double* __restrict__ k0, int32_t* __restrict__ flags) {
    long s = blockIdx.x * long(blockDim.x) + threadIdx.x;
    if (s >= ns) return;
    const bool clamped = (bcm[s] & kBcEdgeClamped) != 0;
    V3<double> x1 = load3(X, idx[s]), x2 = load3(X, idx[ns + s]), x3 = load3(X, idx[2 * ns + s]),
               x4 = load3(X, idx[3 * ns + s]);
    if (clamped) x4 = x2 + x3 - x1;  // the virtual node
    V3<double> a = x1 - x2, e = x3 - x2, b = x4 - x2;
    V3<double> ua = cross(e, a);  // (x2-x1) x (x3-x1)
    V3<double> ub = cross(b, e);  // (x3-x4) x (x2-x4)
    double la = norm(ua), lb = norm(ub);
    int flag = 0;
    if (!(la > 0.0) || !(lb > 0.0)) flag = kFlagDegenerate;
    V3<double> m = (1.0 / la) * ua + (1.0 / lb) * ub;
    double lm = norm(m);
    if (!(lm > 1e-12)) flag = kFlagDegenerate;
    V3<double> n0 = (1.0 / lm) * m;
    // projection onto the tangent plane through x2 (eq 7); the world-frame operator of the quadratic thin
    // plate/shell (App. D, eq 79) measures the unprojected stencil
    const double wp = world_frame ? 0.0 : 1.0;
    V3<double> ac = a - (wp * dot(n0, a)) * n0, ec = e - (wp * dot(n0, e)) * n0, bc = b - (wp * dot(n0, b)) * n0;
    double ee = dot(ec, ec);
    double sp = dot(ac, ec) / ee, sq = dot(bc, ec) / ee;
    double h1 = norm(ac - sp * ec), h4 = norm(bc - sq * ec);
    double elen = sqrt(ee);
    if (!(h1 > 1e-12 * elen) || !(h4 > 1e-12 * elen)) flag = kFlagDegenerate;
    double c = 2.0 / (h1 + h4);
    double scale = sqrt(kb * 0.5 * (clamped ? la : la + lb));
    double L1 = scale * c / h1;
    double L2 = -scale * c * ((1.0 - sp) / h1 + (1.0 - sq) / h4);
    double L3 = -scale * c * (sp / h1 + sq / h4);
    double L4 = scale * c / h4;
    if (clamped) {
        L1 += L4;
        L4 = 0.0;
    }
    B[s] = L1;
    B[ns + s] = L2;
    B[2 * ns + s] = L3;
    B[3 * ns + s] = L4;
    // rows sum to zero, so the rest curvature can be taken on differences from x2
    k0[s] = shell_model ? L1 * dot(n0, a) + L3 * dot(n0, e) + L4 * dot(n0, b) : 0.0;
    flags[s] = flag;
}

__device__ inline double inv3x3(const double (&M)[3][3], double (&Mi)[3][3]) {
    double c00 = M[1][1] * M[2][2] - M[1][2] * M[2][1];
    double c01 = M[1][2] * M[2][0] - M[1][0] * M[2][2];
    double c02 = M[1][0] * M[2][1] - M[1][1] * M[2][0];
    double det = M[0][0] * c00 + M[0][1] * c01 + M[0][2] * c02;
    double id = 1.0 / det;
    Mi[0][0] = c00 * id;
    Mi[1][0] = c01 * id;
    Mi[2][0] = c02 * id;
    Mi[0][1] = (M[0][2] * M[2][1] - M[0][1] * M[2][2]) * id;
    Mi[1][1] = (M[0][0] * M[2][2] - M[0][2] * M[2][0]) * id;
    Mi[2][1] = (M[0][1] * M[2][0] - M[0][0] * M[2][1]) * id;
    Mi[0][2] = (M[0][1] * M[1][2] - M[0][2] * M[1][1]) * id;
    Mi[1][2] = (M[0][2] * M[1][0] - M[0][0] * M[1][2]) * id;
    Mi[2][2] = (M[0][0] * M[1][1] - M[0][1] * M[1][0]) * id;
    double n1 = 0.0, n2 = 0.0;  // 1-norm condition number
    for (int j = 0; j < 3; ++j) {
        n1 = fmax(n1, fabs(M[0][j]) + fabs(M[1][j]) + fabs(M[2][j]));
        n2 = fmax(n2, fabs(Mi[0][j]) + fabs(Mi[1][j]) + fabs(Mi[2][j]));
    }
    return (det != 0.0 && isfinite(det)) ? n1 * n2 : INFINITY;
}

__global__ void precompute_tri(const double* __restrict__ X, const int32_t* __restrict__ idx, long ns, int fvm,
                               int shell_model, double* __restrict__ B, double* __restrict__ k0,
                               int32_t* __restrict__ flags, const int32_t* __restrict__ bc) {
    long s = blockIdx.x * long(blockDim.x) + threadIdx.x;
    if (s >= ns) return;
    const int miss = bc[s] & 7;          // bit L set: flap L+3 absent (its idx points at vertex 1)
    const int clamp = (bc[s] >> 3) & 7;  // bit L set: and its edge clamped
    V3<double> x1 = load3(X, idx[s]);
    V3<double> d[6];
    d[0] = mk(0.0, 0.0, 0.0);
    for (int j = 1; j < 6; ++j) d[j] = load3(X, idx[j * ns + s]) - x1;
    V3<double> u = cross(d[1], d[2]);
    double twoA = norm(u);
    int flag = twoA > 0.0 ? 0 : kFlagDegenerate;
    V3<double> ez = (1.0 / twoA) * u;
    V3<double> ex = (1.0 / norm(d[1])) * d[1];
    V3<double> ey = cross(ez, ex);
    double px[6], py[6];
    for (int j = 0; j < 6; ++j) {
        px[j] = dot(d[j], ex);
        py[j] = dot(d[j], ey);
    }
    for (int L = 0; L < 3; ++L) {
        if (miss & (1 << L)) {
            int M = (L + 1) % 3, N = (L + 2) % 3;
            px[L + 3] = px[M] + px[N] - px[L];
            py[L + 3] = py[M] + py[N] - py[L];
        }
    }
    // directional hinge operator across each edge of the central triangle
    double Lp[3][6];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 6; ++j) Lp[i][j] = 0.0;
    for (int i = 0; i < 3; ++i) {
        int a = (i + 1) % 3, b = (i + 2) % 3, f = i + 3;
        double ex2 = px[b] - px[a], ey2 = py[b] - py[a];
        double ee = ex2 * ex2 + ey2 * ey2;
        double tx = px[i] - px[a], ty = py[i] - py[a];
        double fx = px[f] - px[a], fy = py[f] - py[a];
        double st = (tx * ex2 + ty * ey2) / ee, sf = (fx * ex2 + fy * ey2) / ee;
        double ht = hypot(tx - st * ex2, ty - st * ey2), hf = hypot(fx - sf * ex2, fy - sf * ey2);
        double el = sqrt(ee);
        if (!(ht > 1e-12 * el) || !(hf > 1e-12 * el)) flag = kFlagDegenerate;
        double c = 2.0 / (ht + hf);
        Lp[i][i] = c / ht;
        Lp[i][a] = -c * ((1.0 - st) / ht + (1.0 - sf) / hf);
        Lp[i][b] = -c * (st / ht + sf / hf);
        Lp[i][f] = c / hf;
    }
    double Bm[3][6];
    if (fvm) {
        double R[3][3];
        for (int i = 0; i < 3; ++i) {
            int a = (i + 1) % 3, b = (i + 2) % 3;
            double ex2 = px[b] - px[a], ey2 = py[b] - py[a];
            double il = 1.0 / hypot(ex2, ey2);
            double ms = ey2 * il, mt = -ex2 * il;  // in-plane unit normal of edge i
            R[0][i] = ms * ms;
            R[1][i] = mt * mt;
            R[2][i] = 2.0 * ms * mt;
        }
        for (int r = 0; r < 3; ++r)
            for (int j = 0; j < 6; ++j) Bm[r][j] = R[r][0] * Lp[0][j] + R[r][1] * Lp[1][j] + R[r][2] * Lp[2][j];
    } else {
        double M[3][3], Mi[3][3];
        for (int r = 0; r < 3; ++r) {
            double a0 = 0.0, a1 = 0.0, a2 = 0.0;
            for (int j = 0; j < 6; ++j) {
                a0 += Lp[r][j] * (0.5 * px[j] * px[j]);
                a1 += Lp[r][j] * (0.5 * py[j] * py[j]);
                a2 += Lp[r][j] * (0.5 * px[j] * py[j]);
            }
            M[r][0] = a0;
            M[r][1] = a1;
            M[r][2] = a2;
        }
        double cond = inv3x3(M, Mi);
        if (!(cond < 1e12)) flag = kFlagDegenerate;
        for (int r = 0; r < 3; ++r)
            for (int j = 0; j < 6; ++j) Bm[r][j] = Mi[r][0] * Lp[0][j] + Mi[r][1] * Lp[1][j] + Mi[r][2] * Lp[2][j];
    }
    int first_free = -1;
    for (int L = 0; L < 3; ++L) {
        if (!(miss & (1 << L))) continue;
        int M = (L + 1) % 3, N = (L + 2) % 3, F = L + 3;
        const bool cl = (clamp >> L) & 1;
        if (!cl && first_free < 0) first_free = L;
        for (int r = 0; r < 3; ++r) {
            double w = Bm[r][F];
            if (cl) {
                Bm[r][L] += w;
            } else {
                Bm[r][M] += w;
                Bm[r][N] += w;
                Bm[r][L] -= w;
            }
            Bm[r][F] = 0.0;
        }
    }
    if (fvm && first_free >= 0) {
        // keep only the curvature components normal and along the free edge: P = T(-phi) diag(1,1,0) T(phi)
        int M = (first_free + 1) % 3, N = (first_free + 2) % 3;
        double ex2 = px[N] - px[M], ey2 = py[N] - py[M];
        double il = 1.0 / hypot(ex2, ey2);
        double c = ex2 * il, sn = ey2 * il;
        double T0[3] = {c * c, sn * sn, c * sn}, T1[3] = {sn * sn, c * c, -c * sn};   // rows of T(phi)
        double Ic0[3] = {c * c, sn * sn, 2.0 * c * sn}, Ic1[3] = {sn * sn, c * c, -2.0 * c * sn};  // cols of T(-phi)
        double Bn[3][6];
        for (int j = 0; j < 6; ++j) {
            double r0 = T0[0] * Bm[0][j] + T0[1] * Bm[1][j] + T0[2] * Bm[2][j];
            double r1 = T1[0] * Bm[0][j] + T1[1] * Bm[1][j] + T1[2] * Bm[2][j];
            for (int r = 0; r < 3; ++r) Bn[r][j] = Ic0[r] * r0 + Ic1[r] * r1;
        }
        for (int r = 0; r < 3; ++r)
            for (int j = 0; j < 6; ++j) Bm[r][j] = Bn[r][j];
    }
    double sc = sqrt(0.5 * twoA);
    for (int r = 0; r < 3; ++r) {
        double kr = 0.0;
        for (int j = 0; j < 6; ++j) {
            B[(r * 6 + j) * ns + s] = sc * Bm[r][j];
            kr += Bm[r][j] * dot(ez, d[j]);
        }
        k0[r * ns + s] = shell_model ? sc * kr : 0.0;
    }
    flags[s] = flag;
}

__global__ void tile_copy(const int32_t* __restrict__ src, long nt, const int32_t* __restrict__ idx,
                          const double* __restrict__ B, const double* __restrict__ k0, const double* __restrict__ X,
                          const int32_t* __restrict__ bc, long ns, int k, int r, bool shell, int32_t* __restrict__ tidx,
                          double* __restrict__ trec64, float* __restrict__ trec32) {
    long e = blockIdx.x * long(blockDim.x) + threadIdx.x;
    if (e >= nt) return;
    const long s = src[e];  // -1: alignment padding, filled with vertex 0 and zeros (never read)
    const long blk = e / kStreamBlock, lane = e % kStreamBlock;
    if (trec32) {
        // mixed: ids, the operator's entries other than the origin column, rounded to float32, and (shells)
        // the rest curvatures of the rounded operator, kappa0_i = sum_j B~_ij (X_j - X_o) . n0 with the
        // rest normal n0 of the force kernel's construction (float64 sums, stored as float64)
        const int nf = rec32_fields(k, r, shell), nch = stream_chunks(nf, 4);
        float* base = trec32 + (blk * nch * kStreamBlock + lane) * 4;
        auto put = [&](int f, float v) { base[(f / 4) * kStreamBlock * 4 + f % 4] = v; };
        const int o = k == 4 ? 1 : 0;  // origin: the hinge's first end (edge) or the central vertex 0
        const bool clamped_plate = s >= 0 && !shell && (bc[s] & kBcClampedAny) != 0;
        for (int j = 0; j < k; ++j) {
            uint32_t id = s < 0 ? 0u : uint32_t(idx[j * ns + s]);
            if (j == 0 && clamped_plate) id |= kRecClampBit;
            put(j, __uint_as_float(id));
        }
        int f = k;
        for (int i = 0; i < r; ++i)
            for (int j = 0; j < k; ++j)
                if (j != o) put(f++, s < 0 ? 0.0f : float(B[(i * k + j) * ns + s]));
        if (shell) {
            double h0[6] = {0, 0, 0, 0, 0, 0};
            if (s >= 0) {
                V3<double> P[6];
                for (int j = 0; j < k; ++j) P[j] = load3(X, idx[j * ns + s]) - load3(X, idx[o * ns + s]);
                V3<double> n0;
                if (k == 4) {
                    // bisector of the two hinge triangles' unit normals (hinge 1 -> 2, tips 0 and 3)
                    const V3<double> ua = cross(P[2], P[0]), ub = cross(P[3], P[2]);
                    const V3<double> m = (1.0 / norm(ua)) * ua + (1.0 / norm(ub)) * ub;
                    n0 = (1.0 / norm(m)) * m;
                } else {
                    const V3<double> u = cross(P[1], P[2]);
                    n0 = (1.0 / norm(u)) * u;
                }
                for (int j = 0; j < k; ++j) h0[j] = dot(P[j], n0);
            }
            for (int i = 0; i < r; ++i) {
                double kr = 0.0;
                for (int j = 0; j < k; ++j)
                    if (j != o && s >= 0) kr += double(float(B[(i * k + j) * ns + s])) * h0[j];
                const unsigned long long bits = __double_as_longlong(kr);
                put(f++, __uint_as_float(uint32_t(bits & 0xffffffffull)));
                put(f++, __uint_as_float(uint32_t(bits >> 32)));
            }
        }
        if (k == 4 && !shell) {
            // edge plate: the tip's coordinates in the rest tangent plane (the plane of the bisector
            // normal, in which the operator annihilates affine fields), x3 - x1 ~ alpha (x0 - x1) +
            // beta (x2 - x1) for every affine motion of the rest stencil
            double ab[2] = {0.0, 0.0};
            if (s >= 0) {
                const V3<double> x1 = load3(X, idx[ns + s]);
                const V3<double> A = load3(X, idx[s]) - x1, Cc = load3(X, idx[2 * ns + s]) - x1;
                const V3<double> Bb = load3(X, idx[3 * ns + s]) - x1;
                const V3<double> ua = cross(Cc, A), ub = cross(Bb, Cc);
                V3<double> n0 = (1.0 / norm(ua)) * ua + (1.0 / norm(ub)) * ub;
                n0 = (1.0 / norm(n0)) * n0;
                const V3<double> Ap = A - dot(A, n0) * n0, Cp = Cc - dot(Cc, n0) * n0, Bp = Bb - dot(Bb, n0) * n0;
                const double g11 = dot(Ap, Ap), g12 = dot(Ap, Cp), g22 = dot(Cp, Cp);
                const double r1 = dot(Ap, Bp), r2 = dot(Cp, Bp), idet = 1.0 / (g11 * g22 - g12 * g12);
                ab[0] = (g22 * r1 - g12 * r2) * idet;
                ab[1] = (g11 * r2 - g12 * r1) * idet;
            }
            for (; f < kRecEdgeAffine; ++f) put(f, 0.0f);
            for (int q = 0; q < 2; ++q) {
                const unsigned long long bits = __double_as_longlong(ab[q]);
                put(f++, __uint_as_float(uint32_t(bits & 0xffffffffull)));
                put(f++, __uint_as_float(uint32_t(bits >> 32)));
            }
        }
        for (; f < 4 * nch; ++f) put(f, 0.0f);
    } else {
        const int nchi = stream_chunks(k, 4), nchv = stream_chunks(rec64_fields(k, r), 2);
        int32_t* bi = tidx + (blk * nchi * kStreamBlock + lane) * 4;
        double* bv = trec64 + (blk * nchv * kStreamBlock + lane) * 2;
        auto put_i = [&](int f, int32_t v) { bi[(f / 4) * kStreamBlock * 4 + f % 4] = v; };
        auto put_v = [&](int f, double v) { bv[(f / 2) * kStreamBlock * 2 + f % 2] = v; };
        for (int j = 0; j < 4 * nchi; ++j) put_i(j, (s < 0 || j >= k) ? 0 : idx[j * ns + s]);
        for (int q = 0; q < r * k; ++q) put_v(q, s < 0 ? 0.0 : B[q * ns + s]);
        for (int q = 0; q < r; ++q) put_v(r * k + q, s < 0 ? 0.0 : k0[q * ns + s]);
        for (int f = rec64_fields(k, r); f < 2 * nchv; ++f) put_v(f, 0.0);
    }
}


// FP64 plates: the clamped stencils' rest curvature vectors C0_i = sum_j B_ij X_j (on differences from
// vertex 1; B's rows sum to zero), their force at the rest shape, f_j = -sum_i B_ij (D C0)_i, and energy
// 1/2 C0 . D C0.  bias = -f summed per vertex (so that f(x) + bias is the force of C = B (x - X)), e0 the
// energy.  D is 1 for the edge operator (k_b A_E is folded into B) and D_b for triangles (A is folded into
// B).  One thread per vertex walks its stencils in ascending order (and per-stencil energies are summed
// in a fixed order), so the result is the same in every run.
__device__ void clamp_stencil(const double* __restrict__ X, const int32_t* __restrict__ idx,
                              const double* __restrict__ B, long ns, long s, int k, int r, double kb, double nu,
                              double (&g)[3][3], double& en) {
    const long o = idx[s];
    double C[3][3];
    for (int i = 0; i < r; ++i) {
        C[i][0] = C[i][1] = C[i][2] = 0.0;
        for (int j = 1; j < k; ++j) {
            const long v = idx[j * ns + s];
            const double b = B[(i * k + j) * ns + s];
            for (int a = 0; a < 3; ++a) C[i][a] += b * (X[3 * v + a] - X[3 * o + a]);
        }
    }
    if (r == 1) {
        for (int a = 0; a < 3; ++a) g[0][a] = C[0][a];
    } else {
        for (int a = 0; a < 3; ++a) {
            g[0][a] = kb * (C[0][a] + nu * C[1][a]);
            g[1][a] = kb * (nu * C[0][a] + C[1][a]);
            g[2][a] = kb * 0.5 * (1.0 - nu) * C[2][a];
        }
    }
    en = 0.0;
    for (int i = 0; i < r; ++i)
        for (int a = 0; a < 3; ++a) en += 0.5 * C[i][a] * g[i][a];
}

__global__ void clamp_bias_rows(const double* __restrict__ X, const int32_t* __restrict__ idx,
                                const double* __restrict__ B, const int32_t* __restrict__ bc,
                                const int64_t* __restrict__ inc_ptr, const int64_t* __restrict__ inc, long ns,
                                long nv, int k, int r, double kb, double nu, double* __restrict__ bias) {
    const long v = blockIdx.x * long(blockDim.x) + threadIdx.x;
    if (v >= nv) return;
    double acc[3] = {0.0, 0.0, 0.0};
    for (int64_t e = inc_ptr[v]; e < inc_ptr[v + 1]; ++e) {
        const long s = long(inc[e] >> 3);
        const int j = int(inc[e] & 7);
        if (!(bc[s] & kBcClampedAny)) continue;
        double g[3][3], en;
        clamp_stencil(X, idx, B, ns, s, k, r, kb, nu, g, en);
        for (int a = 0; a < 3; ++a) {
            double fb = 0.0;
            for (int i = 0; i < r; ++i) fb += B[(i * k + j) * ns + s] * g[i][a];
            acc[a] += fb;
        }
    }
    for (int a = 0; a < 3; ++a) bias[3 * v + a] = acc[a];
}

// e0 = the clamped stencils' rest energy, one work-group, each thread a fixed strided subset, then a
// fixed tree
__global__ void clamp_energy(const double* __restrict__ X, const int32_t* __restrict__ idx,
                             const double* __restrict__ B, const int32_t* __restrict__ bc, long ns, int k, int r,
                             double kb, double nu, double* __restrict__ e0) {
    double acc[1] = {0.0};
    for (long s = threadIdx.x; s < ns; s += blockDim.x) {
        if (!(bc[s] & kBcClampedAny)) continue;
        double g[3][3], en;
        clamp_stencil(X, idx, B, ns, s, k, r, kb, nu, g, en);
        acc[0] += en;
    }
    __shared__ double sh[16];
    block_sum<1>(acc, sh);
    if (threadIdx.x == 0) *e0 = acc[0];
}

}  // namespace

void launch_precompute(shell_stencils_s& st, const int32_t* bc, hipStream_t s) {
    const long ns = st.ns;
    if (ns == 0) return;
    int blk = 256;
    long grid = (ns + blk - 1) / blk;
    if (model_is_edge(st.model)) {
        precompute_edge<<<grid, blk, 0, s>>>(st.X.p, st.idx.p, ns, st.kb, model_is_shell(st.model),
                                             (st.cfg_flags & SHELL_FLAG_WORLD_FRAME) != 0, bc, st.B.p, st.k0.p,
                                             st.flags.p);
    } else {
        precompute_tri<<<grid, blk, 0, s>>>(st.X.p, st.idx.p, ns, model_is_fvm(st.model), model_is_shell(st.model),
                                            st.B.p, st.k0.p, st.flags.p, bc);
    }
    SHELL_HIP(hipGetLastError());
}

void launch_tile_copy(shell_stencils_s& st, const int32_t* bc, hipStream_t s) {
    const long nt = st.nst_pad;
    if (nt == 0) return;
    int blk = 256;
    tile_copy<<<(nt + blk - 1) / blk, blk, 0, s>>>(st.tsrc.p, nt, st.idx.p, st.B.p, st.k0.p, st.X.p, bc, st.ns,
                                                   st.k, st.r, model_is_shell(st.model), st.tidx.p, st.trec64.p,
                                                   st.trec32.p);
    SHELL_HIP(hipGetLastError());
}

void launch_clamp_bias(shell_stencils_s& st, const int32_t* bc, hipStream_t s) {
    const long ns = st.ns;
    st.bias.alloc(size_t(3 * st.nv));
    DevArray<double> e0(1);
    const Incidence inc = build_incidence(st.h_idx, st.k, ns, st.nv);
    DevArray<int64_t> iptr(inc.ptr.size()), icode(std::max<size_t>(inc.code.size(), 1));
    iptr.upload(inc.ptr.data(), inc.ptr.size(), s);
    icode.upload(inc.code.data(), inc.code.size(), s);
    if (st.nv > 0)
        clamp_bias_rows<<<int((st.nv + 255) / 256), 256, 0, s>>>(st.X.p, st.idx.p, st.B.p, bc, iptr.p, icode.p, ns,
                                                                 st.nv, st.k, st.r, st.kb, st.poisson, st.bias.p);
    clamp_energy<<<1, 1024, 0, s>>>(st.X.p, st.idx.p, st.B.p, bc, ns, st.k, st.r, st.kb, st.poisson, e0.p);
    SHELL_HIP(hipGetLastError());
    e0.download(&st.bias_e0, 1, s);
    SHELL_HIP(hipStreamSynchronize(s));
}

}  // namespace shell
