// Membrane (Sec. 3, eq 1) on constant strain triangles with the Saint Venant-Kirchhoff model, float64.
//
// Rest data per triangle (membrane_rest): the rest frame e1 along X1 - X0, e2 = n x e1; Dm the 2x2 matrix
// of the rest edge vectors in that frame; G = Dm^-1 and the area A.  Force (membrane_tiles): with Ds the
// current edge vectors x1 - x0, x2 - x0, F = Ds G (3x2), Green strain E = (F^T F - I)/2 in Voigt form
// [E11, E22, 2 E12], stress sigma = D_m eps with D_m = h E_el (plane stress), energy A/2 eps . sigma;
// dPsi/dDs = A F S G^T (S the stress as a 2x2 tensor), so f1 and f2 are minus its columns and f0 their
// sum.  The triangles are grouped by the same vertex tiles as the bending stencils (halo triangles
// repeat): each work-group accumulates the forces of its own vertices in LDS and adds them to the force
// the bending kernel stored, one read and one write per vertex and no global atomics.  In mixed precision
// the edge vectors are the rest edges plus the displacement differences, in float64.
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
                                                               const double* __restrict__ u4,
                                                               const double* __restrict__ X,
                                                               const int32_t* __restrict__ tid,
                                                               const double* __restrict__ trest,
                                                               const int64_t* __restrict__ boff, long nv, int T,
                                                               double c, double nu, R* __restrict__ f,
                                                               double* __restrict__ epart) {
    extern __shared__ unsigned char smem_raw[];
    double* acc = reinterpret_cast<double*>(smem_raw);
    const long blk = blockIdx.x;
    const long base = blk * long(T);
    const int nown = int(min(long(T), nv - base));
    for (int i = threadIdx.x; i < 3 * nown; i += blockDim.x) acc[i] = 0.0;
    __syncthreads();
    double en[1] = {0.0};
    const long e0 = boff[2 * blk], e1 = boff[2 * blk + 1];
    for (long e = e0 + threadIdx.x; e < e1; e += blockDim.x) {
        const long v[3] = {tid[4 * e], tid[4 * e + 1], tid[4 * e + 2]};
        double d1[3], d2[3];
        for (int i = 0; i < 3; ++i) {
            if (pos) {
                d1[i] = pos[3 * v[1] + i] - pos[3 * v[0] + i];
                d2[i] = pos[3 * v[2] + i] - pos[3 * v[0] + i];
            } else {
                d1[i] = (X[3 * v[1] + i] - X[3 * v[0] + i]) + (u4[4 * v[1] + i] - u4[4 * v[0] + i]);
                d2[i] = (X[3 * v[2] + i] - X[3 * v[0] + i]) + (u4[4 * v[2] + i] - u4[4 * v[0] + i]);
            }
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
            if (o1 < unsigned(nown)) atomicAdd(acc + 3 * o1 + i, -h0);
            if (o2 < unsigned(nown)) atomicAdd(acc + 3 * o2 + i, -h1);
            if (o0 < unsigned(nown)) atomicAdd(acc + 3 * o0 + i, h0 + h1);
        }
    }
    __syncthreads();
    R* out = f + 3 * base;
    for (int i = threadIdx.x; i < 3 * nown; i += blockDim.x) out[i] = R(double(out[i]) + acc[i]);
    __shared__ double sh[kMembThreads / 64];
    block_sum<1>(en, sh);
    if (threadIdx.x == 0) epart[blk] = en[0];
}

}  // namespace

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

void launch_membrane_forces(shell_stencils_s& st, const double* pos, const double* u4, void* f, hipStream_t s) {
    if (st.nv == 0 || st.nblocks == 0) return;
    const double c = st.young * st.thickness / (1.0 - st.poisson * st.poisson);
    const size_t lds = size_t(3 * st.T) * sizeof(double);
    const unsigned grid = unsigned(st.nblocks);
    if (st.precision == SHELL_PREC_MIXED)
        membrane_tiles<float><<<grid, kMembThreads, lds, s>>>(pos, u4, st.X.p, st.mtid.p, st.mtrest.p, st.mboff.p,
                                                              st.nv, st.T, c, st.poisson, static_cast<float*>(f),
                                                              st.mepart.p);
    else
        membrane_tiles<double><<<grid, kMembThreads, lds, s>>>(pos, u4, st.X.p, st.mtid.p, st.mtrest.p, st.mboff.p,
                                                               st.nv, st.T, c, st.poisson, static_cast<double*>(f),
                                                               st.mepart.p);
    SHELL_HIP(hipGetLastError());
}

}  // namespace shell
