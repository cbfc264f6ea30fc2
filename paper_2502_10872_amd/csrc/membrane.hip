// Membrane (Sec. 3, eq 1) on constant strain triangles with the Saint Venant-Kirchhoff model, float64.
//
// Rest data per triangle (membrane_rest): the rest frame e1 along X1 - X0, e2 = n x e1; Dm the 2x2 matrix
// of the rest edge vectors in that frame; G = Dm^-1 and the area A.  Force (membrane_forces): with Ds the
// current edge vectors x1 - x0, x2 - x0, F = Ds G (3x2), Green strain E = (F^T F - I)/2 in Voigt form
// [E11, E22, 2 E12], stress sigma = D_m eps with D_m = h E_el (plane stress), energy A/2 eps . sigma;
// dPsi/dDs = A F S G^T (S the stress as a 2x2 tensor), so f1 and f2 are minus its columns and f0 their
// sum.  One thread per triangle; the three vertex forces are added atomically into the force array the
// bending kernel wrote (float64, or float in mixed precision, where the edge vectors are formed in float64
// from the rest edges plus the displacement differences).
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

template <typename R>
__global__ void membrane_forces(const double* __restrict__ pos, const double* __restrict__ u4,
                                const double* __restrict__ X, const int32_t* __restrict__ tris,
                                const double* __restrict__ rest, long nt, double c, double nu, R* __restrict__ f,
                                double* __restrict__ epart) {
    long t = blockIdx.x * long(blockDim.x) + threadIdx.x;
    double en[1] = {0.0};
    if (t < nt) {
        const long v0 = tris[3 * t], v1 = tris[3 * t + 1], v2 = tris[3 * t + 2];
        double d1[3], d2[3];
        for (int i = 0; i < 3; ++i) {
            if (pos) {
                d1[i] = pos[3 * v1 + i] - pos[3 * v0 + i];
                d2[i] = pos[3 * v2 + i] - pos[3 * v0 + i];
            } else {
                d1[i] = (X[3 * v1 + i] - X[3 * v0 + i]) + (u4[4 * v1 + i] - u4[4 * v0 + i]);
                d2[i] = (X[3 * v2 + i] - X[3 * v0 + i]) + (u4[4 * v2 + i] - u4[4 * v0 + i]);
            }
        }
        const double G[2][2] = {{rest[5 * t], rest[5 * t + 1]}, {rest[5 * t + 2], rest[5 * t + 3]}};
        const double A = rest[5 * t + 4];
        double F[3][2];
        for (int i = 0; i < 3; ++i)
            for (int b = 0; b < 2; ++b) F[i][b] = d1[i] * G[0][b] + d2[i] * G[1][b];
        double C00 = F[0][0] * F[0][0] + F[1][0] * F[1][0] + F[2][0] * F[2][0];
        double C11 = F[0][1] * F[0][1] + F[1][1] * F[1][1] + F[2][1] * F[2][1];
        double C01 = F[0][0] * F[0][1] + F[1][0] * F[1][1] + F[2][0] * F[2][1];
        const double e0 = 0.5 * (C00 - 1.0), e1 = 0.5 * (C11 - 1.0), e2 = C01;
        const double s0 = c * (e0 + nu * e1), s1 = c * (nu * e0 + e1), s2 = c * 0.5 * (1.0 - nu) * e2;
        en[0] = 0.5 * A * (e0 * s0 + e1 * s1 + e2 * s2);
        for (int i = 0; i < 3; ++i) {
            const double P0 = A * (F[i][0] * s0 + F[i][1] * s2), P1 = A * (F[i][0] * s2 + F[i][1] * s1);
            const double h0 = P0 * G[0][0] + P1 * G[0][1], h1 = P0 * G[1][0] + P1 * G[1][1];
            atomicAdd(f + 3 * v1 + i, R(-h0));
            atomicAdd(f + 3 * v2 + i, R(-h1));
            atomicAdd(f + 3 * v0 + i, R(h0 + h1));
        }
    }
    __shared__ double sh[256 / 64];
    block_sum<1>(en, sh);
    if (threadIdx.x == 0 && epart) epart[blockIdx.x] = en[0];
}

}  // namespace

void launch_membrane_rest(shell_stencils_s& st, hipStream_t s) {
    const long nt = st.nt;
    st.memb.alloc(size_t(5 * nt));
    DevArray<int32_t> bad(1);
    SHELL_HIP(hipMemsetAsync(bad.p, 0, sizeof(int32_t), s));
    if (nt > 0) membrane_rest<<<int((nt + 255) / 256), 256, 0, s>>>(st.X.p, st.tris.p, nt, st.memb.p, bad.p);
    SHELL_HIP(hipGetLastError());
    int32_t h = 0;
    bad.download(&h, 1, s);
    SHELL_HIP(hipStreamSynchronize(s));
    SHELL_CHECK(h == 0, SHELL_E_DEGENERATE, "degenerate triangle (zero area) for the membrane");
    st.mepart.alloc(size_t((nt + 255) / 256));
}

void launch_membrane_forces(shell_stencils_s& st, const double* pos, const double* u4, void* f, hipStream_t s) {
    const long nt = st.nt;
    if (nt == 0) return;
    const double c = st.young * st.thickness / (1.0 - st.poisson * st.poisson);
    const int grid = int((nt + 255) / 256);
    if (st.precision == SHELL_PREC_MIXED)
        membrane_forces<float><<<grid, 256, 0, s>>>(pos, u4, st.X.p, st.tris.p, st.memb.p, nt, c, st.poisson,
                                                    static_cast<float*>(f), st.mepart.p);
    else
        membrane_forces<double><<<grid, 256, 0, s>>>(pos, u4, st.X.p, st.tris.p, st.memb.p, nt, c, st.poisson,
                                                     static_cast<double*>(f), st.mepart.p);
    SHELL_HIP(hipGetLastError());
}

}  // namespace shell
