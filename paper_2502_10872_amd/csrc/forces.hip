// Per-stencil bending forces, the per-timestep hot kernel.
//
// Layout: vertices are numbered in tiles of T consecutive ids (compact surface patches).  One
// work-group owns one tile and walks the list of every stencil that touches the tile (stencils on a
// tile boundary appear in each tile they touch).  Each stencil's force on the tile's own vertices is
// added into a float64 LDS accumulator; contributions to other tiles' vertices are left to those
// tiles.  The tile is then written to HBM once: no global atomics, no zero-fill, one coalesced store
// per vertex.  Stencil data is streamed in blocks of 64 stencils, in 16-byte chunks of fields (a
// wave's 64 loads of one chunk are one contiguous 1 KB run, so every load is coalesced and a wave
// touches one region of memory); a tile's list stays in spatial order so the gathers of one wave touch
// few cache lines.  (float32 LDS atomics contended badly on shared vertices; the float64 accumulator
// does not.)
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
// Mixed precision: the kernels gather the float64 displacements u = x - X from the rest shape and
// difference them in float64; everything after the difference is float32.  The curvature is formed
// relative to the rest shape, C = C0 + B (u^e), with C0 = B X^e precomputed in float64, so float32
// rounds the displacement differences (of the size of the deformation) instead of the position
// differences (of the size of an edge): the net force of a smooth deformation is a cancelling sum over
// stencils, and with position differences its relative error grew with the mesh resolution and with
// the inverse of the deformation (2e-3 at 1024x1024 for an amplitude of side/100).  The shell normals
// use the position differences of their vertices, rebuilt as the streamed rest differences plus the
// displacement differences.
#include <hip/hip_ext.h>

#include <algorithm>

#include "devmath.hpp"
#include "internal.hpp"

namespace shell {

namespace {

// Edge stencil (vertices 0-3, hinge 1-2) from the differences a = x0 - x1, c = x2 - x1, b = x3 - x1 and the
// curvature vector C = sum_j L_j x_j formed by the caller.
template <typename R, bool SHELL>
__device__ __forceinline__ void edge_stencil(V3<R> a, V3<R> c, V3<R> b, V3<R> C, const R (&L)[4], R kappa0,
                                             V3<R> (&f)[4], R& energy) {
    if constexpr (!SHELL) {
        energy = R(0.5) * dot(C, C);
#pragma unroll
        for (int j = 0; j < 4; ++j) f[j] = (-L[j]) * C;
    } else {
        V3<R> ua = cross(c, a), ub = cross(b, c);
        R ila = R(1) / norm(ua), ilb = R(1) / norm(ub);
        V3<R> na = ila * ua, nb = ilb * ub;
        V3<R> m = na + nb;
        R ilm = R(1) / norm(m);
        V3<R> n = ilm * m;
        R delta = dot(n, C) - kappa0;
        energy = R(0.5) * delta * delta;
        // w = (I - n n^T) C / |m|, then through each unit triangle normal
        V3<R> w = ilm * (C - dot(C, n) * n);
        V3<R> wa = ila * (w - dot(w, na) * na);
        V3<R> wb = ilb * (w - dot(w, nb) * nb);
        V3<R> g1 = cross(wa, c);
        V3<R> g2 = cross(wa, a - c) + cross(wb, c - b);
        V3<R> g3 = cross(wb, b) - cross(wa, a);
        V3<R> g4 = cross(c, wb);
        f[0] = (-delta) * (L[0] * n + g1);
        f[1] = (-delta) * (L[1] * n + g2);
        f[2] = (-delta) * (L[2] * n + g3);
        f[3] = (-delta) * (L[3] * n + g4);
    }
}

// Triangle stencil from the differences d_j = x_j - x_0 (d_0 = 0) and the curvature vectors
// C_i = sum_j B_ij x_j formed by the caller.
template <typename R, bool SHELL>
__device__ __forceinline__ void tri_stencil(const V3<R> (&d)[6], const V3<R> (&C)[3], const R (&B)[3][6],
                                            const R (&k0)[3], R kb, R nu, V3<R> (&f)[6], R& energy) {
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
        V3<R> u = cross(d[1], d[2]);
        R ilu = R(1) / norm(u);
        V3<R> n = ilu * u;
        R de0 = dot(n, C[0]) - k0[0], de1 = dot(n, C[1]) - k0[1], de2 = dot(n, C[2]) - k0[2];
        R g0 = kb * (de0 + nu * de1), g1 = kb * (nu * de0 + de1), g2 = kb * t * de2;
        energy = R(0.5) * (de0 * g0 + de1 * g1 + de2 * g2);
        V3<R> Cg = g0 * C[0];
        fma3(Cg, g1, C[1]);
        fma3(Cg, g2, C[2]);
        V3<R> w = ilu * (Cg - dot(Cg, n) * n);
#pragma unroll
        for (int j = 0; j < 6; ++j) {
            R bj = g0 * B[0][j] + g1 * B[1][j] + g2 * B[2][j];
            f[j] = (-bj) * n;
        }
        // (du/dx1)^T w = w x (x3 - x2), (du/dx2)^T w = w x (x1 - x3), (du/dx3)^T w = w x (x2 - x1)
        f[0] = f[0] - cross(w, d[2] - d[1]);
        f[1] = f[1] - cross(d[2], w);
        f[2] = f[2] - cross(w, d[1]);
    }
}

// 16-byte stream chunks (clang vector types, which load through address-space pointers in one
// instruction).  The streams are read with non-temporal loads, which keep them from displacing the
// gathered positions or displacements from L2 (measured 2-5% faster than plain loads for the float
// record).
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef int i32x4 __attribute__((ext_vector_type(4)));
typedef double f64x2 __attribute__((ext_vector_type(2)));

// tile accumulator in float64 for both precisions (ds_add_f64)
template <typename R>
__device__ __forceinline__ void lds_add(double* acc, int slot, V3<R> v) {
    atomicAdd(acc + 3 * slot + 0, double(v.x));
    atomicAdd(acc + 3 * slot + 1, double(v.y));
    atomicAdd(acc + 3 * slot + 2, double(v.z));
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
    extern __shared__ unsigned char smem_raw[];
    double* acc = reinterpret_cast<double*>(smem_raw);
    long it = xcd_logical(blockIdx.x, gridDim.x);
    if (it >= nitems) return;
    const WorkItem wi = items[it];
    const ForceDesc& d = descs[wi.mesh];
    // global-address views of the descriptor's pointers: global loads wait on the vector-memory counter
    // only, so the LDS accumulation does not stall behind loads in flight
    const gbl<const double>* x = G(static_cast<const double*>(d.x));
    const R kb = R(d.kb), nu = R(d.nu);
    const long blk = wi.unit;
    const long base = blk * long(d.T);
    const int nown = int(min(long(d.T), d.nv - base));
    for (int i = threadIdx.x; i < 3 * nown; i += blockDim.x) acc[i] = 0.0;
    __syncthreads();
    double e_own = 0.0;
    // a tile's list starts on a 64-stencil block and the work-group's stride is a whole number of
    // blocks, so each wave reads whole blocks: every field of its 64 stencils is one contiguous run
    constexpr int NB = EDGE ? 4 : 18;               // operator entries per stencil
    constexpr int NK = EDGE ? 1 : 3;                // rest-curvature slots per stencil (zero for plates)
    constexpr bool REL = sizeof(R) == 4;            // float: curvature relative to the rest shape
    constexpr int NC = REL ? 3 * NK : 1;            // rest curvature vector components (float only)
    constexpr int ND = REL ? (rec32_rest_diffs(K, SHELL) ? rec32_rest_diffs(K, SHELL) : 1) : 1;
    // 16-byte chunks per stencil: mixed, one record of ids, operator, rest curvatures, C0 and rest
    // differences; FP64, the ids and the float64 values in two streams
    constexpr int NCH32 = stream_chunks(rec32_fields(K, NK, SHELL), 4);
    constexpr int NCHI = stream_chunks(K, 4);
    constexpr int NCHV = stream_chunks(rec64_fields(K, NK), 2);
    struct In {
        int vid[K];
        V3<double> pg[K];  // FP64: positions; mixed: displacements from the rest shape
        R ob[NB + NK];
        R c0[NC];
        R rd[ND];          // mixed shells: rest differences
    };
    auto load = [&](long e, In& in) {
        const long first = (e / kStreamBlock) * kStreamBlock, lane = e % kStreamBlock;
        if constexpr (REL) {
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
#pragma unroll
            for (int j = 0; j < K; ++j) in.vid[j] = __float_as_int(f[j]);
#pragma unroll
            for (int q = 0; q < NB + NK; ++q) in.ob[q] = f[K + q];
#pragma unroll
            for (int q = 0; q < NC; ++q) in.c0[q] = f[K + NB + NK + q];
            if constexpr (SHELL) {
#pragma unroll
                for (int q = 0; q < ND; ++q) in.rd[q] = f[K + NB + NK + NC + q];
            }
            // padded displacements: (x, y) and (z, 0) are two aligned 16-byte loads per vertex
            const gbl<const f64x2>* u2 = G(reinterpret_cast<const f64x2*>(d.x));
#pragma unroll
            for (int j = 0; j < K; ++j) {
                const f64x2 a = u2[2L * in.vid[j]], b = u2[2L * in.vid[j] + 1];
                in.pg[j] = {a.x, a.y, b.x};
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
#pragma unroll
            for (int q = 0; q < NB + NK; ++q) in.ob[q] = R(fv[q]);
#pragma unroll
            for (int j = 0; j < K; ++j)
                in.pg[j] = {x[3L * in.vid[j]], x[3L * in.vid[j] + 1], x[3L * in.vid[j] + 2]};
        }
    };
    // float64 difference of the gathered vectors of vertices j and o, rounded to R (FP64: of positions;
    // mixed: of displacements)
    auto diff = [&](const In& in, int j, int o) { return cvt<R>(in.pg[j] - in.pg[o]); };
    auto rest = [&](const In& in, int q) { return mk(in.rd[3 * q], in.rd[3 * q + 1], in.rd[3 * q + 2]); };
    auto compute = [&](const In& in) {
        V3<R> fs[K];
        R en;
        if constexpr (EDGE) {
            const R L[4] = {in.ob[0], in.ob[1], in.ob[2], in.ob[3]};
            V3<R> a = diff(in, 0, 1), c = diff(in, 2, 1), b = diff(in, 3, 1);
            V3<R> C;
            if constexpr (REL) {
                // a, c, b are displacement differences here: C = C0 + B u^e, then the position
                // differences of the normal are the rest ones plus these
                C = mk(in.c0[0], in.c0[1], in.c0[2]);
                fma3(C, L[0], a);
                fma3(C, L[2], c);
                fma3(C, L[3], b);
                if constexpr (SHELL) {
                    a = rest(in, 0) + a;
                    c = rest(in, 1) + c;
                    b = rest(in, 2) + b;
                }
            } else {
                C = L[0] * a;
                fma3(C, L[2], c);
                fma3(C, L[3], b);
            }
            edge_stencil<R, SHELL>(a, c, b, C, L, in.ob[4], fs, en);
        } else {
            R Bm[3][6], k0[3];
#pragma unroll
            for (int i = 0; i < 3; ++i) {
#pragma unroll
                for (int j = 0; j < 6; ++j) Bm[i][j] = in.ob[i * 6 + j];
                k0[i] = in.ob[NB + i];
            }
            V3<R> dd[6], C[3];
            dd[0] = mk(R(0), R(0), R(0));
#pragma unroll
            for (int j = 1; j < 6; ++j) dd[j] = diff(in, j, 0);
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                if constexpr (REL)
                    C[i] = mk(in.c0[3 * i], in.c0[3 * i + 1], in.c0[3 * i + 2]);
                else
                    C[i] = mk(R(0), R(0), R(0));
#pragma unroll
                for (int j = 1; j < 6; ++j) fma3(C[i], Bm[i][j], dd[j]);
            }
            if constexpr (REL && SHELL) {
                // the normal and its gradient use the position differences of the central triangle
                dd[1] = rest(in, 0) + dd[1];
                dd[2] = rest(in, 1) + dd[2];
            }
            tri_stencil<R, SHELL>(dd, C, Bm, k0, kb, nu, fs, en);
        }
        // the tile that owns vertex 1 of the stencil counts its energy
        if (unsigned(in.vid[0] - base) < unsigned(nown)) e_own += double(en);
#pragma unroll
        for (int j = 0; j < K; ++j) {
            unsigned slot = unsigned(in.vid[j] - base);
            if (slot < unsigned(nown)) lds_add(acc, int(slot), fs[j]);
        }
    };
    const long e0 = d.boff[2 * blk], e1 = d.boff[2 * blk + 1];
    for (long e = e0 + threadIdx.x; e < e1; e += blockDim.x) {
        In a;
        load(e, a);
        compute(a);
    }
    __syncthreads();
    gbl<R>* out = G(static_cast<R*>(d.f)) + 3 * base;
    if constexpr (!REL) {
        if (d.bias) {
            // plates with clamped edges: the constant force and energy terms that make the clamped
            // stencils rest-relative, f + F0 and E - F0 . x (+ E0 once, when the partials are summed)
            const gbl<const double>* b = G(d.bias) + 3 * base;
            for (int i = threadIdx.x; i < 3 * nown; i += blockDim.x) {
                const double bi = b[i];
                out[i] = acc[i] + bi;
                e_own -= bi * x[3 * base + i];
            }
        } else {
            for (int i = threadIdx.x; i < 3 * nown; i += blockDim.x) out[i] = R(acc[i]);
        }
    } else {
        for (int i = threadIdx.x; i < 3 * nown; i += blockDim.x) out[i] = R(acc[i]);
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
    const uint32_t lds = uint32_t(size_t(3 * lds_T) * sizeof(double));
    // start/stop (may be null) receive the dispatch's own begin and end times
    if (precision == SHELL_PREC_FP64)
        hipExtLaunchKernelGGL(force_tiles<MODEL, double>, grid, dim3(threads_d), lds, s, start, stop, 0, descs,
                              items, nitems);
    else
        hipExtLaunchKernelGGL(force_tiles<MODEL, float>, grid, dim3(threads_f), lds, s, start, stop, 0, descs,
                              items, nitems);
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

// dst[i] = (src[perm[i]] - X[i], 0): caller-order positions to internal-order displacements from the rest
// shape, padded to four doubles (the mixed-precision force kernels' input)
__global__ void gather_displacements(const double* __restrict__ src, const int32_t* __restrict__ perm,
                                     const double* __restrict__ X, double* __restrict__ dst, long nv) {
    long i = blockIdx.x * long(blockDim.x) + threadIdx.x;
    if (i >= nv) return;
    long u = perm[i];
    for (int c = 0; c < 3; ++c) dst[4 * i + c] = src[3 * u + c] - X[3 * i + c];
    dst[4 * i + 3] = 0.0;
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

void launch_energy_finalize(const double* epart, int64_t n, double add, double* energy, hipStream_t s,
                            const double* extra, int64_t m) {
    energy_finalize<<<1, 256, 0, s>>>(epart, n, add, extra, m, energy);
    SHELL_HIP(hipGetLastError());
}

void launch_gather_displacements(const double* src, const int32_t* perm, const double* X, double* dst, int64_t nv,
                                 hipStream_t s) {
    if (!nv) return;
    gather_displacements<<<(nv + 255) / 256, 256, 0, s>>>(src, perm, X, dst, nv);
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
