// Small device-side helpers: 3-vectors, XCD-aware work-group mapping, wave/block reductions.
#pragma once

#include <hip/hip_runtime.h>

namespace shell {

template <typename R>
struct V3 {
    R x, y, z;
};

template <typename R>
__device__ __forceinline__ V3<R> mk(R x, R y, R z) {
    return V3<R>{x, y, z};
}
template <typename R>
__device__ __forceinline__ V3<R> operator+(V3<R> a, V3<R> b) {
    return {a.x + b.x, a.y + b.y, a.z + b.z};
}
template <typename R>
__device__ __forceinline__ V3<R> operator-(V3<R> a, V3<R> b) {
    return {a.x - b.x, a.y - b.y, a.z - b.z};
}
template <typename R>
__device__ __forceinline__ V3<R> operator-(V3<R> a) {
    return {-a.x, -a.y, -a.z};
}
template <typename R>
__device__ __forceinline__ V3<R> operator*(R s, V3<R> a) {
    return {s * a.x, s * a.y, s * a.z};
}
template <typename R>
__device__ __forceinline__ R dot(V3<R> a, V3<R> b) {
    return a.x * b.x + a.y * b.y + a.z * b.z;
}
template <typename R>
__device__ __forceinline__ V3<R> cross(V3<R> a, V3<R> b) {
    return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}
template <typename R>
__device__ __forceinline__ R norm(V3<R> a) {
    return sqrt(dot(a, a));
}
// a += s * b
template <typename R>
__device__ __forceinline__ void fma3(V3<R>& a, R s, V3<R> b) {
    a.x = fma(s, b.x, a.x);
    a.y = fma(s, b.y, a.y);
    a.z = fma(s, b.z, a.z);
}
template <typename R, typename S>
__device__ __forceinline__ V3<R> cvt(V3<S> a) {
    return {R(a.x), R(a.y), R(a.z)};
}

__device__ __forceinline__ V3<double> load3(const double* p, long i) {
    return {p[3 * i], p[3 * i + 1], p[3 * i + 2]};
}

// Pointers read out of a descriptor in memory are generic (flat) to the compiler.  Casting them to the
// global address space gives global loads and stores, which count on the vector-memory counter only,
// so LDS traffic and memory loads in flight no longer wait on each other.
template <typename T>
using gbl = __attribute__((address_space(1))) T;
template <typename T>
__device__ __forceinline__ gbl<T>* G(T* p) {
    return (gbl<T>*)p;
}

// MI355X dispatches consecutive work-groups round-robin over its 8 XCDs, each with a private L2.
// Remap so that XCD x processes one contiguous range of logical work-groups (neighbouring vertices
// and stencils then share an L2).  The grid must be launched with xcd_grid(n) work-groups; logical
// ids >= n are idle.
constexpr int kXcds = 8;
__host__ __device__ __forceinline__ long xcd_grid(long n) { return ((n + kXcds - 1) / kXcds) * kXcds; }
__device__ __forceinline__ long xcd_logical(long bid, long ngrid) {
    long per = ngrid / kXcds;
    return (bid % kXcds) * per + bid / kXcds;
}

// wave64 sum of a double through lane shuffles
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Block sum of NQ doubles per thread; result valid in thread 0.  `sh` needs NQ * (blockDim/64) doubles.
template <int NQ>
__device__ __forceinline__ void block_sum(double (&v)[NQ], double* sh) {
    int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
#pragma unroll
    for (int q = 0; q < NQ; ++q) v[q] = wave_sum(v[q]);
    __syncthreads();
    if (lane == 0)
#pragma unroll
        for (int q = 0; q < NQ; ++q) sh[q * nw + wid] = v[q];
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            double s = 0;
            for (int w = 0; w < nw; ++w) s += sh[q * nw + w];
            v[q] = s;
        }
    }
}

}  // namespace shell

namespace shell {

// Order-independent float64 accumulation of the owner-computes tiles in LDS.  Floating-point atomics
// add in whatever order the waves arrive, so their last bits would change from run to run.  Instead each
// contribution v (in units of a per-mesh power-of-two force scale, so exactly rescaled) is split into a
// float64 part h, v rounded to a multiple of 2^-30 (by adding and subtracting 1.5 * 2^22, whose ulp that
// is), and an integer count q of 2^-49 in the rest (the low bits of the rest plus 12, whose ulp is 2^-49),
// each added with its own LDS atomic (ds_add_f64, ds_add_u32; float32 LDS atomics are slow here).  While
// |v| < 2^17, every partial sum of up to 64 h parts is a multiple of 2^-30 below 2^23, so exactly
// representable, and the counts (|q| <= 2^18) are integers: neither total depends on the order of the
// additions.  What is dropped is below 2^-50 of the scale per contribution.  A contribution outside that
// range (2^17 times the scale is about a hundred times the force of a kink at the element scale) is added
// whole to the float64 part, which keeps the sum finite but makes its last bits order-dependent; a
// non-finite one propagates.  LDS: 12 bytes per component.
struct TileAcc {
    double* hi;
    int* lo;
    static constexpr double kMax = 0x1p17;
    __host__ __device__ static constexpr size_t bytes(long n) { return size_t(36 * n); }
    __device__ __forceinline__ TileAcc(void* smem, long n)
        : hi(static_cast<double*>(smem)), lo(reinterpret_cast<int*>(hi + 3 * n)) {}
    // every thread of the work-group calls it
    __device__ __forceinline__ void clear(int n3) {
        for (int i = threadIdx.x; i < n3; i += blockDim.x) {
            hi[i] = 0.0;
            lo[i] = 0;
        }
    }
    __device__ __forceinline__ void add(int k, double v) {
        if (!(fabs(v) < kMax)) {
            atomicAdd(hi + k, v);
            return;
        }
        const double h = (v + 0x1.8p22) - 0x1.8p22;
        // 12 + (v - h) lies in [8, 16), where the ulp is 2^-49 and 12's low 32 mantissa bits are zero
        const int q = __double2loint((v - h) + 0x1.8p3);
        atomicAdd(hi + k, h);
        atomicAdd(lo + k, q);
    }
    __device__ __forceinline__ double get(int k) const { return hi[k] + double(lo[k]) * 0x1p-49; }
};

}  // namespace shell
