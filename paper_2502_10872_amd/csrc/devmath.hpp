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
