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

// 1/|a| for a nonzero vector: the hardware reciprocal square root estimate of |a|^2 (v_rsq), within
// about one ulp in float32; in float64 (an estimate good to some 2^-23) refined by Newton-Raphson steps
// y <- y + y (1 - s y^2) / 2, each of which squares the relative error: two reach float64 rounding, one
// (STEPS = 1) some 2^-46.  A few instructions instead of a correctly rounded square root and division.
__device__ __forceinline__ float inv_norm(V3<float> a) { return __builtin_amdgcn_rsqf(dot(a, a)); }
template <int STEPS = 2>
__device__ __forceinline__ double inv_norm(V3<double> a) {
    const double s = dot(a, a);
    double y = __builtin_amdgcn_rsq(s);
#pragma unroll
    for (int k = 0; k < STEPS; ++k) y = fma(0.5 * y, fma(-s * y, y, 1.0), y);
    return y;
}

// 1/d for d != 0 in float64: the hardware reciprocal estimate (v_rcp, good to some 2^-23) refined by two
// Newton-Raphson steps y <- y + y (1 - d y), each squaring the relative error, to float64 rounding.
__device__ __forceinline__ double inv_fast(double d) {
    double y = __builtin_amdgcn_rcp(d);
    y = fma(y, fma(-d, y, 1.0), y);
    return fma(y, fma(-d, y, 1.0), y);
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

// Order-independent accumulation of the owner-computes tiles in LDS.  Floating-point atomics add in
// whatever order the waves arrive, so their last bits would change from run to run.  Instead each
// contribution v (in units of a per-mesh power-of-two force scale, so exactly rescaled) is held in
// integers whose sums do not depend on the order of the additions (integer LDS atomics; float32 LDS
// atomics are slow here).  Float64 results (PARTS = 2): h, the count of 2^-20 nearest to v (int64, one
// ds_add_u64), and q, the count of 2^-39 nearest to the rest (int32, |q| <= 2^18, one ds_add_u32); the
// total h 2^-20 + q 2^-39 drops less than 2^-40 of the scale per contribution.  Float32 results
// (PARTS = 1): h alone, counting 2^-26, which drops less than 2^-27 of the scale, that is 2^-39 of the
// element's force unit (the scale is 2^-12 of k_b / l for bending, of E h l for the membrane), far below
// the float32 rounding of such forces.  A count below 2^51 in magnitude (a contribution below 2^31 resp.
// 2^25 times the scale, some 2^13 force units or more: nearly all of them) is rounded by one float64
// addition of 1.5 2^52, which leaves the integer in the low mantissa bits; larger ones take the general
// conversion.  A contribution of 2^56 counts or more (2^36 resp. 2^30 times the scale; with 64
// contributions per component the int64 sum stays below 2^62), or a non-finite one, sets a flag on which
// the tile writes NaN, so that the state is reported as non-finite.  LDS: 12 (PARTS = 2) or 8 bytes per
// component, and a flag.
template <int PARTS>
struct TileAccT {
    long long* hi;
    int* lo;
    int* bad;
    static constexpr double kUnit = PARTS == 2 ? 0x1p20 : 0x1p26;  // counts of h per unit of the scale
    __host__ __device__ static constexpr size_t bytes(long n) { return size_t((PARTS == 2 ? 36 : 24) * n + 16); }
    __device__ __forceinline__ TileAccT(void* smem, long n)
        : hi(static_cast<long long*>(smem)), lo(reinterpret_cast<int*>(hi + 3 * n)),
          bad(PARTS == 2 ? reinterpret_cast<int*>(lo + 3 * n) : reinterpret_cast<int*>(hi + 3 * n)) {}
    // every thread of the work-group calls it
    __device__ __forceinline__ void clear(int n3) {
        for (int i = threadIdx.x; i < n3; i += blockDim.x) {
            hi[i] = 0;
            if constexpr (PARTS == 2) lo[i] = 0;
        }
        if (threadIdx.x == 0) *bad = 0;
    }
    // t: the contribution in counts of h, that is v * kUnit (an exact power-of-two rescaling)
    __device__ __forceinline__ void add_counts(int k, double t) {
        constexpr double kMagic = 0x1.8p52;
        long long h;
        double hd;  // h as a float64
        if (fabs(t) < 0x1p51) {
            const double tm = t + kMagic;  // t rounded to an integer (ties to even), held in the low bits
            h = __double_as_longlong(tm) - __double_as_longlong(kMagic);
            hd = tm - kMagic;
        } else if (fabs(t) < 0x1p56) {
            hd = rint(t);
            h = static_cast<long long>(hd);
        } else {
            *bad = 1;
            return;
        }
        atomicAdd(reinterpret_cast<unsigned long long*>(hi + k), static_cast<unsigned long long>(h));
        if constexpr (PARTS == 2) {
            const double rest = t - hd;  // exact, |rest| <= 1/2
            atomicAdd(lo + k, int(static_cast<unsigned>(__double_as_longlong(fma(rest, 0x1p19, kMagic)))));
        }
    }
    // t with |t| < 2^51 known (a whole stencil's contributions tested at once): the rounding alone
    __device__ __forceinline__ void add_counts_small(int k, double t) {
        constexpr double kMagic = 0x1.8p52;
        const double tm = t + kMagic;
        atomicAdd(reinterpret_cast<unsigned long long*>(hi + k),
                  static_cast<unsigned long long>(__double_as_longlong(tm) - __double_as_longlong(kMagic)));
        if constexpr (PARTS == 2) {
            const double rest = t - (tm - kMagic);
            atomicAdd(lo + k, int(static_cast<unsigned>(__double_as_longlong(fma(rest, 0x1p19, kMagic)))));
        }
    }
    // the total in units of the scale, or NaN when a contribution was out of range (after a barrier)
    __device__ __forceinline__ double get(int k) const {
        if (*bad) return __builtin_nan("");
        if constexpr (PARTS == 2) return (double(hi[k]) + double(lo[k]) * 0x1p-19) * 0x1p-20;
        return double(hi[k]) * (1.0 / kUnit);
    }
};
using TileAcc = TileAccT<2>;

}  // namespace shell
