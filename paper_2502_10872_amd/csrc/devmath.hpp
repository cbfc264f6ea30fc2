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

// A 64-bit value that is the same in every lane of the wave, read from the first lane into scalar
// registers (the low word zero-extended).
__device__ __forceinline__ long uniform64(int64_t v) {
    const uint32_t lo = uint32_t(__builtin_amdgcn_readfirstlane(int(uint32_t(v))));
    const int hi = __builtin_amdgcn_readfirstlane(int(v >> 32));
    return long((uint64_t(uint32_t(hi)) << 32) | lo);
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
// atomics are slow here).  Per component an int64 h and an int32 c:
//  - float64 results (PARTS = 2): h counts 2^-20 (the nearest count to v) and c counts 2^-39 (the nearest
//    to the rest, |c| <= 2^18), two atomics per contribution (ds_add_u64, ds_add_u32); the total
//    h 2^-20 + c 2^-39 drops less than 2^-40 of the scale per contribution;
//  - float32 results (PARTS = 1): h counts 2^-26, one atomic per contribution, dropping less than 2^-27
//    of the scale, that is 2^-39 of the element's force unit (the scale is 2^-12 of k_b / l for bending,
//    of E h l for the membrane); a contribution of 2^25 times the scale or more (2^13 force units: the
//    far states of an unconverged step, its predictor included, reach beyond 2^30 times the scale on the
//    1M-vertex cap) puts its nearest multiple of 2^20 into c (counting 2^20) and the rest into h.
// A count below 2^51 in magnitude is rounded by one float64 addition of 1.5 2^52, which leaves the
// integer in the low mantissa bits.  A contribution of 2^36 times the scale or more (with 64
// contributions per component the sums stay below 2^62 and 2^24), or a non-finite one, sets a flag on
// which the tile writes NaN, so that the state is reported as non-finite.  LDS: 12 bytes per component
// and a flag.
template <int PARTS>
struct TileAccT {
    long long* hi;
    int* lo;
    int* bad;
    static constexpr double kUnit = PARTS == 2 ? 0x1p20 : 0x1p26;  // counts of h per unit of the scale
    static constexpr double kMax = 0x1p36;                          // largest contribution, in the scale
    __host__ __device__ static constexpr size_t bytes(long n) { return size_t(36 * n + 16); }
    __device__ __forceinline__ TileAccT(void* smem, long n)
        : hi(static_cast<long long*>(smem)), lo(reinterpret_cast<int*>(hi + 3 * n)),
          bad(reinterpret_cast<int*>(lo + 3 * n)) {}
    // every thread of the work-group calls it
    __device__ __forceinline__ void clear(int n3) {
        for (int i = threadIdx.x; i < n3; i += blockDim.x) {
            hi[i] = 0;
            lo[i] = 0;
        }
        if (threadIdx.x == 0) *bad = 0;
    }
    static constexpr double kMagic = 0x1.8p52;
    // the nearest integer to t, |t| < 2^51, as an int64 (one float64 addition) and as a float64
    __device__ __forceinline__ static long long round_small(double t, double& td) {
        const double tm = t + kMagic;
        td = tm - kMagic;
        return __double_as_longlong(tm) - __double_as_longlong(kMagic);
    }
    // t with |t| < 2^51 known (a whole stencil's contributions tested at once): the rounding alone
    __device__ __forceinline__ void add_counts_small(int k, double t) {
        double td;
        const long long h = round_small(t, td);
        atomicAdd(reinterpret_cast<unsigned long long*>(hi + k), static_cast<unsigned long long>(h));
        if constexpr (PARTS == 2) {
            double cd;
            atomicAdd(lo + k, int(round_small((t - td) * 0x1p19, cd)));  // t - td exact, |t - td| <= 1/2
        }
    }
    // t: the contribution in counts of h, that is v * kUnit (an exact power-of-two rescaling)
    __device__ __forceinline__ void add_counts(int k, double t) {
        if (fabs(t) < 0x1p51) {
            add_counts_small(k, t);
            return;
        }
        if (!(fabs(t) < kMax * kUnit)) {
            *bad = 1;
            return;
        }
        if constexpr (PARTS == 2) {
            const double td = rint(t);
            atomicAdd(reinterpret_cast<unsigned long long*>(hi + k),
                      static_cast<unsigned long long>(static_cast<long long>(td)));
            double cd;
            atomicAdd(lo + k, int(round_small((t - td) * 0x1p19, cd)));
        } else {
            double cd;
            const int c = int(round_small(t * (0x1p-20 / kUnit), cd));  // multiples of 2^20 of the scale
            add_counts_small(k, fma(-cd, 0x1p20 * kUnit, t));            // the rest: exact, below 2^46
            atomicAdd(lo + k, c);
        }
    }
    // the total in units of the scale, or NaN when a contribution was out of range (after a barrier)
    __device__ __forceinline__ double get(int k) const {
        if (*bad) return __builtin_nan("");
        if constexpr (PARTS == 2) return (double(hi[k]) + double(lo[k]) * 0x1p-19) * 0x1p-20;
        return double(hi[k]) * (1.0 / kUnit) + double(lo[k]) * 0x1p20;
    }
};
using TileAcc = TileAccT<2>;

}  // namespace shell
