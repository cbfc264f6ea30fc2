// Row product of the SELL-64 constant Hessian with a three-column [nv][3] vector.
//
// One wave owns one 64-row slice, one lane one row: the slice width and offset are wave-uniform
// (scalar registers), column ids and values are read 64 at a time (coalesced), and entries are taken
// in batches of 8 so that each lane keeps 16 streaming loads and 8 gathers in flight instead of one
// dependent chain per entry.
#pragma once

#include <hip/hip_runtime.h>

#ifndef SHELL_SPMV_BATCH
#define SHELL_SPMV_BATCH 8  // entries per batch: loads in flight per lane
#endif
#ifndef SHELL_SPMV_NT
#define SHELL_SPMV_NT 0  // 1: stream the matrix with non-temporal loads (measured slower in float32)
#endif

namespace shell {

template <typename T>
__device__ __forceinline__ T stream_load(const T* p) {
#if SHELL_SPMV_NT
    return __builtin_nontemporal_load(p);
#else
    return *p;
#endif
}

template <typename MR, typename VR>
__device__ __forceinline__ void sell_row_product(const int32_t* __restrict__ scol, const MR* __restrict__ val,
                                                 const int64_t* __restrict__ sptr,
                                                 const int32_t* __restrict__ width, long row, const VR* __restrict__ p,
                                                 MR& ax, MR& ay, MR& az) {
    const long slice = row >> 6;
    // the whole wave shares the slice (work-groups are whole waves aligned to 64 rows)
    const int w = __builtin_amdgcn_readfirstlane(width[slice]);
    const long s0 = (long(__builtin_amdgcn_readfirstlane(int(sptr[slice] & 0xffffffff))) |
                     (long(__builtin_amdgcn_readfirstlane(int(sptr[slice] >> 32))) << 32)) +
                    (row & 63);
    ax = MR(0);
    ay = MR(0);
    az = MR(0);
    constexpr int U = SHELL_SPMV_BATCH;
    int k = 0;
    for (; k + U <= w; k += U) {
        int c[U];
        MR a[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            c[u] = stream_load(scol + s0 + 64L * (k + u));
            a[u] = stream_load(val + s0 + 64L * (k + u));
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const VR* pc = p + 3L * c[u];
            ax = fma(a[u], MR(pc[0]), ax);
            ay = fma(a[u], MR(pc[1]), ay);
            az = fma(a[u], MR(pc[2]), az);
        }
    }
    const int rem = w - k;  // wave-uniform
    if (rem > 0) {
        int c[U];
        MR a[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if (u < rem) {
                c[u] = stream_load(scol + s0 + 64L * (k + u));
                a[u] = stream_load(val + s0 + 64L * (k + u));
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if (u < rem) {
                const VR* pc = p + 3L * c[u];
                ax = fma(a[u], MR(pc[0]), ax);
                ay = fma(a[u], MR(pc[1]), ay);
                az = fma(a[u], MR(pc[2]), az);
            }
        }
    }
}

}  // namespace shell
