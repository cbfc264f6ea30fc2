// Row product of the SELL-64 constant Hessian with a three-column [nv][3] vector.
//
// One wave owns one 64-row slice, one lane one row: the slice width and offset are wave-uniform
// (scalar registers), column ids and values are read 64 at a time (coalesced), and entries are taken
// in batches of 8 so that each lane keeps 16 streaming loads and 8 gathers in flight instead of one
// dependent chain per entry.
#pragma once

#include <hip/hip_runtime.h>

#include "devmath.hpp"

#ifndef SHELL_SPMV_BATCH
#define SHELL_SPMV_BATCH 8  // entries per batch: loads in flight per lane
#endif
#ifndef SHELL_SPMV_NT
#define SHELL_SPMV_NT 0  // 1: stream the matrix with non-temporal loads (measured slower in float32)
#endif

namespace shell {

template <typename T>
__device__ __forceinline__ T stream_load(const gbl<const T>* p) {
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
    const gbl<const int32_t>* gcol = G(scol);
    const gbl<const MR>* gval = G(val);
    const gbl<const VR>* gp = G(p);
    const long slice = row >> 6;
    // the whole wave shares the slice (work-groups are whole waves aligned to 64 rows)
    const int w = __builtin_amdgcn_readfirstlane(G(width)[slice]);
    const int64_t sp = G(sptr)[slice];
    const long s0 = uniform64(sp) + (row & 63);
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
            c[u] = stream_load(gcol + s0 + 64L * (k + u));
            a[u] = stream_load(gval + s0 + 64L * (k + u));
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const gbl<const VR>* pc = gp + 3L * c[u];
            ax = fma(a[u], MR(pc[0]), ax);
            ay = fma(a[u], MR(pc[1]), ay);
            az = fma(a[u], MR(pc[2]), az);
        }
    }
    const int rem = w - k;  // wave-uniform
    if (rem > 0) {
        // one more batch with the slots past the row's end clamped to its last entry and weighted 0, so
        // that every load is issued at once (the clamped ones hit lines already being fetched)
        int c[U];
        MR a[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const long off = s0 + 64L * (k + (u < rem ? u : rem - 1));
            c[u] = stream_load(gcol + off);
            a[u] = stream_load(gval + off);
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const gbl<const VR>* pc = gp + 3L * c[u];
            const MR au = u < rem ? a[u] : MR(0);
            ax = fma(au, MR(pc[0]), ax);
            ay = fma(au, MR(pc[1]), ay);
            az = fma(au, MR(pc[2]), az);
        }
    }
}

// Stage the p entries of a row group's distinct columns into LDS: ps[3k..3k+2] = p[gcols[k]].
// Each distinct neighbour is fetched once per group instead of once per nonzero (about 12x fewer
// gathers on triangle meshes).  Every thread of the work-group must call it.
template <typename VR>
__device__ __forceinline__ void stage_group_columns(const int32_t* __restrict__ gptr,
                                                    const int32_t* __restrict__ gcols, long group,
                                                    const VR* __restrict__ p, VR* __restrict__ ps) {
    const int a = gptr[group], n = gptr[group + 1] - a;
    for (int k = threadIdx.x; k < n; k += blockDim.x) {
        const gbl<const VR>* pc = G(p) + 3L * G(gcols)[a + k];
        ps[3 * k] = pc[0];
        ps[3 * k + 1] = pc[1];
        ps[3 * k + 2] = pc[2];
    }
}

// The same row product with 16-bit group-local column indices and p read from the staged LDS copy.
template <typename MR, typename VR>
__device__ __forceinline__ void sell_row_product_staged(const uint16_t* __restrict__ lcol,
                                                        const MR* __restrict__ val,
                                                        const int64_t* __restrict__ sptr,
                                                        const int32_t* __restrict__ width, long row,
                                                        const VR* __restrict__ ps, MR& ax, MR& ay, MR& az) {
    const gbl<const uint16_t>* glc = G(lcol);
    const gbl<const MR>* gval = G(val);
    const long slice = row >> 6;
    const int w = __builtin_amdgcn_readfirstlane(G(width)[slice]);
    const int64_t sp = G(sptr)[slice];
    const long s0 = uniform64(sp) + (row & 63);
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
            c[u] = stream_load(glc + s0 + 64L * (k + u));
            a[u] = stream_load(gval + s0 + 64L * (k + u));
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const VR* pc = ps + 3 * c[u];
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
            const long off = s0 + 64L * (k + (u < rem ? u : rem - 1));
            c[u] = stream_load(glc + off);
            a[u] = stream_load(gval + off);
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const VR* pc = ps + 3 * c[u];
            const MR au = u < rem ? a[u] : MR(0);
            ax = fma(au, MR(pc[0]), ax);
            ay = fma(au, MR(pc[1]), ay);
            az = fma(au, MR(pc[2]), az);
        }
    }
}

// One lane's row of a 64-row SELL slice read as a stream of batches of U (column id, value) pairs.  A
// batch can be requested before it is needed: the product asks for the first one before staging its
// row group's directions in LDS, and for each next one while it multiplies the current one.  Slots past
// the row's stored width are clamped to its last slot (the value is then weighted 0 by the consumer).
// Every lane of a wave belongs to the same slice, so width and offset are wave-uniform.
template <typename MR, typename IDX, int U>
struct SellStream {
    const gbl<const IDX>* col;
    const gbl<const MR>* val;
    long s0;
    int w;

    __device__ __forceinline__ SellStream(const IDX* col_, const void* val_, const int64_t* sptr,
                                          const int32_t* width, long row)
        : col(G(col_)), val(G(static_cast<const MR*>(val_))) {
        const long slice = row >> 6;
        w = __builtin_amdgcn_readfirstlane(G(width)[slice]);
        const int64_t sp = G(sptr)[slice];
        s0 = uniform64(sp) + (row & 63);
    }

    // A float64 matrix (twice the bytes of the vectors it meets) is read with non-temporal loads, which
    // keep it from displacing the direction and product vectors that the update kernel reads next from
    // the last-level cache (measured: FP64 iteration 105 -> 96 us on a 1M-vertex mesh); a float32 matrix
    // is read with plain loads (non-temporal measured slower there).
    __device__ __forceinline__ void load(int k, int (&c)[U], MR (&a)[U]) const {
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const long off = s0 + 64L * (k + u < w ? k + u : w - 1);
            if constexpr (sizeof(MR) == 8) {
                c[u] = int(__builtin_nontemporal_load(col + off));
                a[u] = __builtin_nontemporal_load(val + off);
            } else {
                c[u] = int(col[off]);
                a[u] = val[off];
            }
        }
    }
};

}  // namespace shell
