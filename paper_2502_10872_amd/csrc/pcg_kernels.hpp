// Device kernels of the implicit step (see solver.hip for the step they make up): predictor, Jacobi
// diagonal, Newton residual, the two PCG kernels with their binned dot products, Newton and velocity
// updates, lumped mass.  Included once, by solver.hip.
#pragma once

#include <cmath>

#include "devmath.hpp"
#include "internal.hpp"
#include "spmv.hpp"

namespace shell {

namespace {


constexpr int kBlk = kRowGroup;  // rows per work item (one row per thread)
constexpr int kRedBlk = 512;  // residual-norm kernel: one work-group per mesh
constexpr int kMaxPart = 8;   // partial quantities per work-group (buffer sized kMaxPart * groups)

inline long blocks(long n) { return (n + kBlk - 1) / kBlk; }

// Whether z = D^-1 r is stored (mixed precision: a float z, 12 B, is read instead of the FP64 r and the
// Jacobi entry, 28 B, for every staged column; in FP64 storing z would cost more than it saves).
template <typename VR>
constexpr bool kStoredZ = sizeof(VR) == 4;

// Mixed precision keeps the PCG increment y in float32 and folds it into a float64 accumulator y64 every
// kFoldIters iterations of its column (when that column's count is kFoldIters - 1 mod kFoldIters): one
// float32 rounding per iteration would otherwise leave y about sqrt(iterations) * eps_32 off after a long
// solve (4e-6 after 19,000 iterations on the 256 x 256 sphere cap), while a float64 y would add 24 B per
// row to every update.  The fold reads and writes y64 once per kFoldIters iterations.  The condition
// uses the device-side iteration count, so where the folds fall does not depend on how the iterations
// were launched.
constexpr int kFoldIters = 16;

// Whether the product applies K_s in difference form, (K_s p)_i = sum_j K_ij (p_j - p_i) (float32
// matrix).  Every row of K_s sums to zero (constants are in its null space, eq 12), but float32 entries
// rounded one at a time do not: a row then sums to about eps_32 |K_ii|, which on a fine mesh outweighs
// the mass term m_i / dt^2 in the step matrix and spoils its smoothest modes (on the 512 x 512 sphere cap
// the solution of one step system moves by 1e-3).  In difference form the diagonal entry meets p_i - p_i
// = 0 and the implied diagonal is minus the sum of the rounded off-diagonals, so each row sums to zero
// exactly (solution error 2e-7 on the same system).  The float64 matrix keeps the plain form.
template <typename MR>
constexpr bool kDiffForm = sizeof(MR) == 4;

// fixed-order sum of NQ partials over ngroups work-groups; result in thread 0's out[]
template <int NQ>
__device__ void reduce_partials(const double* __restrict__ part, long ngroups, double (&out)[NQ]) {
    __shared__ double sh[NQ * (kRedBlk / 64)];
    for (int q = 0; q < NQ; ++q) out[q] = 0.0;
    // partials are stored quantity-major, part[q * ngroups + group], so these loads coalesce
#pragma unroll 4
    for (long b = threadIdx.x; b < ngroups; b += kRedBlk)
#pragma unroll
        for (int q = 0; q < NQ; ++q) out[q] += part[q * ngroups + b];
    block_sum<NQ>(out, sh);
}

// this work-group's (mesh, row group); false if the grid slot is idle
__device__ __forceinline__ bool work_item(const WorkItem* __restrict__ items, long nitems, WorkItem& wi) {
    long it = xcd_logical(blockIdx.x, gridDim.x);
    if (it >= nitems) return false;
    wi = items[it];
    return true;
}

// ---------------------------------------------------------------- PCG dot products
// Each work-group sums its rows' partial dot products of a mesh (in its fixed walk order and a fixed
// block tree) and stores them, without atomics, in its own slot of that mesh's partials: slot = its
// logical work-group id.  The kernel that needs a total sums the slots of the work-groups that can touch
// the mesh ([pq_lo, pq_hi) for the product launch, [rz_lo, rz_hi) for the update launch, set by the host
// for each launch shape) in a fixed order (bin_totals), so every work-group obtains the same bits, and so
// does every run.  Slots of
// work-groups in the range that never meet the mesh stay at the zero written when the solve starts.
// Partials are double-buffered by iteration parity, so a kernel never writes a set a running kernel
// reads.
constexpr int kSlots = 1024;  // largest logical work-group count of a PCG launch
constexpr int kBinQ = 8;      // quantity slots per set
constexpr int kSetPq = 0, kSetRz = 1;  // p.q (3 quantities); r.z and r.r (6)

__device__ __forceinline__ double* bin_set(const SolveDesc& d, long par, int set) {
    return d.bins + (size_t(par & 1) * 2 + size_t(set)) * kBinQ * kSlots;
}

// totals of NQ quantities over the slots [lo, hi), in every thread of the work-group (every thread calls
// it; it holds barriers): wave w adds slots lo + 64 w + lane, lo + 64 (w + W) + lane, ... (W waves) and
// sums them across the wave with a butterfly, then every thread adds the W wave sums in order.  One slot
// per lane and quantity on a 512-slot set, so the update kernel starts after one round of loads.
template <int NQ>
__device__ __forceinline__ void bin_totals(const double* set, int lo, int hi, double (&tot)[NQ], double* sh) {
    const gbl<const double>* b = G(set);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = blockDim.x >> 6;
    double v[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) v[q] = 0.0;
    for (int k = lo + 64 * w + lane; k < hi; k += 64 * nw)
#pragma unroll
        for (int q = 0; q < NQ; ++q) v[q] += b[q * kSlots + k];
#pragma unroll
    for (int q = 0; q < NQ; ++q) v[q] = wave_sum(v[q]);
    __syncthreads();  // a previous use of sh is over
    if (lane == 0)
#pragma unroll
        for (int q = 0; q < NQ; ++q) sh[q * nw + w] = v[q];
    __syncthreads();
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        double t = 0.0;
        for (int k = 0; k < nw; ++k) t += sh[q * nw + k];
        tot[q] = t;
    }
}

// the same totals computed by each wave on its own (no barrier), lane k adding slots lo + k, lo + k + 64,
// ... in order: the product kernel uses it, whose waves then go on to issue their own loads at once
template <int NQ>
__device__ __forceinline__ void bin_totals_wave(const double* set, int lo, int hi, double (&tot)[NQ]) {
    const gbl<const double>* b = G(set);
#pragma unroll
    for (int q = 0; q < NQ; ++q) tot[q] = 0.0;
    for (int k = lo + int(threadIdx.x & 63); k < hi; k += 64)
#pragma unroll
        for (int q = 0; q < NQ; ++q) tot[q] += b[q * kSlots + k];
#pragma unroll
    for (int q = 0; q < NQ; ++q) tot[q] = wave_sum(tot[q]);
}

template <int NQ>
__device__ __forceinline__ void bin_store(double* set, int slot, const double (&v)[NQ]) {
#pragma unroll
    for (int q = 0; q < NQ; ++q) G(set)[q * kSlots + slot] = v[q];
}

// zeroes every set of a mesh's partials; every thread of the work-group takes part
__device__ __forceinline__ void bin_clear_all(const SolveDesc& d) {
    for (int k = threadIdx.x; k < 2 * 2 * kBinQ * kSlots; k += blockDim.x) G(d.bins)[k] = 0.0;
}

__global__ __launch_bounds__(kBlk) void k_predictor(const SolveDesc* __restrict__ descs, const WorkItem* __restrict__ items, long nitems) {
    WorkItem wi;
    if (!work_item(items, nitems, wi)) return;
    const SolveDesc& d = descs[wi.mesh];
    long i = long(wi.unit) * kBlk + threadIdx.x;
    if (i >= d.nv) return;
    const unsigned held = d.pinned[i];
    for (int c = 0; c < 3; ++c) {
        double xi = d.x[3 * i + c];
        d.xt[3 * i + c] = xi;
        // dt = 0 (the quasi-static solve): x_hat = x without reading the velocity
        double xh = ((held >> c & 1u) || d.dt == 0.0) ? xi : xi + d.dt * d.v[3 * i + c] + d.dt * d.dt * d.grav[c];
        d.xhat[3 * i + c] = xh;
        d.x[3 * i + c] = xh;
    }
}

template <typename VR>
__global__ __launch_bounds__(kBlk) void k_dinv(const SolveDesc* __restrict__ descs, const WorkItem* __restrict__ items, long nitems) {
    WorkItem wi;
    if (!work_item(items, nitems, wi)) return;
    const SolveDesc& d = descs[wi.mesh];
    long i = long(wi.unit) * kBlk + threadIdx.x;
    if (i >= d.nv) return;
    const bool pin = (d.pinned[i] & 7u) == 7u;  // every coordinate held
    const double den = d.mass[i] + d.dt2 * d.kdiag[i];  // zero only for a quasi-static row without stiffness
    static_cast<VR*>(d.dinv)[i] = (pin || den == 0.0) ? VR(0) : VR(1.0 / den);
    // the product reads one value per row for both the mass and the fixed flag
    static_cast<VR*>(d.mq)[i] = pin ? VR(-1) : VR(d.mass[i]);
}

// g = M (x - x_hat) - dt^2 (f + F), fixed rows zero (F: the quasi-static load, absent in a time step);
// partial |g|^2
template <typename VR>
__global__ __launch_bounds__(kBlk) void k_residual(const SolveDesc* __restrict__ descs, const WorkItem* __restrict__ items, long nitems,
                           int from_xhat) {
    WorkItem wi;
    if (!work_item(items, nitems, wi)) return;
    const SolveDesc& d = descs[wi.mesh];
    const VR* __restrict__ f = static_cast<const VR*>(d.f);
    const double* __restrict__ xh = from_xhat ? d.xhat : d.x;
    long i = long(wi.unit) * kBlk + threadIdx.x;
    double acc[1] = {0.0};
    if (i < d.nv) {
        const unsigned held = d.pinned[i];
        double m = d.mass[i];
        for (int c = 0; c < 3; ++c) {
            double fi = double(f[3 * i + c]);
            if (d.fext) fi += d.fext[3 * i + c];
            double gi = (held >> c & 1u) ? 0.0 : m * (d.x[3 * i + c] - xh[3 * i + c]) - d.dt2 * fi;
            d.g[3 * i + c] = gi;
            acc[0] += gi * gi;
        }
    }
    __shared__ double sh[kBlk / 64];
    block_sum<1>(acc, sh);
    if (threadIdx.x == 0) d.part[wi.unit] = acc[0];
}

// |g|^2 of each mesh; also zeroes the dot-product partials of the coming solve
__global__ __launch_bounds__(kRedBlk) void k_fin_residual(const SolveDesc* __restrict__ descs, const int32_t* __restrict__ meshes) {
    const SolveDesc& d = descs[meshes[blockIdx.x]];
    double tot[1];
    reduce_partials<1>(d.part, d.ngroups, tot);
    bin_clear_all(d);
    if (threadIdx.x == 0) {
        d.st[0].gsq = tot[0];
        d.st[0].nonfinite = !isfinite(tot[0]);
    }
}

// What the rest of a product needs of the recurrence state.
struct ProductState {
    double beta[3];
    int done;
};

// The recurrence state entering product t: at t == 0 from the initial residual, else the previous state
// (parity t) advanced by the update of iteration t - 1 (beta, activity, counts, budget).  Every lane of
// every work-group computes beta and done identically from the partials; thread 0 of row group 0's
// work-group stores the new state (parity t + 1) field by field.
__device__ __forceinline__ ProductState product_state(const SolveDesc& d, const WorkItem& wi, long t) {
    const PcgState* so = d.st + (t & 1);
    PcgState* sn = d.st + ((t + 1) & 1);
    const bool writer = wi.unit == 0 && threadIdx.x == 0;
    double tot[6];
    bin_totals_wave<6>(bin_set(d, t + 1, kSetRz), d.rz_lo, d.rz_hi, tot);
    ProductState r;
    int any = 0;
    if (t == 0) {
        for (int c = 0; c < 3; ++c) {
            const double tol2 = d.tol2_abs[c] > 0.0 ? d.tol2_abs[c] : d.rtol2 * tot[3 + c];
            const int act = (0 < d.target[c]) && (d.replay || tot[3 + c] > tol2);
            r.beta[c] = 0.0;
            any |= act;
            if (writer) {
                sn->rz[c] = tot[c];
                sn->rr[c] = tot[3 + c];
                sn->tol2[c] = tol2;
                sn->alpha[c] = 0.0;
                sn->beta[c] = 0.0;
                sn->iters[c] = 0;
                sn->target[c] = d.target[c];
                sn->active[c] = act;
            }
        }
        r.done = !any;
        if (writer) {
            sn->done = r.done;
            sn->budget = 0;
            sn->replay = d.replay;
            sn->nonfinite = 0;
        }
    } else if (so->done) {
        for (int c = 0; c < 3; ++c) r.beta[c] = 0.0;
        r.done = 1;
        if (writer) *sn = *so;
    } else {
        const int replay = so->replay;
        int budget = so->budget, nonfinite = so->nonfinite;
        for (int c = 0; c < 3; ++c) {
            int act = so->active[c], it = so->iters[c];
            const int target = so->target[c];
            const double rz = so->rz[c], tol2 = so->tol2[c];
            double beta = 0.0;
            if (act) {
                beta = rz != 0.0 ? tot[c] / rz : 0.0;
                it += 1;
                const bool more = replay || tot[3 + c] > tol2;
                if (!replay && it >= target && more) budget = 1;
                act = (it < target) && more;
                if (!isfinite(tot[3 + c])) {
                    nonfinite = 1;
                    act = 0;
                }
            }
            r.beta[c] = beta;
            any |= act;
            if (writer) {
                const bool was = so->active[c];
                sn->rz[c] = was ? tot[c] : rz;
                sn->rr[c] = was ? tot[3 + c] : so->rr[c];
                sn->tol2[c] = tol2;
                sn->alpha[c] = so->alpha[c];
                sn->beta[c] = beta;
                sn->iters[c] = it;
                sn->target[c] = target;
                sn->active[c] = act;
            }
        }
        r.done = !any;
        if (writer) {
            sn->done = r.done;
            sn->budget = budget;
            sn->replay = replay;
            sn->nonfinite = nonfinite;
            sn->gsq = so->gsq;
        }
    }
    return r;
}

// Inputs of the search-direction update p = z + beta p_old, z = D^-1 r.
template <typename VR>
struct DirIn {
    const gbl<const double>* r;
    const gbl<const VR>* dinv;
    const gbl<const VR>* z;  // stored z (mixed precision)
    const gbl<const VR>* pold;
    VR beta[3];
};

// The operands of vertex j's direction, loaded ahead of beta: the loads can be issued before the
// recurrence state is known.  p_old is read even where beta is 0 (it is allocated; its contents then do
// not matter).  The stored z equals D^-1 r computed the same way, so both forms give the same bits.
template <typename VR>
struct DirLoad {
    VR dj;
    double rj[3];
    VR zj[3], po[3];
    __device__ __forceinline__ void load(const DirIn<VR>& in, long j) {
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            if constexpr (kStoredZ<VR>)
                zj[c] = in.z[3 * j + c];
            else
                rj[c] = in.r[3 * j + c];
            po[c] = in.pold[3 * j + c];
        }
        if constexpr (!kStoredZ<VR>) dj = in.dinv[j];
    }
    __device__ __forceinline__ void finish(const VR (&beta)[3], VR (&pj)[3]) const {
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            VR z;
            if constexpr (kStoredZ<VR>)
                z = zj[c];
            else
                z = dj * VR(rj[c]);
            pj[c] = beta[c] != VR(0) ? fma(beta[c], po[c], z) : z;
        }
    }
};

// p of vertex j with the operands' loads issued together
template <typename VR>
__device__ __forceinline__ void direction(const DirIn<VR>& in, long j, VR (&pj)[3]) {
    DirLoad<VR> l;
    l.load(in, j);
    l.finish(in.beta, pj);
}

// Row product for row groups too wide to stage: each neighbour's new direction is formed from its own
// gathers (four entries in flight per lane).
template <typename MR, typename VR>
__device__ __forceinline__ void row_product_direction(const SolveDesc& d, long row, const DirIn<VR>& in,
                                                      const VR (&pi)[3], MR& ax, MR& ay, MR& az) {
    const gbl<const int32_t>* scol = G(d.scol);
    const gbl<const MR>* val = G(static_cast<const MR*>(d.val));
    const long slice = row >> 6;
    const int w = __builtin_amdgcn_readfirstlane(G(d.width)[slice]);
    const long s0 = G(d.sptr)[slice] + (row & 63);
    ax = MR(0);
    ay = MR(0);
    az = MR(0);
    constexpr int U = 4;
    for (int k = 0; k < w; k += U) {
        int c[U];
        MR a[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const bool in_row = k + u < w;  // wave-uniform
            c[u] = in_row ? scol[s0 + 64L * (k + u)] : int(row);
            a[u] = in_row ? val[s0 + 64L * (k + u)] : MR(0);
        }
        VR pc[U][3];
#pragma unroll
        for (int u = 0; u < U; ++u) direction<VR>(in, c[u], pc[u]);
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if constexpr (kDiffForm<MR>) {
                ax = fma(a[u], MR(pc[u][0]) - MR(pi[0]), ax);
                ay = fma(a[u], MR(pc[u][1]) - MR(pi[1]), ay);
                az = fma(a[u], MR(pc[u][2]) - MR(pi[2]), az);
            } else {
                ax = fma(a[u], MR(pc[u][0]), ax);
                ay = fma(a[u], MR(pc[u][1]), ay);
                az = fma(a[u], MR(pc[u][2]), az);
            }
        }
    }
}

#ifndef SHELL_PRODUCT_BATCH
#define SHELL_PRODUCT_BATCH 8  // matrix entries per batch of the product's stream
#endif

// A vertex with some of its coordinates held: those coordinates' rows of q are zero (with the residual
// zero there from the start, r, z, p and the increment then stay zero on them).  Vertices with every
// coordinate held are the fixed rows of mq.
template <typename VR>
__device__ __forceinline__ void zero_held_rows(const SolveDesc& d, long i, VR (&qv)[3]) {
    const unsigned held = G(d.pinned)[i];
    if (held & 1u) qv[0] = VR(0);
    if (held & 2u) qv[1] = VR(0);
    if (held & 4u) qv[2] = VR(0);
}

// Unstaged product (row groups too wide for LDS): the same quantities with every neighbour's direction
// formed from its own gathers.
template <typename VR, typename MR>
__device__ __forceinline__ void product_direct(const SolveDesc& d, const WorkItem& wi, const DirIn<VR>& in,
                                               gbl<VR>* pnew, double (&acc)[3]) {
    const long i = long(wi.unit) * kBlk + threadIdx.x;
    if (i >= d.nv) return;
    const VR mq = G(static_cast<const VR*>(d.mq))[i];
    const MR m = MR(mq);
    const bool pin = mq < VR(0);
    VR pi[3];
    direction<VR>(in, i, pi);
    MR ax, ay, az;
    row_product_direction<MR, VR>(d, i, in, pi, ax, ay, az);
    VR qv[3] = {0, 0, 0};
    if (!pin) {
        const MR dt2 = MR(d.dt2);
        qv[0] = VR(fma(m, MR(pi[0]), dt2 * ax));
        qv[1] = VR(fma(m, MR(pi[1]), dt2 * ay));
        qv[2] = VR(fma(m, MR(pi[2]), dt2 * az));
    }
    if (d.partial_held) zero_held_rows(d, i, qv);
    gbl<VR>* q = G(static_cast<VR*>(d.q));
#pragma unroll
    for (int e = 0; e < 3; ++e) {
        pnew[3 * i + e] = pi[e];
        q[3 * i + e] = qv[e];
        acc[e] += double(pi[e]) * double(qv[e]);
    }
}

// Staged product of one row group: p = z + beta p_old for the group's distinct columns (staged in LDS)
// and its own rows (written), then q = (M + dt^2 K_s) p on the free rows (fixed rows 0); p.q added to
// acc.  The row's first batch of matrix entries is requested together with the staged columns'
// operands, and every next batch while the current one is multiplied.  Every thread of the work-group
// calls it (it holds a barrier); it starts with one so that the LDS of the previous group is free.
template <typename VR, typename MR>
__device__ __forceinline__ void product_staged(const SolveDesc& d, const WorkItem& wi, const DirIn<VR>& in,
                                               gbl<VR>* pnew, VR* ps, double (&acc)[3]) {
    // batches of 8 float or 4 double values (two batches in flight per lane)
    constexpr int U = sizeof(MR) == 8 ? SHELL_PRODUCT_BATCH / 2 : SHELL_PRODUCT_BATCH;
    const long i = long(wi.unit) * kBlk + threadIdx.x;
    // every slice holds 64 rows, so a wave whose first row exists reads its slice for all its lanes
    const bool wave_live = i - (threadIdx.x & 63) < d.nv;
    const bool own = i < d.nv;
    SellStream<MR, uint16_t, U> row(d.lcol, d.val, d.sptr, d.width, wave_live ? i : 0);
    int c[U];
    MR a[U];
    if (wave_live && row.w > 0) row.load(0, c, a);
    MR m = 0;
    bool pin = true;
    DirLoad<VR> own_op;
    if (own) {
        const VR mq = G(static_cast<const VR*>(d.mq))[i];
        m = MR(mq);
        pin = mq < VR(0);
        own_op.load(in, i);
    }
    // staged columns: two per pass so that each lane has two sets of gathers in flight (a lane past
    // the end repeats its first column: same value, same LDS slot)
    const int ga = G(d.gptr)[wi.unit], n = G(d.gptr)[wi.unit + 1] - ga;
    const gbl<const int32_t>* gc = G(d.gcols + ga);
    int k = threadIdx.x, k2 = k + kBlk < n ? k + kBlk : k;
    DirLoad<VR> op0, op1;
    if (k < n) {
        op0.load(in, gc[k]);
        op1.load(in, gc[k2]);
    }
    __syncthreads();
    while (k < n) {
        VR p0[3], p1[3];
        op0.finish(in.beta, p0);
        op1.finish(in.beta, p1);
#pragma unroll
        for (int e = 0; e < 3; ++e) {
            ps[3 * k + e] = p0[e];
            ps[3 * k2 + e] = p1[e];
        }
        k += 2 * kBlk;
        if (k >= n) break;
        k2 = k + kBlk < n ? k + kBlk : k;
        op0.load(in, gc[k]);
        op1.load(in, gc[k2]);
    }
    __syncthreads();
    if (!wave_live) return;
    // the row's own direction (the same bits as its staged copy)
    VR pi[3] = {0, 0, 0};
    if (own) own_op.finish(in.beta, pi);
    MR ax = 0, ay = 0, az = 0;
    for (int kk = 0; kk < row.w; kk += U) {
        int cn[U];
        MR an[U];
        const bool more = kk + U < row.w;  // wave-uniform
        if (more) row.load(kk + U, cn, an);
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const VR* pc = ps + 3 * c[u];
            const MR au = kk + u < row.w ? a[u] : MR(0);
            if constexpr (kDiffForm<MR>) {
                ax = fma(au, MR(pc[0]) - MR(pi[0]), ax);
                ay = fma(au, MR(pc[1]) - MR(pi[1]), ay);
                az = fma(au, MR(pc[2]) - MR(pi[2]), az);
            } else {
                ax = fma(au, MR(pc[0]), ax);
                ay = fma(au, MR(pc[1]), ay);
                az = fma(au, MR(pc[2]), az);
            }
        }
        if (more)
#pragma unroll
            for (int u = 0; u < U; ++u) {
                c[u] = cn[u];
                a[u] = an[u];
            }
    }
    if (!own) return;
    VR qv[3] = {0, 0, 0};
    if (!pin) {
        const MR dt2 = MR(d.dt2);
        qv[0] = VR(fma(m, MR(pi[0]), dt2 * ax));
        qv[1] = VR(fma(m, MR(pi[1]), dt2 * ay));
        qv[2] = VR(fma(m, MR(pi[2]), dt2 * az));
    }
    if (d.partial_held) zero_held_rows(d, i, qv);
    gbl<VR>* q = G(static_cast<VR*>(d.q));
#pragma unroll
    for (int e = 0; e < 3; ++e) {
        pnew[3 * i + e] = pi[e];
        q[3 * i + e] = qv[e];
        acc[e] += double(pi[e]) * double(qv[e]);
    }
}

// The work items [first, last) of this work-group: `per` consecutive items of the XCD-remapped
// logical work-group (consecutive items are neighbouring row groups, usually of one mesh)
__device__ __forceinline__ bool item_range(long nitems, int per, long& first, long& last) {
    first = xcd_logical(blockIdx.x, gridDim.x) * per;
    last = first + per < nitems ? first + per : nitems;
    return first < nitems;
}

// The product's work items: each XCD takes one contiguous run of per * W items (W work-groups per XCD),
// and its work-groups interleave within that run (items first, first + W, ...).  The W row groups in
// flight on one XCD at any time are then neighbours, whose staged columns overlap, so a column fetched
// for one group is found in that XCD's L2 by the next (measured 5% faster than consecutive items per
// work-group on a 1M-vertex mesh).  A mesh's unit 0 still opens a run of that mesh in its work-group's
// item list, which the recurrence-state writer and the bin clearing rely on.
__device__ __forceinline__ bool item_stride(long nitems, int per, long& first, long& last, long& step) {
    const long W = gridDim.x / kXcds;
    const long L = xcd_logical(blockIdx.x, gridDim.x);
    const long run = long(per) * W;
    first = (L / W) * run + L % W;
    last = (L / W + 1) * run < nitems ? (L / W + 1) * run : nitems;
    step = W;
    return first < last;
}

// Sums a work-group's per-thread partials and stores them in its slot of one mesh's partials
template <int NQ>
__device__ __forceinline__ void flush_partials(double* set, double (&acc)[NQ], double* sh) {
    block_sum<NQ>(acc, sh);
    if (threadIdx.x == 0) bin_store<NQ>(set, int(xcd_logical(blockIdx.x, gridDim.x)), acc);
#pragma unroll
    for (int q = 0; q < NQ; ++q) acc[q] = 0.0;
}

// PCG iteration t, first kernel.  Each work-group takes `per` interleaved row groups.  Where its item
// list enters a mesh it computes that mesh's recurrence state (see product_state; the same values each
// time it enters it), then forms the directions and products of the mesh's groups, and adds their p.q
// into the mesh's bins when it leaves the mesh.
template <typename VR, typename MR>
__global__ __launch_bounds__(kBlk) __attribute__((amdgpu_waves_per_eu(4))) void k_pcg_spmv(const SolveDesc* __restrict__ descs,
                                                   const WorkItem* __restrict__ items, long nitems, long t,
                                                   int per) {
    long first, last, step;
    if (!item_stride(nitems, per, first, last, step)) return;
    extern __shared__ unsigned char smem_raw[];
    VR* ps = reinterpret_cast<VR*>(smem_raw);
    __shared__ double sh[3 * (kBlk / 64)];
    double acc[3] = {0, 0, 0};
    int cur = -1;
    ProductState S{};
    DirIn<VR> in{};
    gbl<VR>* pnew = nullptr;
    for (long it = first; it < last; it += step) {
        const WorkItem wi = items[it];
        const SolveDesc& d = descs[wi.mesh];
        if (wi.mesh != cur) {
            if (cur >= 0 && !S.done) flush_partials<3>(bin_set(descs[cur], t, kSetPq), acc, sh);
            cur = wi.mesh;
            S = product_state(d, wi, t);
            const bool odd = t & 1;
            in.r = G(static_cast<const double*>(d.r));
            in.dinv = G(static_cast<const VR*>(d.dinv));
            in.z = G(reinterpret_cast<const VR*>(d.z));
            in.pold = G(static_cast<const VR*>(odd ? d.p0 : d.p1));
            for (int c = 0; c < 3; ++c) in.beta[c] = VR(S.beta[c]);
            pnew = G(static_cast<VR*>(odd ? d.p1 : d.p0));
        }
        if (S.done) continue;
        if (d.gptr)
            product_staged<VR, MR>(d, wi, in, pnew, ps, acc);
        else
            product_direct<VR, MR>(d, wi, in, pnew, acc);
    }
    if (cur >= 0 && !S.done) flush_partials<3>(bin_set(descs[cur], t, kSetPq), acc, sh);
}

// PCG iteration t, second kernel.  Each work-group takes `per` consecutive row groups; per mesh it meets
// it reads the state entering the iteration and the p.q bins once (alpha = r.z / p.q per active
// column; row group 0's work-group clears the p.q bins of the next product), then advances y += alpha
// p, r -= alpha q on its rows and adds their r.z (z = D^-1 r; stored in mixed precision) and r.r into
// the bins.  In mixed precision the increment y is stored in float (the update is formed in float64):
// it feeds nothing inside the solve, and the Newton loop recomputes the residual of x + y in float64,
// which corrects its rounding at the next iteration; r stays float64.
template <typename VR, bool FOLD>
__device__ __forceinline__ void update_group(const SolveDesc& d, const WorkItem& wi, long t, const double (&al)[3],
                                             int fold, double (&acc)[6]) {
    const long i = long(wi.unit) * kBlk + threadIdx.x;
    if (i >= d.nv) return;
    const gbl<const VR>* p = G(static_cast<const VR*>((t & 1) ? d.p1 : d.p0));
    const gbl<const VR>* q = G(static_cast<const VR*>(d.q));
    gbl<VR>* y = G(static_cast<VR*>(d.y));
    gbl<double>* r = G(d.r);
    const VR di = G(static_cast<const VR*>(d.dinv))[i];
    VR pv[3], qv[3];
    double yv[3], rv[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        pv[c] = p[3 * i + c];
        qv[c] = q[3 * i + c];
        yv[c] = double(y[3 * i + c]);
        rv[c] = r[3 * i + c];
    }
    VR zv[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        yv[c] = fma(al[c], double(pv[c]), yv[c]);
        rv[c] = fma(-al[c], double(qv[c]), rv[c]);
        zv[c] = di * VR(rv[c]);
        acc[c] += rv[c] * double(zv[c]);
        acc[3 + c] += rv[c] * rv[c];
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        if constexpr (FOLD) {
            if (fold & (1 << c)) {  // wave-uniform: the same for every row of the mesh
                G(d.y64)[3 * i + c] += yv[c];
                yv[c] = 0.0;
            }
        }
        y[3 * i + c] = VR(yv[c]);
        r[3 * i + c] = rv[c];
        if constexpr (kStoredZ<VR>) G(reinterpret_cast<VR*>(d.z))[3 * i + c] = zv[c];
    }
}

template <typename VR>
__global__ __launch_bounds__(kBlk) void k_pcg_update(const SolveDesc* __restrict__ descs,
                                                     const WorkItem* __restrict__ items, long nitems, long t,
                                                     int per) {
    long first, last;
    if (!item_range(nitems, per, first, last)) return;
    __shared__ double sh[6 * (kBlk / 64)];
    __shared__ double shb[3 * (kBlk / 64)];
    double acc[6] = {0, 0, 0, 0, 0, 0};
    int cur = -1, done = 1, fold = 0;
    double al[3] = {0, 0, 0};
    for (long it = first; it < last; ++it) {
        const WorkItem wi = items[it];
        const SolveDesc& d = descs[wi.mesh];
        if (wi.mesh != cur) {
            if (cur >= 0 && !done) flush_partials<6>(bin_set(descs[cur], t, kSetRz), acc, sh);
            cur = wi.mesh;
            const PcgState* st = d.st + ((t + 1) & 1);
            double pq[3];
            bin_totals<3>(bin_set(d, t, kSetPq), d.pq_lo, d.pq_hi, pq, shb);
            done = st->done;
            fold = 0;
            for (int c = 0; c < 3; ++c) {
                al[c] = (st->active[c] && pq[c] != 0.0) ? st->rz[c] / pq[c] : 0.0;
                if (st->active[c] && st->iters[c] % kFoldIters == kFoldIters - 1) fold |= 1 << c;
            }
        }
        if (done) continue;
        if constexpr (sizeof(VR) == 4) {
            if (fold)
                update_group<VR, true>(d, wi, t, al, fold, acc);
            else
                update_group<VR, false>(d, wi, t, al, 0, acc);
        } else {
            update_group<VR, false>(d, wi, t, al, 0, acc);
        }
    }
    if (cur >= 0 && !done) flush_partials<6>(bin_set(descs[cur], t, kSetRz), acc, sh);
}

// r = -g, y = 0; r.z (z = D^-1 r) and r.r into the partials read by the first product (parity 1).  The
// first product forms p = z itself.  Launched with the update kernel's grid and walk, so that its
// partials sit in the slots the update's would.
template <typename VR>
__global__ __launch_bounds__(kBlk) void k_pcg_init(const SolveDesc* __restrict__ descs,
                                                   const WorkItem* __restrict__ items, long nitems, int per) {
    long first, last;
    if (!item_range(nitems, per, first, last)) return;
    __shared__ double sh[6 * (kBlk / 64)];
    double acc[6] = {0, 0, 0, 0, 0, 0};
    int cur = -1;
    for (long it = first; it < last; ++it) {
        const WorkItem wi = items[it];
        const SolveDesc& d = descs[wi.mesh];
        if (wi.mesh != cur) {
            if (cur >= 0) flush_partials<6>(bin_set(descs[cur], 1, kSetRz), acc, sh);
            cur = wi.mesh;
        }
        const long i = long(wi.unit) * kBlk + threadIdx.x;
        if (i >= d.nv) continue;
        const VR di = G(static_cast<const VR*>(d.dinv))[i];
        const gbl<const double>* g = G(static_cast<const double*>(d.g));
        double gi[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) gi[c] = g[3 * i + c];
        gbl<double>* r = G(d.r);
        gbl<VR>* y = G(static_cast<VR*>(d.y));
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const double ri = -gi[c];
            const VR zi = di * VR(ri);
            r[3 * i + c] = ri;
            y[3 * i + c] = VR(0);
            if constexpr (kStoredZ<VR>) G(d.y64)[3 * i + c] = 0.0;
            if constexpr (kStoredZ<VR>) G(reinterpret_cast<VR*>(d.z))[3 * i + c] = zi;
            acc[c] += ri * double(zi);
            acc[3 + c] += ri * ri;
        }
    }
    if (cur >= 0) flush_partials<6>(bin_set(descs[cur], 1, kSetRz), acc, sh);
}

// Mixed refinement, first kernel: the float part of the increment folded into its float64 part,
// y64 += y, y = 0, so that y64 holds the whole increment for the float64 product.
template <typename VR>
__global__ __launch_bounds__(kBlk) void k_pcg_fold(const SolveDesc* __restrict__ descs, const WorkItem* __restrict__ items,
                                                   long nitems) {
    const long it = xcd_logical(blockIdx.x, gridDim.x);
    if (it >= nitems) return;
    const WorkItem wi = items[it];
    const SolveDesc& d = descs[wi.mesh];
    const long i = long(wi.unit) * kBlk + threadIdx.x;
    if (i >= d.nv) return;
    gbl<VR>* y = G(static_cast<VR*>(d.y));
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        G(d.y64)[3 * i + c] += double(y[3 * i + c]);
        y[3 * i + c] = VR(0);
    }
}

// Mixed refinement, second kernel (residual replacement): the true residual of the increment,
// r = -g - (M + dt^2 K_s) y64 with the float64 matrix (zero on held coordinates), restarts the PCG; r.z
// and r.r into the partials read by the first product, as k_pcg_init does.  Launched with the update
// kernel's grid and walk.
template <typename VR>
__global__ __launch_bounds__(kBlk) void k_pcg_refine_init(const SolveDesc* __restrict__ descs,
                                                          const WorkItem* __restrict__ items, long nitems, int per) {
    long first, last;
    if (!item_range(nitems, per, first, last)) return;
    __shared__ double sh[6 * (kBlk / 64)];
    double acc[6] = {0, 0, 0, 0, 0, 0};
    int cur = -1;
    for (long it = first; it < last; ++it) {
        const WorkItem wi = items[it];
        const SolveDesc& d = descs[wi.mesh];
        if (wi.mesh != cur) {
            if (cur >= 0) flush_partials<6>(bin_set(descs[cur], 1, kSetRz), acc, sh);
            cur = wi.mesh;
        }
        const long i = long(wi.unit) * kBlk + threadIdx.x;
        if (i >= d.nv) continue;
        const VR di = G(static_cast<const VR*>(d.dinv))[i];
        const unsigned held = d.pinned[i];
        gbl<double>* r = G(d.r);
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const double ri = (held >> c & 1u) ? 0.0 : -G(static_cast<const double*>(d.g))[3 * i + c] - G(d.rq)[3 * i + c];
            const VR zi = di * VR(ri);
            r[3 * i + c] = ri;
            if constexpr (kStoredZ<VR>) G(reinterpret_cast<VR*>(d.z))[3 * i + c] = zi;
            acc[c] += ri * double(zi);
            acc[3 + c] += ri * ri;
        }
    }
    if (cur >= 0) flush_partials<6>(bin_set(descs[cur], 1, kSetRz), acc, sh);
}

// x += s y (Newton update); s = 1 unless a quasi-static increment limit set it
template <typename VR>
__global__ __launch_bounds__(kBlk) void k_newton_update(const SolveDesc* __restrict__ descs, const WorkItem* __restrict__ items,
                                long nitems) {
    WorkItem wi;
    if (!work_item(items, nitems, wi)) return;
    const SolveDesc& d = descs[wi.mesh];
    long i = long(wi.unit) * kBlk + threadIdx.x;
    if (i >= d.nv) return;
    const VR* y = static_cast<const VR*>(d.y);
    const double sc = d.ustep ? *d.ustep : 1.0;
    for (int c = 0; c < 3; ++c) {
        double yi = double(y[3 * i + c]);
        if constexpr (sizeof(VR) == 4) yi += d.y64[3 * i + c];
        d.x[3 * i + c] += sc * yi;
    }
}

// largest |y| entry of each row group, into the partials
template <typename VR>
__global__ __launch_bounds__(kBlk) void k_absmax(const SolveDesc* __restrict__ descs, const WorkItem* __restrict__ items,
                                                 long nitems) {
    WorkItem wi;
    if (!work_item(items, nitems, wi)) return;
    const SolveDesc& d = descs[wi.mesh];
    long i = long(wi.unit) * kBlk + threadIdx.x;
    double m = 0.0;
    if (i < d.nv) {
        const VR* y = static_cast<const VR*>(d.y);
        for (int c = 0; c < 3; ++c) {
            double yi = double(y[3 * i + c]);
            if constexpr (sizeof(VR) == 4) yi += d.y64[3 * i + c];
            m = fmax(m, fabs(yi));
        }
    }
    __shared__ double sh[kBlk];
    sh[threadIdx.x] = m;
    __syncthreads();
    for (int w = kBlk / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) sh[threadIdx.x] = fmax(sh[threadIdx.x], sh[threadIdx.x + w]);
        __syncthreads();
    }
    if (threadIdx.x == 0) d.part[wi.unit] = sh[0];
}

// incremental displacement limit (eq 64's eps_u): s = eps_u / max|y| when that is below one
__global__ __launch_bounds__(kRedBlk) void k_fin_step_limit(const SolveDesc* __restrict__ descs,
                                                            const int32_t* __restrict__ meshes) {
    const SolveDesc& d = descs[meshes[blockIdx.x]];
    double m = 0.0;
    for (long b = threadIdx.x; b < d.ngroups; b += kRedBlk) m = fmax(m, d.part[b]);
    __shared__ double sh[kRedBlk];
    sh[threadIdx.x] = m;
    __syncthreads();
    for (int w = kRedBlk / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) sh[threadIdx.x] = fmax(sh[threadIdx.x], sh[threadIdx.x + w]);
        __syncthreads();
    }
    if (threadIdx.x == 0 && d.ustep) *d.ustep = sh[0] > d.eps_u ? d.eps_u / sh[0] : 1.0;
}

__global__ __launch_bounds__(kBlk) void k_velocity(const SolveDesc* __restrict__ descs, const WorkItem* __restrict__ items, long nitems) {
    WorkItem wi;
    if (!work_item(items, nitems, wi)) return;
    const SolveDesc& d = descs[wi.mesh];
    long i = long(wi.unit) * kBlk + threadIdx.x;
    if (i >= d.nv) return;
    for (int c = 0; c < 3; ++c) d.v[3 * i + c] = (d.x[3 * i + c] - d.xt[3 * i + c]) / d.dt;
}

// lumped mass rho h sum(A_T)/3 from the rest triangles around each vertex, in ascending triangle order
__global__ void k_mass_rows(const double* __restrict__ X, const int32_t* __restrict__ tris,
                            const int64_t* __restrict__ vt_ptr, const int64_t* __restrict__ vt, long nv,
                            double rho_h, double* __restrict__ mass) {
    const long v = blockIdx.x * long(blockDim.x) + threadIdx.x;
    if (v >= nv) return;
    double m = 0.0;
    for (int64_t e = vt_ptr[v]; e < vt_ptr[v + 1]; ++e) {
        const long t = long(vt[e] >> 3);
        const V3<double> xa = load3(X, tris[3 * t]);
        m += rho_h * 0.5 * norm(cross(load3(X, tris[3 * t + 1]) - xa, load3(X, tris[3 * t + 2]) - xa)) / 3.0;
    }
    mass[v] = m;
}


}  // namespace

}  // namespace shell
