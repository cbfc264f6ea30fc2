// Implicit Euler step (Sec. 5): x_hat = x^t + dt v^t + dt^2 g, Newton iterations on the incremental
// potential (eq 62 without contact) against the constant matrix A = M + dt^2 K_s (x) I3, each solve
// by three Jacobi-PCG recurrences (x, y, z coordinates decouple exactly because A is A_s (x) I3)
// sharing one sparse product, then v = (x^{t+1} - x^t)/dt.
//
// Every scalar of the recurrences lives on the device: each reduction kernel writes per-work-group
// partial sums and a one-work-group finalize kernel sums them in a fixed order and updates alpha, beta
// and the per-column activity flags.  (Kernel boundaries make the partials visible across the XCDs'
// private L2 caches; an in-kernel device-scope fence per work-group would write back the L2 each time.)
// Kernels of converged solves return at once, so the host launches iterations in chunks and reads one
// flag per chunk.
//
// Precision: FP64 throughout, or mixed: float32 matrix values, Jacobi diagonal and the vectors p, q,
// z; float64 solution y, residual r, all dot products and the Newton residual.
#include <cmath>
#include <cstring>

#include "devmath.hpp"
#include "internal.hpp"
#include "spmv.hpp"

struct PcgState {
    double rz[3], rr[3], tol2[3], alpha[3], beta[3];
    double gsq;
    int32_t iters[3], target[3], active[3];
    int32_t done, budget, replay, nonfinite;
};

namespace shell {

namespace {

constexpr int kBlk = 256;
constexpr int kMaxPart = 8;  // partial quantities per work-group (buffer sized kMaxPart * groups)

constexpr int kRedBlk = 512;  // finalize kernels: one work-group

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

__global__ void k_predictor(double* __restrict__ x, const double* __restrict__ v, double* __restrict__ xt,
                            double* __restrict__ xhat, const uint8_t* __restrict__ pinned, long nv, double dt,
                            double g0, double g1, double g2) {
    long i = blockIdx.x * long(blockDim.x) + threadIdx.x;
    if (i >= nv) return;
    const double gr[3] = {g0, g1, g2};
    bool pin = pinned[i];
    for (int d = 0; d < 3; ++d) {
        double xi = x[3 * i + d];
        xt[3 * i + d] = xi;
        double xh = pin ? xi : xi + dt * v[3 * i + d] + dt * dt * gr[d];
        xhat[3 * i + d] = xh;
        x[3 * i + d] = xh;
    }
}

template <typename FR>
__global__ void k_residual(const double* __restrict__ x, const double* __restrict__ xhat, const FR* __restrict__ f,
                           const double* __restrict__ mass, const uint8_t* __restrict__ pinned, long nv, double dt2,
                           double* __restrict__ g, double* __restrict__ part) {
    long blk = xcd_logical(blockIdx.x, gridDim.x);
    long ngroups = (nv + kBlk - 1) / kBlk;
    if (blk >= ngroups) return;
    long i = blk * kBlk + threadIdx.x;
    double acc[1] = {0.0};
    if (i < nv) {
        bool pin = pinned[i];
        double m = mass[i];
        for (int d = 0; d < 3; ++d) {
            double gi = pin ? 0.0 : m * (x[3 * i + d] - xhat[3 * i + d]) - dt2 * double(f[3 * i + d]);
            g[3 * i + d] = gi;
            acc[0] += gi * gi;
        }
    }
    __shared__ double sh[kBlk / 64];
    block_sum<1>(acc, sh);
    if (threadIdx.x == 0) part[blk] = acc[0];
}

__global__ void k_fin_residual(const double* __restrict__ part, long ngroups, PcgState* __restrict__ st) {
    double tot[1];
    reduce_partials<1>(part, ngroups, tot);
    if (threadIdx.x == 0) {
        st->gsq = tot[0];
        st->nonfinite = !isfinite(tot[0]);
    }
}

// r = -g, y = 0, z = D^-1 r, p = z; column norms and tolerances
template <typename VR>
__global__ void k_pcg_init(const double* __restrict__ g, const VR* __restrict__ dinv, long nv,
                           double* __restrict__ y, double* __restrict__ r, VR* __restrict__ z, VR* __restrict__ p,
                           double* __restrict__ part) {
    long blk = xcd_logical(blockIdx.x, gridDim.x);
    long ngroups = (nv + kBlk - 1) / kBlk;
    if (blk >= ngroups) return;
    long i = blk * kBlk + threadIdx.x;
    double acc[6] = {0, 0, 0, 0, 0, 0};
    if (i < nv) {
        VR di = dinv[i];
        for (int d = 0; d < 3; ++d) {
            double ri = -g[3 * i + d];
            VR zi = di * VR(ri);
            r[3 * i + d] = ri;
            y[3 * i + d] = 0.0;
            z[3 * i + d] = zi;
            p[3 * i + d] = zi;
            acc[d] += ri * double(zi);
            acc[3 + d] += ri * ri;
        }
    }
    __shared__ double sh[6 * (kBlk / 64)];
    block_sum<6>(acc, sh);
    if (threadIdx.x == 0)
        for (int q = 0; q < 6; ++q) part[q * ngroups + blk] = acc[q];
}

__global__ void k_fin_init(const double* __restrict__ part, long ngroups, PcgState* __restrict__ st, double rtol2,
                           int replay, int t0, int t1, int t2) {
    double tot[6];
    reduce_partials<6>(part, ngroups, tot);
    if (threadIdx.x == 0) {
        const int tg[3] = {t0, t1, t2};
        int any = 0;
        for (int d = 0; d < 3; ++d) {
            st->rz[d] = tot[d];
            st->rr[d] = tot[3 + d];
            st->tol2[d] = rtol2 * tot[3 + d];
            st->alpha[d] = 0.0;
            st->beta[d] = 0.0;
            st->iters[d] = 0;
            st->target[d] = tg[d];
            st->active[d] = (0 < tg[d]) && (replay || tot[3 + d] > st->tol2[d]);
            any |= st->active[d];
        }
        st->done = !any;
        st->budget = 0;
        st->replay = replay;
        st->nonfinite = 0;
    }
}

// q = (M + dt^2 K_s) p on the free rows (pinned rows 0); alpha = r.z / p.q per active column
template <typename VR, typename MR>
__global__ void k_pcg_spmv(const int32_t* __restrict__ scol, const MR* __restrict__ val,
                           const int64_t* __restrict__ sptr, const int32_t* __restrict__ width,
                           const double* __restrict__ mass, const uint8_t* __restrict__ pinned, long nv, MR dt2,
                           const VR* __restrict__ p, VR* __restrict__ q, double* __restrict__ part,
                           const PcgState* __restrict__ st) {
    if (st->done) return;
    long blk = xcd_logical(blockIdx.x, gridDim.x);
    long ngroups = (nv + kBlk - 1) / kBlk;
    if (blk >= ngroups) return;
    long i = blk * kBlk + threadIdx.x;
    double acc[3] = {0, 0, 0};
    if (i < nv) {
        MR ax, ay, az;
        sell_row_product<MR, VR>(scol, val, sptr, width, i, p, ax, ay, az);
        VR px = p[3 * i], py = p[3 * i + 1], pz = p[3 * i + 2];
        VR qx = 0, qy = 0, qz = 0;
        if (!pinned[i]) {
            MR m = MR(mass[i]);
            qx = VR(fma(m, MR(px), dt2 * ax));
            qy = VR(fma(m, MR(py), dt2 * ay));
            qz = VR(fma(m, MR(pz), dt2 * az));
        }
        q[3 * i] = qx;
        q[3 * i + 1] = qy;
        q[3 * i + 2] = qz;
        acc[0] = double(px) * double(qx);
        acc[1] = double(py) * double(qy);
        acc[2] = double(pz) * double(qz);
    }
    __shared__ double sh[3 * (kBlk / 64)];
    block_sum<3>(acc, sh);
    if (threadIdx.x == 0)
        for (int q3 = 0; q3 < 3; ++q3) part[q3 * ngroups + blk] = acc[q3];
}

__global__ void k_fin_alpha(const double* __restrict__ part, long ngroups, PcgState* __restrict__ st) {
    if (st->done) return;
    double tot[3];
    reduce_partials<3>(part, ngroups, tot);
    if (threadIdx.x == 0)
        for (int d = 0; d < 3; ++d) st->alpha[d] = (st->active[d] && tot[d] != 0.0) ? st->rz[d] / tot[d] : 0.0;
}

// y += alpha p, r -= alpha q, z = D^-1 r; new r.z, r.r; beta and activity per column
template <typename VR>
__global__ void k_pcg_update(const VR* __restrict__ p, const VR* __restrict__ q, const VR* __restrict__ dinv, long nv,
                             double* __restrict__ y, double* __restrict__ r, VR* __restrict__ z,
                             double* __restrict__ part, const PcgState* __restrict__ st) {
    if (st->done) return;
    long blk = xcd_logical(blockIdx.x, gridDim.x);
    long ngroups = (nv + kBlk - 1) / kBlk;
    if (blk >= ngroups) return;
    long i = blk * kBlk + threadIdx.x;
    const double al[3] = {st->alpha[0], st->alpha[1], st->alpha[2]};
    double acc[6] = {0, 0, 0, 0, 0, 0};
    if (i < nv) {
        VR di = dinv[i];
        for (int d = 0; d < 3; ++d) {
            double yi = fma(al[d], double(p[3 * i + d]), y[3 * i + d]);
            double ri = fma(-al[d], double(q[3 * i + d]), r[3 * i + d]);
            VR zi = di * VR(ri);
            y[3 * i + d] = yi;
            r[3 * i + d] = ri;
            z[3 * i + d] = zi;
            acc[d] += ri * double(zi);
            acc[3 + d] += ri * ri;
        }
    }
    __shared__ double sh[6 * (kBlk / 64)];
    block_sum<6>(acc, sh);
    if (threadIdx.x == 0)
        for (int q6 = 0; q6 < 6; ++q6) part[q6 * ngroups + blk] = acc[q6];
}

__global__ void k_fin_beta(const double* __restrict__ part, long ngroups, PcgState* __restrict__ st) {
    if (st->done) return;
    double tot[6];
    reduce_partials<6>(part, ngroups, tot);
    if (threadIdx.x == 0) {
        int any = 0;
        for (int d = 0; d < 3; ++d) {
            if (st->active[d]) {
                st->beta[d] = st->rz[d] != 0.0 ? tot[d] / st->rz[d] : 0.0;
                st->rz[d] = tot[d];
                st->rr[d] = tot[3 + d];
                st->iters[d] += 1;
                bool more = st->replay || tot[3 + d] > st->tol2[d];
                if (!st->replay && st->iters[d] >= st->target[d] && more) st->budget = 1;
                st->active[d] = (st->iters[d] < st->target[d]) && more;
                if (!isfinite(tot[3 + d])) {
                    st->nonfinite = 1;
                    st->active[d] = 0;
                }
            } else {
                st->beta[d] = 0.0;
            }
            any |= st->active[d];
        }
        st->done = !any;
    }
}

template <typename VR>
__global__ void k_pcg_direction(const VR* __restrict__ z, VR* __restrict__ p, long nv,
                                const PcgState* __restrict__ st) {
    if (st->done) return;
    long i = blockIdx.x * long(blockDim.x) + threadIdx.x;
    if (i >= nv) return;
    for (int d = 0; d < 3; ++d) {
        VR b = VR(st->beta[d]);
        p[3 * i + d] = fma(b, p[3 * i + d], z[3 * i + d]);
    }
}

__global__ void k_add(double* __restrict__ x, const double* __restrict__ y, long n) {
    long i = blockIdx.x * long(blockDim.x) + threadIdx.x;
    if (i < n) x[i] += y[i];
}

__global__ void k_velocity(const double* __restrict__ x, const double* __restrict__ xt, double* __restrict__ v,
                           long n, double dt) {
    long i = blockIdx.x * long(blockDim.x) + threadIdx.x;
    if (i < n) v[i] = (x[i] - xt[i]) / dt;
}

template <typename VR>
__global__ void k_dinv(const double* __restrict__ mass, const double* __restrict__ kdiag,
                       const uint8_t* __restrict__ pinned, long nv, double dt2, VR* __restrict__ dinv) {
    long i = blockIdx.x * long(blockDim.x) + threadIdx.x;
    if (i < nv) dinv[i] = pinned[i] ? VR(0) : VR(1.0 / (mass[i] + dt2 * kdiag[i]));
}

// lumped mass rho h sum(A_T)/3 from the rest triangles
__global__ void k_mass(const double* __restrict__ X, const int32_t* __restrict__ tris, long nt, double rho_h,
                       double* __restrict__ mass) {
    long t = blockIdx.x * long(blockDim.x) + threadIdx.x;
    if (t >= nt) return;
    int a = tris[3 * t], b = tris[3 * t + 1], c = tris[3 * t + 2];
    V3<double> xa = load3(X, a);
    double third = rho_h * 0.5 * norm(cross(load3(X, b) - xa, load3(X, c) - xa)) / 3.0;
    atomicAdd(mass + a, third);
    atomicAdd(mass + b, third);
    atomicAdd(mass + c, third);
}

__global__ void k_zero(double* __restrict__ p, long n) {
    long i = blockIdx.x * long(blockDim.x) + threadIdx.x;
    if (i < n) p[i] = 0.0;
}

inline long blocks(long n) { return (n + kBlk - 1) / kBlk; }

template <typename VR, typename MR>
void pcg_iterations(shell_sim_s& sim, int count, double dt2, hipStream_t s) {
    shell_hessian_s& h = *sim.h;
    const long nv = sim.nv;
    long grid = xcd_grid(blocks(nv));
    PcgState* st = reinterpret_cast<PcgState*>(sim.state.p);
    const MR* val = std::is_same<MR, float>::value ? reinterpret_cast<const MR*>(h.valf.p)
                                                    : reinterpret_cast<const MR*>(h.val.p);
    VR* p = reinterpret_cast<VR*>(sim.p.p);
    VR* q = reinterpret_cast<VR*>(sim.q.p);
    VR* z = reinterpret_cast<VR*>(sim.z.p);
    const VR* dinv = reinterpret_cast<const VR*>(sim.dinv.p);
    const long ng = blocks(nv);
    for (int it = 0; it < count; ++it) {
        k_pcg_spmv<VR, MR><<<grid, kBlk, 0, s>>>(h.scol.p, val, h.sptr.p, h.width.p, sim.mass.p, sim.pinned.p, nv,
                                                 MR(dt2), p, q, sim.partials.p, st);
        k_fin_alpha<<<1, kRedBlk, 0, s>>>(sim.partials.p, ng, st);
        k_pcg_update<VR><<<grid, kBlk, 0, s>>>(p, q, dinv, nv, sim.y.p, sim.r.p, z, sim.partials.p, st);
        k_fin_beta<<<1, kRedBlk, 0, s>>>(sim.partials.p, ng, st);
        k_pcg_direction<VR><<<blocks(nv), kBlk, 0, s>>>(z, p, nv, st);
    }
    SHELL_HIP(hipGetLastError());
}

void read_state(shell_sim_s& sim, hipStream_t s) {
    SHELL_HIP(hipMemcpyAsync(sim.state_host, sim.state.p, sizeof(PcgState), hipMemcpyDeviceToHost, s));
    SHELL_HIP(hipStreamSynchronize(s));
}

template <typename VR, typename MR>
shell_status_t step_impl(shell_sim_s& sim, const shell_step_params_t& prm, hipStream_t s) {
    shell_stencils_s& st = *sim.st;
    const long nv = sim.nv;
    const long n3 = 3 * nv;
    const double dt = prm.dt, dt2 = dt * dt;
    PcgState* dst = reinterpret_cast<PcgState*>(sim.state.p);
    const PcgState* hst = reinterpret_cast<const PcgState*>(sim.state_host);
    shell_step_stats_t stats{};
    stats.status = SHELL_OK;
    if (nv == 0) {
        sim.stats = stats;
        sim.step++;
        return SHELL_OK;
    }
    if (sim.dinv_dt != dt) {
        k_dinv<VR><<<blocks(nv), kBlk, 0, s>>>(sim.mass.p, sim.h->kdiag.p, sim.pinned.p, nv, dt2,
                                              reinterpret_cast<VR*>(sim.dinv.p));
        sim.dinv_dt = dt;
    }
    k_predictor<<<blocks(nv), kBlk, 0, s>>>(sim.x.p, sim.v.p, sim.xt.p, sim.xhat.p, sim.pinned.p, nv, dt,
                                            prm.gravity[0], prm.gravity[1], prm.gravity[2]);
    SHELL_HIP(hipGetLastError());
    const long rgrid = xcd_grid(blocks(nv));
    const int first_chunk = prm.chunk > 0 ? prm.chunk : 8;
    const int max_chunk = prm.chunk > 0 ? prm.chunk : 128;
    bool budget = false;
    double gn0 = 0.0, gn = 0.0;
    for (int k = 0;; ++k) {
        launch_forces(st, sim.x.p, sim.f.p, nullptr, s);
        k_residual<VR><<<rgrid, kBlk, 0, s>>>(sim.x.p, sim.xhat.p, reinterpret_cast<const VR*>(sim.f.p), sim.mass.p,
                                             sim.pinned.p, nv, dt2, sim.g.p, sim.partials.p);
        k_fin_residual<<<1, kRedBlk, 0, s>>>(sim.partials.p, blocks(nv), dst);
        SHELL_HIP(hipGetLastError());
        read_state(sim, s);
        if (hst->nonfinite) {
            stats.status = SHELL_E_NONFINITE;
            break;
        }
        gn = std::sqrt(hst->gsq);
        if (k == 0) gn0 = gn;
        if (gn0 == 0.0 || (k > 0 && gn <= prm.newton_rtol * gn0) || k == prm.max_newton) break;
        int tg[3];
        for (int d = 0; d < 3; ++d)
            tg[d] = prm.mode == SHELL_PCG_REPLAY ? prm.replay_counts[3 * k + d] : prm.max_pcg;
        k_pcg_init<VR><<<rgrid, kBlk, 0, s>>>(sim.g.p, reinterpret_cast<const VR*>(sim.dinv.p), nv, sim.y.p, sim.r.p,
                                             reinterpret_cast<VR*>(sim.z.p), reinterpret_cast<VR*>(sim.p.p),
                                             sim.partials.p);
        k_fin_init<<<1, kRedBlk, 0, s>>>(sim.partials.p, blocks(nv), dst, prm.pcg_rtol * prm.pcg_rtol,
                                         prm.mode == SHELL_PCG_REPLAY, tg[0], tg[1], tg[2]);
        SHELL_HIP(hipGetLastError());
        if (prm.mode == SHELL_PCG_REPLAY) {
            int most = std::max(tg[0], std::max(tg[1], tg[2]));
            pcg_iterations<VR, MR>(sim, most, dt2, s);
            read_state(sim, s);
        } else {
            read_state(sim, s);
            int chunk = first_chunk;
            while (!hst->done) {
                pcg_iterations<VR, MR>(sim, chunk, dt2, s);
                read_state(sim, s);
                chunk = std::min(2 * chunk, max_chunk);
            }
        }
        if (hst->nonfinite) {
            stats.status = SHELL_E_NONFINITE;
            break;
        }
        budget |= hst->budget != 0;
        for (int d = 0; d < 3; ++d) {
            stats.counts[k][d] = hst->iters[d];
            stats.pcg_total += hst->iters[d];
        }
        k_add<<<blocks(n3), kBlk, 0, s>>>(sim.x.p, sim.y.p, n3);
        SHELL_HIP(hipGetLastError());
        stats.newton_iters++;
    }
    k_velocity<<<blocks(n3), kBlk, 0, s>>>(sim.x.p, sim.xt.p, sim.v.p, n3, dt);
    SHELL_HIP(hipGetLastError());
    stats.grad_norm0 = gn0;
    stats.grad_norm = gn;
    if (stats.status == SHELL_OK && budget) stats.status = SHELL_E_BUDGET;
    sim.stats = stats;
    sim.step++;
    sim.last_stream = s;
    return shell_status_t(stats.status);
}

}  // namespace

void sim_alloc(shell_sim_s& sim) {
    const long nv = sim.nv, n3 = 3 * nv;
    for (auto* a : {&sim.x, &sim.v, &sim.xt, &sim.xhat, &sim.g, &sim.y, &sim.r, &sim.f, &sim.z, &sim.p, &sim.q})
        a->alloc(size_t(std::max(n3, 1L)));
    sim.mass.alloc(size_t(std::max(nv, 1L)));
    sim.dinv.alloc(size_t(std::max(nv, 1L)));
    sim.pinned.alloc(size_t(std::max(nv, 1L)));
    sim.partials.alloc(size_t(kMaxPart * std::max(blocks(nv), 1L) + kMaxPart));
    sim.state.alloc(sizeof(PcgState));
    SHELL_HIP(hipMemset(sim.state.p, 0, sizeof(PcgState)));
    SHELL_HIP(hipHostMalloc(reinterpret_cast<void**>(&sim.state_host), sizeof(PcgState)));
    std::memset(sim.state_host, 0, sizeof(PcgState));
}

void sim_mass(shell_sim_s& sim, hipStream_t s) {
    shell_stencils_s& st = *sim.st;
    if (!sim.nv) return;
    k_zero<<<blocks(sim.nv), kBlk, 0, s>>>(sim.mass.p, sim.nv);
    if (st.nt) k_mass<<<blocks(st.nt), kBlk, 0, s>>>(st.X.p, st.tris.p, st.nt, st.density * st.thickness, sim.mass.p);
    SHELL_HIP(hipGetLastError());
}

namespace {

template <typename VR, typename MR>
void time_impl(shell_sim_s& sim, double dt, int reps, shell_kernel_times_t& out, hipStream_t s) {
    shell_stencils_s& st = *sim.st;
    shell_hessian_s& h = *sim.h;
    const long nv = sim.nv;
    const double dt2 = dt * dt;
    PcgState* dst = reinterpret_cast<PcgState*>(sim.state.p);
    const long grid = xcd_grid(blocks(nv));
    const MR* val = std::is_same<MR, float>::value ? reinterpret_cast<const MR*>(h.valf.p)
                                                    : reinterpret_cast<const MR*>(h.val.p);
    VR* p = reinterpret_cast<VR*>(sim.p.p);
    VR* q = reinterpret_cast<VR*>(sim.q.p);
    VR* z = reinterpret_cast<VR*>(sim.z.p);
    const VR* dinv = reinterpret_cast<const VR*>(sim.dinv.p);
    if (sim.dinv_dt != dt) {
        k_dinv<VR><<<blocks(nv), kBlk, 0, s>>>(sim.mass.p, h.kdiag.p, sim.pinned.p, nv, dt2, reinterpret_cast<VR*>(sim.dinv.p));
        sim.dinv_dt = dt;
    }
    hipEvent_t e0, e1;
    SHELL_HIP(hipEventCreate(&e0));
    SHELL_HIP(hipEventCreate(&e1));
    auto init = [&]() {
        // a residual from the current forces, then an always-active recurrence
        launch_forces(st, sim.x.p, sim.f.p, nullptr, s);
        k_residual<VR><<<grid, kBlk, 0, s>>>(sim.x.p, sim.x.p, reinterpret_cast<const VR*>(sim.f.p), sim.mass.p,
                                             sim.pinned.p, nv, dt2, sim.g.p, sim.partials.p);
        k_pcg_init<VR><<<grid, kBlk, 0, s>>>(sim.g.p, dinv, nv, sim.y.p, sim.r.p, z, p, sim.partials.p);
        k_fin_init<<<1, kRedBlk, 0, s>>>(sim.partials.p, blocks(nv), dst, 0.0, 1, 1 << 30, 1 << 30, 1 << 30);
        k_pcg_spmv<VR, MR><<<grid, kBlk, 0, s>>>(h.scol.p, val, h.sptr.p, h.width.p, sim.mass.p, sim.pinned.p, nv,
                                                 MR(dt2), p, q, sim.partials.p, dst);
        k_fin_alpha<<<1, kRedBlk, 0, s>>>(sim.partials.p, blocks(nv), dst);
        SHELL_HIP(hipGetLastError());
    };
    auto timed = [&](auto&& launch) {
        launch();  // warm
        SHELL_HIP(hipEventRecord(e0, s));
        for (int i = 0; i < reps; ++i) launch();
        SHELL_HIP(hipEventRecord(e1, s));
        SHELL_HIP(hipEventSynchronize(e1));
        float ms = 0.f;
        SHELL_HIP(hipEventElapsedTime(&ms, e0, e1));
        return double(ms) / reps;
    };
    out.reps = reps;
    out.force_ms = timed([&] { launch_forces(st, sim.x.p, sim.f.p, nullptr, s); });
    init();
    out.spmv_ms = timed([&] {
        k_pcg_spmv<VR, MR><<<grid, kBlk, 0, s>>>(h.scol.p, val, h.sptr.p, h.width.p, sim.mass.p, sim.pinned.p, nv,
                                                 MR(dt2), p, q, sim.partials.p, dst);
    });
    init();
    out.update_ms = timed([&] {
        k_pcg_update<VR><<<grid, kBlk, 0, s>>>(p, q, dinv, nv, sim.y.p, sim.r.p, z, sim.partials.p, dst);
    });
    init();
    out.direction_ms = timed([&] { k_pcg_direction<VR><<<blocks(nv), kBlk, 0, s>>>(z, p, nv, dst); });
    SHELL_HIP(hipGetLastError());
    SHELL_HIP(hipStreamSynchronize(s));
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
}

}  // namespace

void sim_time_kernels(shell_sim_s& sim, double dt, int reps, shell_kernel_times_t& out, hipStream_t s) {
    if (sim.nv == 0) return;
    if (sim.st->precision == SHELL_PREC_MIXED)
        time_impl<float, float>(sim, dt, reps, out, s);
    else
        time_impl<double, double>(sim, dt, reps, out, s);
}

shell_status_t sim_step(shell_sim_s& sim, const shell_step_params_t& p, hipStream_t s) {
    if (sim.st->precision == SHELL_PREC_MIXED) return step_impl<float, float>(sim, p, s);
    return step_impl<double, double>(sim, p, s);
}

}  // namespace shell
