// Implicit Euler step (Sec. 5): x_hat = x^t + dt v^t + dt^2 g, Newton iterations on the incremental
// potential (eq 62 without contact) against the constant matrix A = M + dt^2 K_s (x) I3, each solve
// by three Jacobi-PCG recurrences (x, y, z coordinates decouple exactly because A is A_s (x) I3)
// sharing one sparse product, then v = (x^{t+1} - x^t)/dt.
//
// Every kernel takes an array of per-mesh descriptors and a list of (mesh, 512-row group) work items,
// so one launch per phase advances any set of meshes (a single simulation is a set of one).
//
// Every scalar of the recurrences lives on the device.  A PCG iteration is two streaming kernels: the
// product kernel advances the recurrence state by the previous update (beta, activity flags, counts),
// forms the new search direction p = z + beta p_old for its row group's distinct columns while staging
// them in LDS, writes p for its own rows and q = A p; the update kernel computes alpha and advances y
// and r.  The dot products reach the next kernel as per-work-group partials in fixed slots, summed in
// a fixed order by every work-group that needs them (see the partials in pcg_kernels.hpp), so no
// reduction kernel sits between them and the result does not depend on scheduling.  p alternates
// between two buffers because other row groups still read the previous direction while it is
// rewritten.  Kernels of converged meshes return at once, so the host launches iterations in chunks and
// reads the flags once per chunk.
//
// Precision: FP64 throughout, or mixed: float32 matrix values (applied in difference form), Jacobi
// diagonal and the vectors p, q, z and f; the increment y in float32 folded into float64 every 16
// iterations; float64 residual r, all dot products and the Newton residual.
#include <algorithm>
#include <cfloat>
#include <cmath>
#include <cstring>

#include <hip/hip_ext.h>

#include "devmath.hpp"
#include "internal.hpp"
#include "pcg_kernels.hpp"

namespace shell {

hipEvent_t StepProfiler::take() {
    if (pool.empty()) {
        hipEvent_t e;
        SHELL_HIP(hipEventCreate(&e));
        return e;
    }
    hipEvent_t e = pool.back();
    pool.pop_back();
    return e;
}

void StepProfiler::drain() {
    for (const Sample& e : pending) {
        float t = 0.f;
        SHELL_HIP(hipEventElapsedTime(&t, e.a, e.b));
        ms[e.phase] += double(t);
        count[e.phase] += 1;
        pool.push_back(e.a);
        pool.push_back(e.b);
    }
    pending.clear();
}

void StepProfiler::reset() {
    for (int k = 0; k < SHELL_NUM_PHASES; ++k) {
        ms[k] = 0.0;
        count[k] = 0;
    }
    counter = 0;
}

GraphCache::~GraphCache() {
    RuntimeLock lk(runtime_mutex());
    for (auto& e : entries) (void)hipGraphExecDestroy(e.second);
    if (capture) (void)hipStreamDestroy(capture);
}

StepProfiler::~StepProfiler() {
    for (const Sample& e : pending) {
        pool.push_back(e.a);
        pool.push_back(e.b);
    }
    for (hipEvent_t e : pool) (void)hipEventDestroy(e);
}

namespace {

// Device views of one launch set: the row-group items and, per model, the tile items.
struct Launch {
    const SolveDesc* sdesc;
    const ForceDesc* fdesc;
    const WorkItem* rows;
    long nrows;
    const WorkItem* tiles[6];
    long ntiles[6];
    const int32_t* meshes;
    int nmeshes;
    int precision;
    int lds_T;
    size_t lds_spmv;  // bytes of staged p entries per row group (largest over the meshes)
    int per;          // row groups per work-group of the PCG kernels
    long pcg_grid;    // their grid
    int per_u;        // row groups per work-group of the update kernel
    long upd_grid;    // its grid
};

#ifndef SHELL_PCG_WORKGROUPS
#define SHELL_PCG_WORKGROUPS 512  // work-groups of a PCG kernel: two of 512 threads resident per CU
#endif
// The update kernel's work-groups take per * MERGE / SPLIT row groups each when the launch holds one mesh
// (per otherwise).  Its work per row is short, so its fixed cost per work-group (reading the bins and
// the state, adding its partial sums) weighs more: on a 1M-vertex mesh twice the row groups per
// work-group (one work-group per CU) measured 1% faster, half as many 5% slower and a quarter 29%
// slower.  With many meshes longer walks cross more meshes, each crossing a re-read of bins and state:
// twice the groups made the 64-mesh batch's update 19% slower.
#ifndef SHELL_UPDATE_SPLIT
#define SHELL_UPDATE_SPLIT 1
#endif
#ifndef SHELL_UPDATE_MERGE
#define SHELL_UPDATE_MERGE 2
#endif

// Sampled timing: `launch(start, stop)` launches its kernel(s) with hipExtLaunchKernelGGL, which writes
// the dispatch's own begin and end times into the events (the times a kernel trace reports); both are
// null when the launch is not sampled.
template <typename F>
void timed_launch(StepProfiler* prof, bool sample, int phase, hipStream_t s, F&& launch) {
    if (!sample) {
        launch(hipEvent_t(nullptr), hipEvent_t(nullptr));
        return;
    }
    StepProfiler::Sample e{phase, prof->take(), prof->take()};
    launch(e.a, e.b);
    prof->pending.push_back(e);
}

// `count` PCG iterations after product t: (update t, product t + 1) pairs; returns the last product's t.
// The state the host reads afterwards is parity t + 1.
template <typename VR, typename MR>
long pcg_chunk(const Launch& L, long t, int count, hipStream_t s, StepProfiler* prof) {
    const long grid = L.pcg_grid;
    for (int it = 0; it < count; ++it, ++t) {
        const bool smp = prof && prof->sample_iteration();
        if (!smp) {  // plain launches (also the form recorded into graphs)
            k_pcg_update<VR><<<L.upd_grid, kBlk, 0, s>>>(L.sdesc, L.rows, L.nrows, t, L.per_u);
            k_pcg_spmv<VR, MR><<<grid, kBlk, L.lds_spmv, s>>>(L.sdesc, L.rows, L.nrows, t + 1, L.per);
            continue;
        }
        timed_launch(prof, true, SHELL_PHASE_UPDATE, s, [&](hipEvent_t e0, hipEvent_t e1) {
            hipExtLaunchKernelGGL(k_pcg_update<VR>, dim3(unsigned(L.upd_grid)), dim3(kBlk), 0, s, e0, e1, 0, L.sdesc,
                                  L.rows, L.nrows, t, L.per_u);
        });
        timed_launch(prof, true, SHELL_PHASE_PRODUCT, s, [&](hipEvent_t e0, hipEvent_t e1) {
            hipExtLaunchKernelGGL(k_pcg_spmv<VR, MR>, dim3(unsigned(grid)), dim3(kBlk), uint32_t(L.lds_spmv), s, e0,
                                  e1, 0, L.sdesc, L.rows, L.nrows, t + 1, L.per);
        });
    }
    SHELL_HIP(hipGetLastError());
    return t;
}

constexpr int kMinGraphChunk = 8, kMaxGraphChunk = 128, kMaxGraphs = 32;

// `count` PCG iterations after product t through the batch's graph cache: power-of-two pieces of
// 8..128 iterations are replayed from captured graphs (captured on first use on a private stream),
// a remainder below 8 is launched directly.  A captured piece is valid for any start with the same
// parity: the kernels use t only for buffer parity and t > 0.
template <typename VR, typename MR>
long pcg_iterations(shell_batch_s& b, const Launch& L, long t, int count, hipStream_t s, bool use_graphs) {
    StepProfiler* prof = b.prof.get();
    if (!use_graphs || (prof && prof->every > 0)) return pcg_chunk<VR, MR>(L, t, count, s, prof);
    if (!b.graphs) b.graphs = std::make_unique<GraphCache>();
    GraphCache& gc = *b.graphs;
    if (!gc.capture) {
        RuntimeLock lk(runtime_mutex());
        SHELL_HIP(hipStreamCreateWithFlags(&gc.capture, hipStreamNonBlocking));
    }
    while (count > 0) {
        int c = kMinGraphChunk;
        while (2 * c <= count && 2 * c <= kMaxGraphChunk) c *= 2;
        if (c > count) return pcg_chunk<VR, MR>(L, t, count, s, nullptr);
        const GraphCache::Key key{L.sdesc, L.rows, L.nrows, L.pcg_grid, L.lds_spmv, L.per, L.per_u, c, int(t & 1),
                                  L.precision};
        hipGraphExec_t ex = nullptr;
        for (auto& e : gc.entries)
            if (e.first == key) ex = e.second;
        if (!ex) {
            RuntimeLock lk(runtime_mutex());
            hipGraph_t g = nullptr;
            SHELL_HIP(hipStreamBeginCapture(gc.capture, hipStreamCaptureModeThreadLocal));
            try {
                pcg_chunk<VR, MR>(L, t, c, gc.capture, nullptr);
            } catch (...) {
                (void)hipStreamEndCapture(gc.capture, &g);
                if (g) (void)hipGraphDestroy(g);
                throw;
            }
            SHELL_HIP(hipStreamEndCapture(gc.capture, &g));
            const hipError_t err = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
            (void)hipGraphDestroy(g);
            SHELL_HIP(err);
            if (int(gc.entries.size()) >= kMaxGraphs) {
                (void)hipGraphExecDestroy(gc.entries.front().second);
                gc.entries.erase(gc.entries.begin());
            }
            gc.entries.emplace_back(key, ex);
        }
        SHELL_HIP(hipGraphLaunch(ex, s));
        t += c;
        count -= c;
    }
    return t;
}

void forces(const Launch& L, hipStream_t s, StepProfiler* prof = nullptr) {
    timed_launch(prof, prof && prof->every > 0, SHELL_PHASE_FORCES, s, [&](hipEvent_t e0, hipEvent_t e1) {
        // the first model's kernel starts the interval, the last one's ends it
        int first = -1, last = -1;
        for (int m = 0; m < 6; ++m)
            if (L.ntiles[m]) {
                if (first < 0) first = m;
                last = m;
            }
        if (first < 0 && e0) {  // nothing to launch: an empty interval
            SHELL_HIP(hipEventRecord(e0, s));
            SHELL_HIP(hipEventRecord(e1, s));
        }
        for (int m = 0; m < 6; ++m)
            if (L.ntiles[m])
                launch_force_items(m, L.precision, L.fdesc, L.tiles[m], L.ntiles[m], L.lds_T, s,
                                   m == first ? e0 : nullptr, m == last ? e1 : nullptr);
    });
}

struct ItemBuilder {
    std::vector<WorkItem> rows, tiles[6];
    std::vector<int32_t> meshes;
    void build(const std::vector<shell_sim_s*>& sims, const std::vector<int>& subset) {
        rows.clear();
        meshes.clear();
        for (auto& t : tiles) t.clear();
        for (int m : subset) {
            const shell_sim_s& sim = *sims[size_t(m)];
            meshes.push_back(m);
            for (long g = 0; g < blocks(sim.nv); ++g) rows.push_back({m, int32_t(g)});
            for (long t = 0; t < sim.st->nblocks; ++t) tiles[sim.st->model].push_back({m, int32_t(t)});
        }
    }
};

// Copies the item lists through pinned staging to the batch's device item buffer.  The stream is
// drained first: earlier copies from the staging and earlier kernels reading the device buffer must
// have finished before either is overwritten.
Launch upload(shell_batch_s& b, const ItemBuilder& ib, hipStream_t s, int pcg_workgroups = SHELL_PCG_WORKGROUPS) {
    SHELL_HIP(hipStreamSynchronize(s));
    size_t total = ib.rows.size();
    for (const auto& t : ib.tiles) total += t.size();
    if (total > b.items_cap || !b.items_host) {
        {
            RuntimeLock lk(runtime_mutex());
            if (b.items_host) (void)hipHostFree(b.items_host);
            b.items_host = nullptr;
            b.items_cap = std::max<size_t>(total, 64) * 2;
            SHELL_HIP(hipHostMalloc(reinterpret_cast<void**>(&b.items_host), b.items_cap * sizeof(WorkItem)));
        }
        b.items.alloc(b.items_cap);
    }
    Launch L{};
    std::copy(ib.rows.begin(), ib.rows.end(), b.items_host);
    L.rows = b.items.p;
    L.nrows = long(ib.rows.size());
    size_t off = ib.rows.size();
    for (int m = 0; m < 6; ++m) {
        std::copy(ib.tiles[m].begin(), ib.tiles[m].end(), b.items_host + off);
        L.tiles[m] = b.items.p + off;
        L.ntiles[m] = long(ib.tiles[m].size());
        off += ib.tiles[m].size();
    }
    std::copy(ib.meshes.begin(), ib.meshes.end(), b.mlist_host);
    if (off) SHELL_HIP(hipMemcpyAsync(b.items.p, b.items_host, off * sizeof(WorkItem), hipMemcpyHostToDevice, s));
    if (!ib.meshes.empty())
        SHELL_HIP(hipMemcpyAsync(b.mlist.p, b.mlist_host, ib.meshes.size() * sizeof(int32_t),
                                 hipMemcpyHostToDevice, s));
    L.meshes = b.mlist.p;
    L.nmeshes = int(ib.meshes.size());
    L.sdesc = b.sdesc.p;
    L.fdesc = b.fdesc.p;
    L.precision = b.precision;
    L.lds_T = b.max_T;
    L.lds_spmv = b.lds_spmv;
    L.per = int(std::max<long>(1, (L.nrows + pcg_workgroups - 1) / pcg_workgroups));
    L.pcg_grid = xcd_grid((L.nrows + L.per - 1) / L.per);
    L.per_u = L.nmeshes == 1 ? std::max(1, L.per * SHELL_UPDATE_MERGE / SHELL_UPDATE_SPLIT) : L.per;
    L.upd_grid = xcd_grid((L.nrows + L.per_u - 1) / L.per_u);
    return L;
}

// The logical work-groups of L's PCG launches that can touch each mesh of the item list (the slots its
// dot-product partials are summed over), into the staged descriptors.  The product kernel's XCD x takes
// the run of items [x run, (x + 1) run), run = per W with W work-groups per XCD, so a mesh's items meet
// at most the work-groups of the XCDs whose runs overlap them; the update kernel's work-group takes
// per_u consecutive items.
void set_slot_ranges(shell_batch_s& b, const Launch& L, const ItemBuilder& ib) {
    const long W = L.pcg_grid / kXcds, run = long(L.per) * W;
    size_t a = 0;
    while (a < ib.rows.size()) {
        const int m = ib.rows[a].mesh;
        size_t e = a;
        while (e < ib.rows.size() && ib.rows[e].mesh == m) ++e;
        SolveDesc& d = b.sdesc_host[m];
        d.pq_lo = int32_t((long(a) / run) * W);
        d.pq_hi = int32_t(std::min(L.pcg_grid, ((long(e) - 1) / run + 1) * W));
        d.rz_lo = int32_t(long(a) / L.per_u);
        d.rz_hi = int32_t((long(e) - 1) / L.per_u + 1);
        a = e;
    }
}

void upload_descs(shell_batch_s& b, hipStream_t s) {
    SHELL_HIP(hipMemcpyAsync(b.sdesc.p, b.sdesc_host, b.sims.size() * sizeof(SolveDesc), hipMemcpyHostToDevice, s));
}

void read_states(shell_batch_s& b, hipStream_t s) {
    SHELL_HIP(hipMemcpyAsync(b.state_host, b.state.p, 2 * b.sims.size() * sizeof(PcgState), hipMemcpyDeviceToHost,
                             s));
    SHELL_HIP(hipStreamSynchronize(s));
    if (b.prof) b.prof->drain();
}

SolveDesc solve_desc(shell_sim_s& sim, PcgState* st) {
    SolveDesc d{};
    d.x = sim.x.p;
    d.X = sim.st->X.p;
    d.xhat = sim.xhat.p;
    d.xt = sim.xt.p;
    d.v = sim.v.p;
    d.g = sim.g.p;
    d.y = sim.y.p;
    d.y64 = sim.y64.p;  // null in FP64
    d.r = sim.r.p;
    d.f = sim.f.p;
    d.p0 = sim.p.p;
    d.p1 = sim.p2.p;
    d.q = sim.q.p;
    d.dinv = sim.dinv.p;
    d.mq = sim.mq.p;
    d.z = sim.z.p;  // null in FP64
    d.mass = sim.mass.p;
    d.kdiag = sim.h->kdiag.p;
    d.pinned = sim.pinned.p;
    d.partial_held = sim.partial_held ? 1 : 0;
    d.scol = sim.h->scol.p;
    d.val = sim.st->precision == SHELL_PREC_MIXED ? static_cast<const void*>(sim.h->valf.p)
                                                   : static_cast<const void*>(sim.h->val.p);
    d.sptr = sim.h->sptr.p;
    d.width = sim.h->width.p;
    d.gptr = sim.h->gptr.p;  // null when the mesh's row groups are too wide to stage
    d.gcols = sim.h->gcols.p;
    d.lcol = sim.h->lcol.p;
    d.st = st;
    d.part = sim.partials.p;
    d.bins = sim.bins.p;
    d.nv = sim.nv;
    d.ngroups = blocks(sim.nv);
    return d;
}

ForceDesc force_desc(shell_sim_s& sim) {
    const shell_stencils_s& st = *sim.st;
    const bool f32 = st.precision == SHELL_PREC_MIXED;
    ForceDesc d{};
    d.x = sim.x.p;
    d.X = st.X.p;
    d.f = sim.f.p;
    d.epart = nullptr;
    d.bias = st.bias.p;
    d.boff = st.boff.p;
    d.tidx = st.tidx.p;
    d.trec = f32 ? static_cast<const void*>(st.trec32.p) : static_cast<const void*>(st.trec64.p);
    d.nst = st.nst_pad;
    d.nv = st.nv;
    d.T = st.T;
    d.model = st.model;
    d.kb = st.kb;
    d.fscale = st.fscale;
    d.nu = st.poisson;
    return d;
}

struct MeshStep {
    const shell_step_params_t* prm = nullptr;
    shell_step_stats_t stats{};
    bool budget = false;
    double gn0 = 0, gn = 0;
    double tol2[3] = {0, 0, 0};  // the current solve's bound on r.r (kept by its refinement passes)
};

// Mixed precision: a tolerance-mode solve asked for a relative residual below this gets residual
// replacement passes (at most kRefinePasses), since the float32 products let the float64 recurrence
// residual drift from the true one by about this much.
constexpr double kRefineBelowRtol = 1e-6;
constexpr int kRefinePasses = 2;

// The step of every mesh of the batch: Newton rounds over the meshes still iterating; each round is
// one force/residual launch set, then one PCG loop over the meshes that still need a solve.
template <typename VR, typename MR>
shell_status_t step_impl(shell_batch_s& b, const shell_step_params_t* prms, int nparams, shell_step_stats_t* out,
                         hipStream_t s, const StaticMode* qs) {
    const int n = int(b.sims.size());
    const int wg = prms[0].pcg_workgroups > 0 ? prms[0].pcg_workgroups : SHELL_PCG_WORKGROUPS;
    const bool graphs = (prms[0].flags & SHELL_STEP_NO_GRAPHS) == 0;
    std::vector<MeshStep> ms(static_cast<size_t>(n));
    SHELL_HIP(hipStreamSynchronize(s));  // the descriptor staging is reused below
    if (b.fdesc_dirty) {
        for (int m = 0; m < n; ++m) b.fdesc_host[m] = force_desc(*b.sims[size_t(m)]);
        SHELL_HIP(hipMemcpyAsync(b.fdesc.p, b.fdesc_host, size_t(n) * sizeof(ForceDesc), hipMemcpyHostToDevice, s));
        b.fdesc_dirty = false;
    }
    for (int m = 0; m < n; ++m) {
        MeshStep& st = ms[size_t(m)];
        st.prm = &prms[nparams == 1 ? 0 : m];
        shell_sim_s& sim = *b.sims[size_t(m)];
        SolveDesc d = solve_desc(sim, b.state.p + 2 * m);
        d.dt = st.prm->dt;
        d.dt2 = d.dt * d.dt;
        for (int c = 0; c < 3; ++c) d.grav[c] = st.prm->gravity[c];
        if (qs) {
            // quasi-static: the matrix is K alone and the residual dPsi/dx - F; dt = 0 keeps the predictor
            // from moving x (x_hat = x)
            d.dt = 0.0;
            d.dt2 = 1.0;
            for (int c = 0; c < 3; ++c) d.grav[c] = 0.0;
            d.mass = sim.zmass.p;
            d.fext = qs->has_load ? sim.fext.p : nullptr;
            d.ustep = qs->eps_u > 0.0 ? sim.ustep.p : nullptr;
            d.eps_u = qs->eps_u;
        }
        d.rtol2 = st.prm->pcg_rtol * st.prm->pcg_rtol;
        b.sdesc_host[m] = d;
    }
    upload_descs(b, s);
    std::vector<int> all(static_cast<size_t>(n)), need_dinv;
    for (int m = 0; m < n; ++m) {
        all[size_t(m)] = m;
        shell_sim_s& sim = *b.sims[size_t(m)];
        const double key = b.sdesc_host[m].dt;  // 0 for the quasi-static matrix
        if (sim.dinv_dt != key) {
            need_dinv.push_back(m);
            sim.dinv_dt = key;
        }
    }
    ItemBuilder ib;
    Launch L;
    if (!need_dinv.empty()) {
        ib.build(b.sims, need_dinv);
        L = upload(b, ib, s, wg);
        k_dinv<VR><<<xcd_grid(L.nrows), kBlk, 0, s>>>(L.sdesc, L.rows, L.nrows);
    }
    ib.build(b.sims, all);
    L = upload(b, ib, s, wg);
    k_predictor<<<xcd_grid(L.nrows), kBlk, 0, s>>>(L.sdesc, L.rows, L.nrows);
    SHELL_HIP(hipGetLastError());

    std::vector<int> iterating = all;
    for (int k = 0; !iterating.empty(); ++k) {
        ib.build(b.sims, iterating);
        L = upload(b, ib, s, wg);
        forces(L, s, b.prof.get());
        k_residual<VR><<<xcd_grid(L.nrows), kBlk, 0, s>>>(L.sdesc, L.rows, L.nrows, 1);
        k_fin_residual<<<L.nmeshes, kRedBlk, 0, s>>>(L.sdesc, L.meshes);
        SHELL_HIP(hipGetLastError());
        read_states(b, s);
        std::vector<int> solve;
        for (int m : iterating) {
            MeshStep& st = ms[size_t(m)];
            const PcgState& ps = b.state_host[2 * m];
            if (ps.nonfinite) {
                st.stats.status = SHELL_E_NONFINITE;
                continue;
            }
            st.gn = std::sqrt(ps.gsq);
            if (k == 0) st.gn0 = st.gn;
            const shell_step_params_t& p = *st.prm;
            const bool met = st.gn0 == 0.0 || (qs ? st.gn < qs->eps_f : (k > 0 && st.gn <= p.newton_rtol * st.gn0));
            if (met) continue;
            if (k == p.max_newton) {
                st.stats.newton_capped = 1;
                continue;
            }
            solve.push_back(m);
        }
        if (solve.empty()) break;
        // One PCG solve over the meshes of `set`: per-mesh targets and the slot ranges of its launch shape
        // (upload() drains the stream first, so the staging is idle), the first kernel (from r = -g, or
        // for a refinement pass from the true residual of the increment so far), the first product, then
        // chunks until every mesh is done.  Returns the last product launched.
        auto run_pcg = [&](const std::vector<int>& set, bool refine) -> long {
            ib.build(b.sims, set);
            L = upload(b, ib, s, wg);
            for (int m : set) {
                const shell_step_params_t& p = *ms[size_t(m)].prm;
                SolveDesc& d = b.sdesc_host[m];
                d.replay = p.mode == SHELL_PCG_REPLAY;
                for (int c = 0; c < 3; ++c) {
                    d.target[c] = d.replay ? p.replay_counts[3 * k + c] : p.max_pcg;
                    d.tol2_abs[c] = refine ? ms[size_t(m)].tol2[c] : 0.0;
                }
            }
            set_slot_ranges(b, L, ib);
            upload_descs(b, s);
            if (refine) {
                k_pcg_fold<VR><<<xcd_grid(L.nrows), kBlk, 0, s>>>(L.sdesc, L.rows, L.nrows);
                for (int m : set) {
                    shell_sim_s& sim = *b.sims[size_t(m)];
                    const SolveDesc& d = b.sdesc_host[m];
                    launch_apply(*sim.h, d.mass, d.dt2, sim.y64.p, sim.rq.p, s);
                }
                k_pcg_refine_init<VR><<<L.upd_grid, kBlk, 0, s>>>(L.sdesc, L.rows, L.nrows, L.per_u);
            } else {
                k_pcg_init<VR><<<L.upd_grid, kBlk, 0, s>>>(L.sdesc, L.rows, L.nrows, L.per_u);
            }
            timed_launch(b.prof.get(), b.prof && b.prof->every > 0, SHELL_PHASE_PRODUCT, s,
                         [&](hipEvent_t e0, hipEvent_t e1) {
                             hipExtLaunchKernelGGL(k_pcg_spmv<VR, MR>, dim3(unsigned(L.pcg_grid)), dim3(kBlk),
                                                   uint32_t(L.lds_spmv), s, e0, e1, 0, L.sdesc, L.rows, L.nrows,
                                                   0L, L.per);
                         });
            SHELL_HIP(hipGetLastError());
            long t = 0;  // the last product launched
            bool all_replay = true;
            int most = 0, first_chunk = 8, max_chunk = 128;
            for (int m : set) {
                const shell_step_params_t& p = *ms[size_t(m)].prm;
                all_replay &= p.mode == SHELL_PCG_REPLAY;
                for (int c = 0; c < 3; ++c) most = std::max(most, b.sdesc_host[m].target[c]);
                if (p.chunk > 0) first_chunk = max_chunk = p.chunk;
            }
            if (all_replay) {
                t = pcg_iterations<VR, MR>(b, L, t, most, s, graphs);
                read_states(b, s);
            } else {
                read_states(b, s);
                int chunk = first_chunk;
                for (;;) {
                    bool done = true;
                    for (int m : set) done &= b.state_host[2 * m + ((t + 1) & 1)].done != 0;
                    if (done) break;
                    t = pcg_iterations<VR, MR>(b, L, t, chunk, s, graphs);
                    read_states(b, s);
                    chunk = std::min(2 * chunk, max_chunk);
                }
            }
            return t;
        };
        // Counts a finished solve (or refinement pass) into the Newton iteration's statistics; false when
        // the mesh's state went non-finite.  Returns the iterations of the pass in `its`.
        auto account = [&](int m, long t, int& its) {
            MeshStep& st = ms[size_t(m)];
            const PcgState& ps = b.state_host[2 * m + ((t + 1) & 1)];
            its = 0;
            if (ps.nonfinite) {
                st.stats.status = SHELL_E_NONFINITE;
                return false;
            }
            st.budget |= ps.budget != 0;
            for (int c = 0; c < 3; ++c) {
                st.stats.counts[k][c] += ps.iters[c];
                st.stats.pcg_total += ps.iters[c];
                its += ps.iters[c];
                st.tol2[c] = ps.tol2[c] > 0.0 ? ps.tol2[c] : DBL_MIN;
            }
            return true;
        };
        long t = run_pcg(solve, false);
        std::vector<int> next, refine;
        for (int m : solve) {
            int its = 0;
            if (!account(m, t, its)) continue;
            MeshStep& st = ms[size_t(m)];
            st.stats.newton_iters++;
            next.push_back(m);
            const shell_step_params_t& p = *st.prm;
            if (b.precision == SHELL_PREC_MIXED && p.mode == SHELL_PCG_TOLERANCE && p.pcg_rtol < kRefineBelowRtol &&
                !st.budget)
                refine.push_back(m);
        }
        // Mixed precision asked for more than the float32 products can give: residual replacement.  The
        // float64 recurrence residual drifts from the true one as float32 products accumulate, so the
        // true residual of the increment is formed with the float64 matrix and the PCG restarted from it,
        // with the first pass's bound on r.r; a pass that starts within the bound takes no iteration.
        const bool refined = !refine.empty();
        for (int pass = 0; pass < kRefinePasses && !refine.empty(); ++pass) {
            for (int m : refine) {
                shell_sim_s& sim = *b.sims[size_t(m)];
                if (!sim.rq.p) sim.rq.alloc(size_t(3 * sim.nv));
                b.sdesc_host[m].rq = sim.rq.p;
            }
            t = run_pcg(refine, true);
            std::vector<int> again;
            for (int m : refine) {
                int its = 0;
                if (!account(m, t, its)) {
                    next.erase(std::remove(next.begin(), next.end(), m), next.end());
                    continue;
                }
                if (its > 0 && !ms[size_t(m)].budget) again.push_back(m);
            }
            refine = again;
        }
        if (refined) {  // the Newton update below takes the launch shape of the whole solve again
            ib.build(b.sims, solve);
            L = upload(b, ib, s, wg);
        }
        if (qs && qs->eps_u > 0.0) {
            k_absmax<VR><<<xcd_grid(L.nrows), kBlk, 0, s>>>(L.sdesc, L.rows, L.nrows);
            k_fin_step_limit<<<L.nmeshes, kRedBlk, 0, s>>>(L.sdesc, L.meshes);
        }
        k_newton_update<VR><<<xcd_grid(L.nrows), kBlk, 0, s>>>(L.sdesc, L.rows, L.nrows);
        SHELL_HIP(hipGetLastError());
        iterating = next;
    }
    if (!qs) {
        ib.build(b.sims, all);
        L = upload(b, ib, s, wg);
        k_velocity<<<xcd_grid(L.nrows), kBlk, 0, s>>>(L.sdesc, L.rows, L.nrows);
        SHELL_HIP(hipGetLastError());
    }
    shell_status_t worst = SHELL_OK;
    for (int m = 0; m < n; ++m) {
        MeshStep& st = ms[size_t(m)];
        st.stats.grad_norm0 = st.gn0;
        st.stats.grad_norm = st.gn;
        if (st.stats.status == SHELL_OK && st.budget) st.stats.status = SHELL_E_BUDGET;
        shell_sim_s& sim = *b.sims[size_t(m)];
        sim.stats = st.stats;
        if (!qs) sim.step++;
        sim.last_stream = s;
        if (out) out[m] = st.stats;
        if (st.stats.status == SHELL_E_NONFINITE || (st.stats.status == SHELL_E_BUDGET && worst == SHELL_OK))
            worst = shell_status_t(st.stats.status);
    }
    return worst;
}

template <typename VR, typename MR>
void time_impl(shell_batch_s& b, double dt, int reps, shell_kernel_times_t& out, hipStream_t s) {
    shell_sim_s& sim = *b.sims[0];
    SHELL_HIP(hipStreamSynchronize(s));
    if (b.fdesc_dirty) {
        b.fdesc_host[0] = force_desc(sim);
        SHELL_HIP(hipMemcpyAsync(b.fdesc.p, b.fdesc_host, sizeof(ForceDesc), hipMemcpyHostToDevice, s));
        b.fdesc_dirty = false;
    }
    SolveDesc d = solve_desc(sim, b.state.p);
    d.dt = dt;
    d.dt2 = dt * dt;
    d.rtol2 = 0.0;
    d.replay = 1;
    d.target[0] = d.target[1] = d.target[2] = 1 << 30;
    b.sdesc_host[0] = d;
    upload_descs(b, s);
    ItemBuilder ib;
    ib.build(b.sims, std::vector<int>{0});
    Launch L = upload(b, ib, s);
    set_slot_ranges(b, L, ib);
    upload_descs(b, s);
    const long grid = xcd_grid(L.nrows);
    k_dinv<VR><<<grid, kBlk, 0, s>>>(L.sdesc, L.rows, L.nrows);
    sim.dinv_dt = dt;
    hipEvent_t e0, e1;
    SHELL_HIP(hipEventCreate(&e0));
    SHELL_HIP(hipEventCreate(&e1));
    auto init = [&]() {
        // a residual from the current forces, then an always-active recurrence through its first update
        forces(L, s);
        k_residual<VR><<<grid, kBlk, 0, s>>>(L.sdesc, L.rows, L.nrows, 0);
        k_fin_residual<<<1, kRedBlk, 0, s>>>(L.sdesc, L.meshes);
        k_pcg_init<VR><<<L.upd_grid, kBlk, 0, s>>>(L.sdesc, L.rows, L.nrows, L.per_u);
        k_pcg_spmv<VR, MR><<<L.pcg_grid, kBlk, L.lds_spmv, s>>>(L.sdesc, L.rows, L.nrows, 0, L.per);
        k_pcg_update<VR><<<L.upd_grid, kBlk, 0, s>>>(L.sdesc, L.rows, L.nrows, 0, L.per_u);
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
    // the force kernels alone
    out.force_ms = timed([&] { forces(L, s); });
    // repeated launches of one iteration's kernel: each re-reads the same state and partials
    init();
    out.spmv_ms = timed([&] {
        k_pcg_spmv<VR, MR><<<L.pcg_grid, kBlk, L.lds_spmv, s>>>(L.sdesc, L.rows, L.nrows, 1, L.per);
    });
    init();
    out.update_ms = timed([&] { k_pcg_update<VR><<<L.upd_grid, kBlk, 0, s>>>(L.sdesc, L.rows, L.nrows, 0, L.per_u); });
    init();
    out.direction_ms = 0.0;  // the direction update is part of the product kernel
    SHELL_HIP(hipGetLastError());
    SHELL_HIP(hipStreamSynchronize(s));
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
}

}  // namespace

void sim_alloc(shell_sim_s& sim) {
    const long nv = sim.nv, n3 = 3 * nv;
    for (auto* a : {&sim.x, &sim.v, &sim.xt, &sim.xhat, &sim.g, &sim.y, &sim.r, &sim.f, &sim.p, &sim.p2, &sim.q})
        a->alloc(size_t(std::max(n3, 1L)));
    sim.bins.alloc(size_t(2 * 2 * kBinQ * kSlots));
    if (sim.st->precision == SHELL_PREC_MIXED) {
        sim.z.alloc(size_t(std::max(n3, 1L)));
        sim.y64.alloc(size_t(std::max(n3, 1L)));
    }
    sim.mass.alloc(size_t(std::max(nv, 1L)));
    sim.dinv.alloc(size_t(std::max(nv, 1L)));
    sim.mq.alloc(size_t(std::max(nv, 1L)));
    sim.pinned.alloc(size_t(std::max(nv, 1L)));
    sim.partials.alloc(size_t(kMaxPart * std::max(blocks(nv), 1L) + kMaxPart));
}

void sim_mass(shell_sim_s& sim, hipStream_t s) {
    shell_stencils_s& st = *sim.st;
    if (!sim.nv) return;
    const Incidence vt = build_incidence(st.h_tris, 3, st.nt, st.nv);
    DevArray<int64_t> ptr(vt.ptr.size()), code(std::max<size_t>(vt.code.size(), 1));
    ptr.upload(vt.ptr.data(), vt.ptr.size(), s);
    code.upload(vt.code.data(), vt.code.size(), s);
    k_mass_rows<<<blocks(sim.nv), kBlk, 0, s>>>(st.X.p, st.tris.p, ptr.p, code.p, sim.nv, st.density * st.thickness,
                                                sim.mass.p);
    SHELL_HIP(hipGetLastError());
    SHELL_HIP(hipStreamSynchronize(s));  // the incidence lists are released on return
}

// (Re)binds a batch to its member simulations.  Buffers only grow; the force descriptors are staged on
// the host and uploaded on the stream of the next step, so this makes no device-wide synchronisation.
void batch_init(shell_batch_s& b) {
    const size_t n = b.sims.size();
    b.graphs.reset();  // graphs bake in buffer addresses of the previous members
    SHELL_CHECK(n > 0, SHELL_E_INVALID_ARG, "empty batch");
    b.precision = b.sims[0]->st->precision;
    b.max_T = 64;
    const bool membrane = b.sims[0]->ms != nullptr;
    for (size_t m = 0; m < n; ++m) {
        SHELL_CHECK((b.sims[m]->ms != nullptr) == membrane, SHELL_E_INVALID_ARG,
                    "a batch holds simulations with the membrane or simulations without it, not both");
        SHELL_CHECK(b.sims[m]->st->precision == b.precision, SHELL_E_INVALID_ARG,
                    "all simulations of a batch need the same precision");
        for (size_t q = 0; q < m; ++q)
            SHELL_CHECK(b.sims[q] != b.sims[m], SHELL_E_INVALID_ARG, "a simulation appears twice in a batch");
        b.max_T = std::max(b.max_T, b.sims[m]->st->T);
    }
    b.membrane = membrane;
    if (membrane) return;  // the members step with their own solver state
    size_t vr = b.precision == SHELL_PREC_MIXED ? sizeof(float) : sizeof(double);
    b.lds_spmv = 0;
    for (size_t m = 0; m < n; ++m)
        if (b.sims[m]->h->gptr.p)
            b.lds_spmv = std::max(b.lds_spmv, size_t(b.sims[m]->h->pat.max_gcols) * 3 * vr);
    if (n > b.capacity) {
        batch_free_host(b);
        b.capacity = std::max<size_t>(n, 2 * b.capacity);
        b.fdesc.alloc(b.capacity);
        b.sdesc.alloc(b.capacity);
        b.state.alloc(2 * b.capacity);
        {
            RuntimeLock lk(runtime_mutex());
            SHELL_HIP(hipHostMalloc(reinterpret_cast<void**>(&b.state_host), 2 * b.capacity * sizeof(PcgState)));
            SHELL_HIP(hipHostMalloc(reinterpret_cast<void**>(&b.sdesc_host), b.capacity * sizeof(SolveDesc)));
            SHELL_HIP(hipHostMalloc(reinterpret_cast<void**>(&b.fdesc_host), b.capacity * sizeof(ForceDesc)));
            SHELL_HIP(hipHostMalloc(reinterpret_cast<void**>(&b.mlist_host), (b.capacity + 1) * sizeof(int32_t)));
        }
        b.mlist.alloc(b.capacity + 1);
    }
    b.fdesc_dirty = true;
}

void batch_free_host(shell_batch_s& b) {
    RuntimeLock lk(runtime_mutex());
    for (void** p : {reinterpret_cast<void**>(&b.state_host), reinterpret_cast<void**>(&b.sdesc_host),
                     reinterpret_cast<void**>(&b.fdesc_host), reinterpret_cast<void**>(&b.mlist_host)}) {
        if (*p) (void)hipHostFree(*p);
        *p = nullptr;
    }
}

void batch_release(shell_batch_s& b) {
    b.graphs.reset();
    batch_free_host(b);
    RuntimeLock lk(runtime_mutex());
    if (b.items_host) (void)hipHostFree(b.items_host);
    b.items_host = nullptr;
    b.items_cap = 0;
}

shell_status_t batch_step(shell_batch_s& b, const shell_step_params_t* p, int nparams, shell_step_stats_t* stats,
                          hipStream_t s, const StaticMode* qs) {
    for (shell_sim_s* sim : b.sims)
        SHELL_CHECK(sim->nv > 0, SHELL_E_INVALID_ARG, "empty simulation in a batch");
    if (b.membrane) {
        SHELL_CHECK(!qs, SHELL_E_UNSUPPORTED, "the quasi-static solve with the membrane runs per simulation");
        return membrane_batch_step(b, p, nparams, stats, s);
    }
    if (b.precision == SHELL_PREC_MIXED) return step_impl<float, float>(b, p, nparams, stats, s, qs);
    return step_impl<double, double>(b, p, nparams, stats, s, qs);
}

void batch_time_kernels(shell_batch_s& b, double dt, int reps, shell_kernel_times_t& out, hipStream_t s) {
    SHELL_CHECK(!b.membrane, SHELL_E_UNSUPPORTED, "kernel timing of a simulation with the membrane runs per simulation");
    if (b.precision == SHELL_PREC_MIXED)
        time_impl<float, float>(b, dt, reps, out, s);
    else
        time_impl<double, double>(b, dt, reps, out, s);
}

}  // namespace shell
