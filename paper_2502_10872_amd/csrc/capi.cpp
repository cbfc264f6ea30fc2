// C ABI entry points (include/shell.h): argument checks, handle lifetime, caller <-> internal vertex
// order, and translation of exceptions into status codes.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <memory>
#include <mutex>
#include <new>

#include "internal.hpp"

using namespace shell;

namespace {

thread_local std::string g_last_error;

template <typename F>
shell_status_t guarded(F&& fn) {
    try {
        g_last_error.clear();
        return fn();
    } catch (const Error& e) {
        g_last_error = e.what();
        return e.status;
    } catch (const std::bad_alloc&) {
        g_last_error = "host allocation failed";
        return SHELL_E_OOM;
    } catch (const std::exception& e) {
        g_last_error = e.what();
        return SHELL_E_INVALID_ARG;
    }
}

hipStream_t as_stream(shell_stream_t s) { return static_cast<hipStream_t>(s); }

// A private non-blocking stream for the copies of a call that has no stream argument (an export, the
// initial state of a simulation): it waits only for its own work, never for another thread's streams
// (the arrays an export reads were complete when their create call returned).
struct HostCopyStream {
    hipStream_t s = nullptr;
    HostCopyStream() {
        RuntimeLock lk(runtime_mutex());
        SHELL_HIP(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
    }
    ~HostCopyStream() {
        RuntimeLock lk(runtime_mutex());
        (void)hipStreamDestroy(s);
    }
    HostCopyStream(const HostCopyStream&) = delete;
    HostCopyStream& operator=(const HostCopyStream&) = delete;
};

void check_params(const shell_step_params_t& p) {
    SHELL_CHECK(p.dt > 0 && std::isfinite(p.dt), SHELL_E_INVALID_ARG, "dt must be positive");
    SHELL_CHECK(p.max_newton >= 0 && p.max_newton <= SHELL_MAX_NEWTON, SHELL_E_INVALID_ARG, "max_newton out of range");
    SHELL_CHECK(p.mode == SHELL_PCG_TOLERANCE || p.mode == SHELL_PCG_REPLAY, SHELL_E_INVALID_ARG, "unknown mode");
    SHELL_CHECK(p.mode != SHELL_PCG_REPLAY || p.replay_counts, SHELL_E_INVALID_ARG, "replay needs counts");
    SHELL_CHECK(p.mode == SHELL_PCG_REPLAY || p.max_pcg > 0, SHELL_E_INVALID_ARG, "max_pcg must be positive");
    SHELL_CHECK(p.chunk >= 0, SHELL_E_INVALID_ARG, "chunk must be >= 0");
    SHELL_CHECK(p.pcg_workgroups >= 0 && p.pcg_workgroups <= 1024, SHELL_E_INVALID_ARG,
                "pcg_workgroups must be in 0..1024");
    SHELL_CHECK((p.flags & ~SHELL_STEP_NO_GRAPHS) == 0, SHELL_E_INVALID_ARG, "unknown step flag");
    for (int c = 0; c < 3; ++c) SHELL_CHECK(std::isfinite(p.gravity[c]), SHELL_E_INVALID_ARG, "gravity not finite");
    if (p.mode == SHELL_PCG_REPLAY)
        for (int q = 0; q < 3 * p.max_newton; ++q)
            SHELL_CHECK(p.replay_counts[q] >= 0, SHELL_E_INVALID_ARG, "negative replay count");
}

__global__ void gather1(const double* __restrict__ src, const int32_t* __restrict__ perm, double* __restrict__ dst,
                        long n) {
    long i = blockIdx.x * long(blockDim.x) + threadIdx.x;
    if (i < n) dst[i] = src[perm[i]];
}

}  // namespace

extern "C" {

const char* shell_status_string(shell_status_t s) {
    switch (s) {
        case SHELL_OK: return "ok";
        case SHELL_E_INVALID_ARG: return "invalid argument";
        case SHELL_E_NONMANIFOLD: return "non-manifold mesh";
        case SHELL_E_ORIENTATION: return "inconsistent triangle orientation";
        case SHELL_E_DEGENERATE: return "degenerate stencil";
        case SHELL_E_NONFINITE: return "non-finite value";
        case SHELL_E_BUDGET: return "iteration budget exhausted";
        case SHELL_E_OOM: return "out of memory";
        case SHELL_E_HIP: return "HIP runtime error";
        case SHELL_E_UNSUPPORTED: return "unsupported";
    }
    return "unknown status";
}

const char* shell_last_error(void) { return g_last_error.c_str(); }

shell_status_t shell_build_stencils(const double* X, int64_t nv, const int32_t* tris, int64_t nt, int32_t model,
                                    const shell_material_t* mat, const int32_t* clamped_edges, int64_t n_clamped,
                                    const shell_config_t* cfg, shell_stream_t stream, shell_stencils_t* out) {
    return guarded([&]() -> shell_status_t {
        SHELL_CHECK(out && mat && (X || nv == 0) && (tris || nt == 0), SHELL_E_INVALID_ARG, "null argument");
        *out = nullptr;
        SHELL_CHECK(model >= SHELL_EP && model <= SHELL_SS, SHELL_E_INVALID_ARG, "unknown model");
        SHELL_CHECK(nv >= 0 && nt >= 0 && nv < (int64_t(1) << 30) && 3 * nt < (int64_t(1) << 31), SHELL_E_INVALID_ARG,
                    "mesh size out of range");
        SHELL_CHECK(n_clamped >= 0 && (clamped_edges || n_clamped == 0), SHELL_E_INVALID_ARG, "bad clamped edge list");
        for (int64_t e = 0; e < 2 * n_clamped; ++e)
            SHELL_CHECK(clamped_edges[e] >= 0 && clamped_edges[e] < nv, SHELL_E_INVALID_ARG,
                        "clamped edge vertex out of range");
        SHELL_CHECK(mat->young > 0 && mat->thickness > 0 && mat->density >= 0 && mat->poisson > -1.0 &&
                        mat->poisson < 1.0,
                    SHELL_E_INVALID_ARG, "material out of range");
        for (int64_t i = 0; i < 3 * nv; ++i)
            SHELL_CHECK(std::isfinite(X[i]), SHELL_E_NONFINITE, "non-finite rest position");
        int precision = cfg ? cfg->precision : SHELL_PREC_FP64;
        SHELL_CHECK(precision == SHELL_PREC_FP64 || precision == SHELL_PREC_MIXED, SHELL_E_INVALID_ARG,
                    "unknown precision");
        int T = (cfg && cfg->block_vertices > 0) ? cfg->block_vertices : 2048;
        SHELL_CHECK(T >= 64 && T <= 4096, SHELL_E_INVALID_ARG, "block_vertices must be in [64, 4096]");
        int reorder = cfg ? cfg->reorder : 1;
        SHELL_CHECK(reorder >= 0 && reorder <= 2, SHELL_E_INVALID_ARG, "unknown vertex order");
        const int cfg_flags = cfg ? cfg->flags : 0;
        SHELL_CHECK((cfg_flags & ~(SHELL_FLAG_DIRECT_PRODUCT | SHELL_FLAG_WORLD_FRAME | SHELL_FLAG_MEMBRANE)) == 0,
                    SHELL_E_INVALID_ARG, "unknown flag");
        SHELL_CHECK(!(cfg_flags & SHELL_FLAG_WORLD_FRAME) || model_is_edge(model), SHELL_E_INVALID_ARG,
                    "the world-frame operator applies to the edge models (EP, ES)");
        hipStream_t s = as_stream(stream);

        auto st = std::make_unique<shell_stencils_s>();
        st->model = model;
        st->k = model_k(model);
        st->r = model_r(model);
        st->precision = precision;
        st->nv = nv;
        st->nt = nt;
        st->T = T;
        st->cfg_flags = cfg_flags;
        st->young = mat->young;
        st->poisson = mat->poisson;
        st->thickness = mat->thickness;
        st->density = mat->density;
        st->kb = mat->young * std::pow(mat->thickness, 3) / (12.0 * (1.0 - mat->poisson * mat->poisson));
        HostTopology topo = build_topology(model, nv, nt, tris, n_clamped, clamped_edges);
        {
            // force scales of the order-independent tile accumulation (powers of two); the topology
            // check above has validated the triangle ids
            double lsum = 0.0;
            for (int64_t t = 0; t < nt; ++t)
                for (int e = 0; e < 3; ++e) {
                    const double* a = X + 3 * size_t(tris[3 * t + e]);
                    const double* b = X + 3 * size_t(tris[3 * t + (e + 1) % 3]);
                    lsum += std::sqrt((a[0] - b[0]) * (a[0] - b[0]) + (a[1] - b[1]) * (a[1] - b[1]) +
                                      (a[2] - b[2]) * (a[2] - b[2]));
                }
            const double ell = nt ? lsum / double(3 * nt) : 1.0;
            auto pow2 = [](double v) {
                return (std::isfinite(v) && v > 0.0) ? std::ldexp(1.0, int(std::lround(std::log2(v)))) : 1.0;
            };
            st->fscale = pow2(st->kb / ell) * 0x1p-12;
            st->mscale = pow2(mat->young * mat->thickness * ell) * 0x1p-12;
        }

        const int k = st->k, r = st->r;
        st->ns = topo.ns;
        st->perm = vertex_order(X, nv, reorder, T);
        st->reordered = reorder != 0;
        st->iperm.assign(size_t(nv), 0);
        for (int64_t i = 0; i < nv; ++i) st->iperm[size_t(st->perm[size_t(i)])] = int32_t(i);
        // stencils in internal ids, sorted by their first vertex for locality
        std::vector<int64_t> order(size_t(st->ns));
        for (int64_t q = 0; q < st->ns; ++q) order[size_t(q)] = q;
        auto iid = [&](int32_t v) { return v < 0 ? -1 : st->iperm[size_t(v)]; };
        std::stable_sort(order.begin(), order.end(), [&](int64_t a, int64_t b) {
            return iid(topo.idx[size_t(k * a)]) < iid(topo.idx[size_t(k * b)]);
        });
        st->h_idx.resize(size_t(k * st->ns));
        std::vector<int32_t> h_bc(size_t(st->ns));
        bool any_clamped = false;
        for (int64_t q = 0; q < st->ns; ++q) {
            for (int j = 0; j < k; ++j) st->h_idx[size_t(k * q + j)] = iid(topo.idx[size_t(k * order[size_t(q)] + j)]);
            h_bc[size_t(q)] = topo.bc[size_t(order[size_t(q)])];
            any_clamped = any_clamped || (h_bc[size_t(q)] & kBcClampedAny) != 0;
        }
        std::vector<double> Xi(size_t(3 * nv));
        for (int64_t i = 0; i < nv; ++i)
            for (int c = 0; c < 3; ++c) Xi[size_t(3 * i + c)] = X[3 * int64_t(st->perm[size_t(i)]) + c];
        st->h_tris.resize(size_t(3 * nt));
        for (int64_t t = 0; t < 3 * nt; ++t) st->h_tris[size_t(t)] = st->iperm[size_t(tris[t])];

        const size_t ns = size_t(st->ns);
        st->X.alloc(size_t(3 * nv));
        st->X.upload(Xi.data(), Xi.size(), s);
        st->tris.alloc(size_t(3 * nt));
        st->tris.upload(st->h_tris.data(), st->h_tris.size(), s);
        st->perm_d.alloc(size_t(nv));
        st->perm_d.upload(st->perm.data(), size_t(nv), s);
        // unique stencils, SoA; a missing flap points at vertex 1 (its operator column is zero)
        std::vector<int32_t> soa(size_t(k) * ns);
        for (size_t q = 0; q < ns; ++q)
            for (int j = 0; j < k; ++j) {
                int32_t v = st->h_idx[size_t(k) * q + j];
                soa[size_t(j) * ns + q] = v < 0 ? st->h_idx[size_t(k) * q] : v;
            }
        st->idx.alloc(soa.size());
        st->idx.upload(soa.data(), soa.size(), s);
        st->B.alloc(size_t(r * k) * ns);
        st->k0.alloc(size_t(r) * ns);
        st->flags.alloc(ns);
        DevArray<int32_t> bc_d(ns);
        bc_d.upload(h_bc.data(), ns, s);
        launch_precompute(*st, bc_d.p, s);
        std::vector<int32_t> flags(ns);
        st->flags.download(flags.data(), ns, s);
        SHELL_HIP(hipStreamSynchronize(s));
        for (size_t q = 0; q < ns; ++q)
            SHELL_CHECK(flags[q] == 0, SHELL_E_DEGENERATE,
                        "degenerate stencil (zero area or height, or ill-conditioned quadratic fit)");
        // tiles for the force kernel
        Tiling til = build_tiling(st->h_idx, k, st->ns, nv, T);
        st->nblocks = til.nblocks;
        st->ns_tiled = til.count;
        st->nst_pad = int64_t(til.src.size());
        st->h_boff = til.boff;
        st->boff.alloc(til.boff.size());
        st->boff.upload(til.boff.data(), til.boff.size(), s);
        st->tsrc.alloc(til.src.size());
        st->tsrc.upload(til.src.data(), til.src.size(), s);
        const size_t nst = size_t(st->nst_pad);
        // only the precision the force kernel streams is kept in the tiled layout
        if (precision == SHELL_PREC_MIXED) {
            st->trec32.alloc(size_t(4 * stream_chunks(rec32_fields(k, r, model_is_shell(model)), 4)) * nst);
        } else {
            st->tidx.alloc(size_t(4 * stream_chunks(k, 4)) * nst);
            st->trec64.alloc(size_t(2 * stream_chunks(rec64_fields(k, r), 2)) * nst);
        }
        launch_tile_copy(*st, bc_d.p, s);
        if (any_clamped && precision == SHELL_PREC_FP64 && !model_is_shell(model)) launch_clamp_bias(*st, bc_d.p, s);
        st->epart.alloc(size_t(st->nblocks));
        if (cfg_flags & SHELL_FLAG_MEMBRANE) launch_membrane_rest(*st, s);
        SHELL_HIP(hipStreamSynchronize(s));
        *out = st.release();
        return SHELL_OK;
    });
}

shell_status_t shell_stencils_info(shell_stencils_t st, shell_stencils_info_t* info) {
    return guarded([&]() -> shell_status_t {
        SHELL_CHECK(st && info, SHELL_E_INVALID_ARG, "null argument");
        std::memset(info, 0, sizeof(*info));
        info->nv = st->nv;
        info->nt = st->nt;
        info->ns = st->ns;
        info->ns_tiled = st->ns_tiled;
        info->nblocks = st->nblocks;
        info->model = st->model;
        info->k = st->k;
        info->r = st->r;
        info->precision = st->precision;
        info->block_vertices = st->T;
        return SHELL_OK;
    });
}

shell_status_t shell_stencils_export(shell_stencils_t st, int32_t* idx, double* B, double* kappa0) {
    return guarded([&]() -> shell_status_t {
        SHELL_CHECK(st, SHELL_E_INVALID_ARG, "null handle");
        const size_t ns = size_t(st->ns);
        const int k = st->k, r = st->r;
        if (idx)
            for (size_t q = 0; q < ns; ++q)
                for (int j = 0; j < k; ++j) {
                    int32_t v = st->h_idx[size_t(k) * q + j];
                    idx[size_t(k) * q + j] = v < 0 ? -1 : st->perm[size_t(v)];
                }
        if (B || kappa0) {
            std::vector<double> hb(size_t(r * k) * ns), hk(size_t(r) * ns);
            HostCopyStream cs;
            st->B.download(hb.data(), hb.size(), cs.s);
            st->k0.download(hk.data(), hk.size(), cs.s);
            SHELL_HIP(hipStreamSynchronize(cs.s));
            for (size_t q = 0; q < ns; ++q) {
                if (B)
                    for (int c = 0; c < r * k; ++c) B[size_t(r * k) * q + c] = hb[size_t(c) * ns + q];
                if (kappa0)
                    for (int c = 0; c < r; ++c) kappa0[size_t(r) * q + c] = hk[size_t(c) * ns + q];
            }
        }
        return SHELL_OK;
    });
}

shell_status_t shell_eval_forces(shell_stencils_t st, const double* x, void* f, double* energy,
                                 shell_stream_t stream) {
    return guarded([&]() -> shell_status_t {
        SHELL_CHECK(st && (x || st->nv == 0) && (f || st->nv == 0), SHELL_E_INVALID_ARG, "null argument");
        hipStream_t s = as_stream(stream);
        const bool f32 = st->precision == SHELL_PREC_MIXED;
        if (st->nv > 0 && !st->fdesc.p) {
            // caller-order staging, descriptor and tile items, made on first use
            st->xin.alloc(size_t(3 * st->nv));
            st->fout.alloc(size_t(3 * st->nv));
            ForceDesc d{};
            d.x = st->xin.p;
            d.X = st->X.p;
            d.f = st->fout.p;
            d.epart = st->epart.p;
            d.bias = st->bias.p;
            d.boff = st->boff.p;
            d.tidx = st->tidx.p;
            d.trec = f32 ? static_cast<const void*>(st->trec32.p) : static_cast<const void*>(st->trec64.p);
            d.nst = st->nst_pad;
            d.nv = st->nv;
            d.T = st->T;
            d.model = st->model;
            d.kb = st->kb;
            d.fscale = st->fscale;
            d.nu = st->poisson;
            std::vector<WorkItem> items(size_t(st->nblocks));
            for (int64_t t = 0; t < st->nblocks; ++t) items[size_t(t)] = {0, int32_t(t)};
            st->fdesc.alloc(1);
            st->tile_items.alloc(items.size());
            st->fdesc.upload(&d, 1, s);
            st->tile_items.upload(items.data(), items.size(), s);
            SHELL_HIP(hipStreamSynchronize(s));
        }
        if (st->nv > 0) {
            launch_gather_rows(x, st->perm_d.p, st->xin.p, st->nv, s);
            launch_force_items(st->model, st->precision, st->fdesc.p, st->tile_items.p, st->nblocks, st->T, s);
            if (st->cfg_flags & SHELL_FLAG_MEMBRANE) launch_membrane_forces(*st, st->xin.p, st->fout.p, s);
            launch_scatter_rows(st->fout.p, st->perm_d.p, f, st->nv, f32, s);
        }
        if (energy) {
            if (st->nv == 0)
                launch_energy_finalize(nullptr, 0, 0.0, energy, s);  // a kernel, not a memset node
            else
                launch_energy_finalize(st->epart.p, st->nblocks, st->bias_e0, energy, s, st->mepart.p,
                                       int64_t(st->mepart.n));
        }
        return SHELL_OK;
    });
}

// ------------------------------------------------------------------ force evaluation without allocation

namespace {

// The scratch of shell_eval_forces_noalloc on every device the library runs on: the caller-order
// positions in internal order, the internal-order force (float64 or float32), the per-tile energy
// partials, the force descriptor and the tile work items.  The array's name is a host-side stand-in:
// host code uses only the device address hipGetSymbolAddress returns for the current device.
constexpr size_t kScratchBytes = size_t(64) << 20;
__device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mutex;
void* g_scratch_ptr[kMaxDevices] = {};

void* scratch_for_current_device() {
    int dev = 0;
    SHELL_HIP(hipGetDevice(&dev));
    SHELL_CHECK(dev >= 0 && dev < kMaxDevices, SHELL_E_UNSUPPORTED, "device ordinal beyond the scratch table");
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        SHELL_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
        SHELL_CHECK(ptr != nullptr, SHELL_E_HIP, "hipGetSymbolAddress returned no address for the scratch");
        g_scratch_ptr[dev] = ptr;
    }
    return g_scratch_ptr[dev];
}

size_t align256(size_t n) { return (n + 255) & ~size_t(255); }

}  // namespace

shell_status_t shell_eval_forces_noalloc(shell_stencils_t st, const double* x, void* f, double* energy,
                                         shell_stream_t stream) {
    return guarded([&]() -> shell_status_t {
        SHELL_CHECK(st && (x || st->nv == 0) && (f || st->nv == 0), SHELL_E_INVALID_ARG, "null argument");
        hipStream_t s = as_stream(stream);
        const bool f32 = st->precision == SHELL_PREC_MIXED;
        // layout of the scratch: positions, force, energy partials, descriptor, tile items
        const size_t o_x = 0, o_f = align256(o_x + size_t(3 * st->nv) * sizeof(double));
        const size_t o_e = align256(o_f + size_t(3 * st->nv) * sizeof(double));
        const size_t o_d = align256(o_e + size_t(st->nblocks) * sizeof(double));
        const size_t o_i = align256(o_d + sizeof(ForceDesc));
        const size_t need = o_i + size_t(st->nblocks) * sizeof(WorkItem);
        SHELL_CHECK(need <= kScratchBytes, SHELL_E_INVALID_ARG,
                    "mesh too large for the no-allocation force entry point (its 64 MiB scratch holds about "
                    "1.39 million vertices)");
        if (st->nv == 0) {
            if (energy) launch_energy_finalize(nullptr, 0, 0.0, energy, s);
            return SHELL_OK;
        }
        unsigned char* base = static_cast<unsigned char*>(scratch_for_current_device());
        double* xin = reinterpret_cast<double*>(base + o_x);
        void* fout = base + o_f;
        double* epart = reinterpret_cast<double*>(base + o_e);
        ForceDesc* desc = reinterpret_cast<ForceDesc*>(base + o_d);
        WorkItem* items = reinterpret_cast<WorkItem*>(base + o_i);
        ForceDesc d{};
        d.x = xin;
        d.X = st->X.p;
        d.f = fout;
        d.epart = epart;
        d.bias = st->bias.p;
        d.boff = st->boff.p;
        d.tidx = st->tidx.p;
        d.trec = f32 ? static_cast<const void*>(st->trec32.p) : static_cast<const void*>(st->trec64.p);
        d.nst = st->nst_pad;
        d.nv = st->nv;
        d.T = st->T;
        d.model = st->model;
        d.kb = st->kb;
        d.fscale = st->fscale;
        d.nu = st->poisson;
        // descriptor and items written by kernels on the stream (no host-to-device copy to order)
        launch_write_force_desc(d, desc, items, st->nblocks, s);
        launch_gather_rows(x, st->perm_d.p, xin, st->nv, s);
        launch_force_items(st->model, st->precision, desc, items, st->nblocks, st->T, s);
        if (st->cfg_flags & SHELL_FLAG_MEMBRANE) launch_membrane_forces(*st, xin, fout, s);
        launch_scatter_rows(fout, st->perm_d.p, f, st->nv, f32, s);
        if (energy)
            launch_energy_finalize(epart, st->nblocks, st->bias_e0, energy, s, st->mepart.p, int64_t(st->mepart.n));
        return SHELL_OK;
    });
}

shell_status_t shell_assemble_constant_hessian(shell_stencils_t st, shell_stream_t stream, shell_hessian_t* out) {
    return guarded([&]() -> shell_status_t {
        SHELL_CHECK(st && out, SHELL_E_INVALID_ARG, "null argument");
        *out = nullptr;
        hipStream_t s = as_stream(stream);
        auto h = std::make_unique<shell_hessian_s>();
        h->st = st;
        h->pat = build_sell_pattern(st->h_idx, st->k, st->ns, st->nv,
                                    (st->cfg_flags & SHELL_FLAG_DIRECT_PRODUCT) == 0);
        const auto& P = h->pat;
        h->scol.alloc(size_t(P.nslots));
        h->scol.upload(P.scol.data(), size_t(P.nslots), s);
        h->width.alloc(size_t(P.nslices));
        h->width.upload(P.width.data(), size_t(P.nslices), s);
        h->sptr.alloc(size_t(P.nslices + 1));
        h->sptr.upload(P.sptr.data(), size_t(P.nslices + 1), s);
        h->rowlen.alloc(size_t(st->nv));
        h->rowlen.upload(P.rowlen.data(), size_t(st->nv), s);
        if (!P.gptr.empty()) {
            h->gptr.alloc(P.gptr.size());
            h->gptr.upload(P.gptr.data(), P.gptr.size(), s);
            h->gcols.alloc(P.gcols.size());
            h->gcols.upload(P.gcols.data(), P.gcols.size(), s);
            h->lcol.alloc(P.lcol.size());
            h->lcol.upload(P.lcol.data(), P.lcol.size(), s);
        }
        h->val.alloc(size_t(P.nslots));
        if (st->precision == SHELL_PREC_MIXED) h->valf.alloc(size_t(P.nslots));
        h->kdiag.alloc(size_t(st->nv));
        launch_assemble(*h, s);
        *out = h.release();
        return SHELL_OK;
    });
}

shell_status_t shell_hessian_info(shell_hessian_t h, shell_hessian_info_t* info) {
    return guarded([&]() -> shell_status_t {
        SHELL_CHECK(h && info, SHELL_E_INVALID_ARG, "null argument");
        const auto& P = h->pat;
        std::memset(info, 0, sizeof(*info));
        info->nv = P.nv;
        info->nnz = P.nnz;
        info->slots = P.nslots;
        info->nslices = P.nslices;
        info->staged = h->gptr.n > 0 ? 1 : 0;
        info->group_cols = info->staged ? int64_t(P.gcols.size()) : 0;
        info->max_group_cols = P.max_gcols;
        return SHELL_OK;
    });
}

shell_status_t shell_hessian_export_csr(shell_hessian_t h, int64_t* nnz, int64_t* rowptr, int32_t* col,
                                        double* val) {
    return guarded([&]() -> shell_status_t {
        SHELL_CHECK(h && nnz, SHELL_E_INVALID_ARG, "null argument");
        const auto& P = h->pat;
        *nnz = P.nnz;
        if (!col && !val && !rowptr) return SHELL_OK;
        const shell_stencils_s& st = *h->st;
        std::vector<double> sv(size_t(P.nslots));
        HostCopyStream cs;
        h->val.download(sv.data(), sv.size(), cs.s);
        SHELL_HIP(hipStreamSynchronize(cs.s));
        const int64_t nv = st.nv;
        // caller row u = perm[i]; its entries are internal row i's, columns mapped by perm and re-sorted
        std::vector<int64_t> ptr(size_t(nv + 1), 0);
        for (int64_t i = 0; i < nv; ++i) ptr[size_t(st.perm[size_t(i)]) + 1] = P.rowptr[i + 1] - P.rowptr[i];
        for (int64_t u = 0; u < nv; ++u) ptr[u + 1] += ptr[u];
        if (rowptr) std::copy(ptr.begin(), ptr.end(), rowptr);
        if (!col && !val) return SHELL_OK;
        std::vector<std::pair<int32_t, double>> row;
        for (int64_t u = 0; u < nv; ++u) {
            int64_t i = st.iperm[size_t(u)];
            row.clear();
            for (int64_t e = P.rowptr[i]; e < P.rowptr[i + 1]; ++e)
                row.emplace_back(st.perm[size_t(P.col[size_t(e)])], sv[size_t(P.csr2sell[size_t(e)])]);
            std::sort(row.begin(), row.end(),
                      [](const auto& a, const auto& b) { return a.first < b.first; });
            for (size_t q = 0; q < row.size(); ++q) {
                if (col) col[ptr[u] + int64_t(q)] = row[q].first;
                if (val) val[ptr[u] + int64_t(q)] = row[q].second;
            }
        }
        return SHELL_OK;
    });
}

shell_status_t shell_hessian_apply(shell_hessian_t h, const double* mass, double dt2, const double* p, double* q,
                                   shell_stream_t stream) {
    return guarded([&]() -> shell_status_t {
        SHELL_CHECK(h && p && q, SHELL_E_INVALID_ARG, "null argument");
        hipStream_t s = as_stream(stream);
        const shell_stencils_s& st = *h->st;
        const long nv = st.nv;
        if (!nv) return SHELL_OK;
        if (!h->pin.p) {  // caller-order staging, made on first use
            h->pin.alloc(size_t(3 * nv));
            h->qout.alloc(size_t(4 * nv));
        }
        double* min = nullptr;
        if (mass) {
            min = h->qout.p + 3 * nv;
            gather1<<<(nv + 255) / 256, 256, 0, s>>>(mass, st.perm_d.p, min, nv);
            SHELL_HIP(hipGetLastError());
        }
        launch_gather_rows(p, st.perm_d.p, h->pin.p, nv, s);
        launch_apply(*h, min, dt2, h->pin.p, h->qout.p, s);
        launch_scatter_rows(h->qout.p, st.perm_d.p, q, nv, false, s);
        return SHELL_OK;
    });
}

shell_status_t shell_sim_create(shell_stencils_t st, shell_hessian_t h, const double* x0, const double* v0,
                                const uint8_t* pinned, shell_sim_t* out) {
    return guarded([&]() -> shell_status_t {
        SHELL_CHECK(st && h && out && (x0 || st->nv == 0) && h->st == st, SHELL_E_INVALID_ARG, "bad argument");
        *out = nullptr;
        const bool membrane = (st->cfg_flags & SHELL_FLAG_MEMBRANE) != 0;
        auto sim = std::make_unique<shell_sim_s>();
        sim->st = st;
        sim->h = h;
        sim->nv = st->nv;
        sim_alloc(*sim);
        const int64_t nv = st->nv;
        std::vector<double> xi(size_t(3 * nv)), vi(size_t(3 * nv), 0.0);
        std::vector<uint8_t> pi(size_t(nv), 0);
        for (int64_t i = 0; i < nv; ++i) {
            int64_t u = st->perm[size_t(i)];
            for (int c = 0; c < 3; ++c) {
                xi[size_t(3 * i + c)] = x0[3 * u + c];
                if (v0) vi[size_t(3 * i + c)] = v0[3 * u + c];
            }
            if (pinned) pi[size_t(i)] = pinned[u] ? 7 : 0;  // every coordinate held
        }
        HostCopyStream cs;
        hipStream_t s = cs.s;
        sim->x.upload(xi.data(), xi.size(), s);
        sim->v.upload(vi.data(), vi.size(), s);
        sim->pinned.upload(pi.data(), pi.size(), s);
        sim_mass(*sim, s);
        SHELL_HIP(hipStreamSynchronize(s));
        if (nv > 0 && membrane) {
            membrane_sim_init(*sim, s);
        } else if (nv > 0) {
            auto solo = std::make_unique<shell_batch_s>();
            solo->sims = {sim.get()};
            batch_init(*solo);
            sim->solo = solo.release();
        }
        *out = sim.release();
        return SHELL_OK;
    });
}

shell_status_t shell_step_implicit(shell_sim_t sim, const shell_step_params_t* params, shell_step_stats_t* stats,
                                   shell_stream_t stream) {
    return guarded([&]() -> shell_status_t {
        SHELL_CHECK(sim && params, SHELL_E_INVALID_ARG, "null argument");
        const shell_step_params_t& p = *params;
        check_params(p);
        shell_status_t rc = SHELL_OK;
        if (sim->ms) {
            SHELL_CHECK(p.max_newton <= SHELL_MAX_NEWTON, SHELL_E_INVALID_ARG, "max_newton out of range");
            shell_step_stats_t st{};
            rc = membrane_step(*sim, p, st, as_stream(stream));
        } else if (sim->nv > 0) {
            rc = batch_step(*sim->solo, &p, 1, nullptr, as_stream(stream));
        } else {
            sim->stats = shell_step_stats_t{};
            sim->step++;
        }
        if (stats) {
            SHELL_HIP(hipStreamSynchronize(as_stream(stream)));
            *stats = sim->stats;
        }
        if (rc == SHELL_E_BUDGET) g_last_error = "PCG iteration budget exhausted";
        if (rc == SHELL_E_NONFINITE) g_last_error = "non-finite residual";
        return rc;
    });
}

shell_status_t shell_solve_static(shell_sim_t sim, const shell_static_params_t* params, shell_step_stats_t* stats,
                                  shell_stream_t stream) {
    return guarded([&]() -> shell_status_t {
        SHELL_CHECK(sim && params, SHELL_E_INVALID_ARG, "null argument");
        const shell_static_params_t& q = *params;
        SHELL_CHECK(q.eps_f >= 0.0 && std::isfinite(q.eps_f), SHELL_E_INVALID_ARG, "eps_f must be >= 0");
        SHELL_CHECK(q.eps_u >= 0.0 && std::isfinite(q.eps_u), SHELL_E_INVALID_ARG, "eps_u must be >= 0");
        shell_step_params_t p{};
        p.dt = 1.0;  // unused by the quasi-static path
        p.max_newton = q.max_newton;
        p.max_pcg = q.max_pcg;
        p.pcg_rtol = q.pcg_rtol;
        p.mode = q.mode;
        p.chunk = q.chunk;
        p.pcg_workgroups = q.pcg_workgroups;
        p.flags = q.flags;
        p.replay_counts = q.replay_counts;
        check_params(p);
        hipStream_t s = as_stream(stream);
        shell_status_t rc = SHELL_OK;
        StaticMode qs;
        qs.eps_f = q.eps_f;
        qs.eps_u = q.eps_u;
        qs.has_load = q.load != nullptr;
        const int64_t nv = sim->nv;
        if (nv > 0) {
            if (!sim->zmass.p) {
                sim->zmass.alloc(size_t(nv));
                SHELL_HIP(hipMemsetAsync(sim->zmass.p, 0, size_t(nv) * sizeof(double), s));
                sim->ustep.alloc(1);
            }
            if (q.load) {
                for (int64_t i = 0; i < 3 * nv; ++i)
                    SHELL_CHECK(std::isfinite(q.load[i]), SHELL_E_INVALID_ARG, "non-finite load");
                // caller order to internal order
                std::vector<double> h(size_t(3 * nv));
                const std::vector<int32_t>& perm = sim->st->perm;
                for (int64_t i = 0; i < nv; ++i)
                    for (int c = 0; c < 3; ++c) h[size_t(3 * i + c)] = q.load[3 * int64_t(perm[size_t(i)]) + c];
                if (!sim->fext.p) sim->fext.alloc(size_t(3 * nv));
                sim->fext.upload(h.data(), h.size(), s);
                SHELL_HIP(hipStreamSynchronize(s));  // h is released on return
            }
            if (sim->ms) {
                MembraneStatic mq;
                mq.load = qs.has_load ? sim->fext.p : nullptr;
                mq.eps_f = q.eps_f;
                mq.eps_u = q.eps_u;
                shell_step_stats_t st{};
                rc = membrane_static(*sim, p, mq, st, s);
            } else {
                rc = batch_step(*sim->solo, &p, 1, nullptr, s, &qs);
            }
        } else {
            sim->stats = shell_step_stats_t{};
        }
        if (stats) {
            SHELL_HIP(hipStreamSynchronize(s));
            *stats = sim->stats;
        }
        if (rc == SHELL_E_BUDGET) g_last_error = "PCG iteration budget exhausted";
        if (rc == SHELL_E_NONFINITE) g_last_error = "non-finite residual";
        return rc;
    });
}

shell_status_t shell_sim_get_stats(shell_sim_t sim, shell_step_stats_t* out) {
    return guarded([&]() -> shell_status_t {
        SHELL_CHECK(sim && out, SHELL_E_INVALID_ARG, "null argument");
        *out = sim->stats;
        return SHELL_OK;
    });
}

shell_status_t shell_sim_get_state(shell_sim_t sim, double* x, double* v, int64_t* step) {
    return guarded([&]() -> shell_status_t {
        SHELL_CHECK(sim, SHELL_E_INVALID_ARG, "null handle");
        const int64_t nv = sim->nv;
        const auto& perm = sim->st->perm;
        SHELL_HIP(hipStreamSynchronize(sim->last_stream));
        std::vector<double> buf(size_t(3 * nv));
        for (int which = 0; which < 2; ++which) {
            double* dst = which ? v : x;
            if (!dst) continue;
            (which ? sim->v : sim->x).download(buf.data(), buf.size(), sim->last_stream);
            SHELL_HIP(hipStreamSynchronize(sim->last_stream));
            for (int64_t i = 0; i < nv; ++i)
                for (int c = 0; c < 3; ++c) dst[3 * int64_t(perm[size_t(i)]) + c] = buf[size_t(3 * i + c)];
        }
        if (step) *step = sim->step;
        return SHELL_OK;
    });
}

shell_status_t shell_sim_set_state(shell_sim_t sim, const double* x, const double* v, int64_t step) {
    return guarded([&]() -> shell_status_t {
        SHELL_CHECK(sim, SHELL_E_INVALID_ARG, "null handle");
        const int64_t nv = sim->nv;
        const auto& perm = sim->st->perm;
        SHELL_HIP(hipStreamSynchronize(sim->last_stream));
        std::vector<double> buf(size_t(3 * nv));
        for (int which = 0; which < 2; ++which) {
            const double* src = which ? v : x;
            if (!src) continue;
            for (int64_t i = 0; i < nv; ++i)
                for (int c = 0; c < 3; ++c) buf[size_t(3 * i + c)] = src[3 * int64_t(perm[size_t(i)]) + c];
            (which ? sim->v : sim->x).upload(buf.data(), buf.size(), sim->last_stream);
            SHELL_HIP(hipStreamSynchronize(sim->last_stream));
        }
        sim->step = step;
        return SHELL_OK;
    });
}

shell_status_t shell_sim_set_held(shell_sim_t sim, const uint8_t* held) {
    return guarded([&]() -> shell_status_t {
        SHELL_CHECK(sim, SHELL_E_INVALID_ARG, "null handle");
        const int64_t nv = sim->nv;
        const auto& perm = sim->st->perm;
        std::vector<uint8_t> m(size_t(std::max<int64_t>(nv, 1)), 0);
        bool partial = false;
        for (int64_t i = 0; i < nv; ++i) {
            const uint8_t b = held ? held[perm[size_t(i)]] : uint8_t(0);
            SHELL_CHECK(b <= 7, SHELL_E_INVALID_ARG, "a held mask takes bits 0..2 only");
            m[size_t(i)] = b;
            partial = partial || (b != 0 && b != 7);
        }
        SHELL_HIP(hipStreamSynchronize(sim->last_stream));
        if (nv > 0) {
            sim->pinned.upload(m.data(), size_t(nv), sim->last_stream);
            SHELL_HIP(hipStreamSynchronize(sim->last_stream));
        }
        sim->partial_held = partial;
        sim->dinv_dt = -1.0;  // the preconditioner's fixed rows changed
        return SHELL_OK;
    });
}

shell_status_t shell_sim_device_state(shell_sim_t sim, double** x, double** v) {
    return guarded([&]() -> shell_status_t {
        SHELL_CHECK(sim, SHELL_E_INVALID_ARG, "null handle");
        if (x) *x = sim->x.p;
        if (v) *v = sim->v.p;
        return SHELL_OK;
    });
}

shell_status_t shell_sim_time_kernels(shell_sim_t sim, double dt, int32_t reps, shell_kernel_times_t* out,
                                      shell_stream_t stream) {
    return guarded([&]() -> shell_status_t {
        SHELL_CHECK(sim && out && reps > 0 && dt > 0, SHELL_E_INVALID_ARG, "bad argument");
        std::memset(out, 0, sizeof(*out));
        if (sim->ms)
            membrane_time_kernels(*sim, dt, reps, *out, as_stream(stream));
        else if (sim->solo)
            batch_time_kernels(*sim->solo, dt, reps, *out, as_stream(stream));
        return SHELL_OK;
    });
}

namespace {
void profile_set(shell_batch_s& b, int32_t every) {
    if (every == 0) {
        b.prof.reset();
        return;
    }
    if (!b.prof) b.prof = std::make_unique<shell::StepProfiler>();
    b.prof->every = every;
    b.prof->reset();
}

void profile_read(const shell_batch_s* b, shell_profile_t* out) {
    std::memset(out, 0, sizeof(*out));
    if (!b || !b->prof) return;
    for (int k = 0; k < SHELL_NUM_PHASES; ++k) {
        out->ms[k] = b->prof->ms[k];
        out->count[k] = b->prof->count[k];
    }
}
}  // namespace

shell_status_t shell_batch_profile(shell_batch_t batch, int32_t every) {
    return guarded([&]() -> shell_status_t {
        SHELL_CHECK(batch && every >= 0, SHELL_E_INVALID_ARG, "bad argument");
        SHELL_CHECK(!batch->membrane || every == 0, SHELL_E_UNSUPPORTED,
                    "sampled timing covers the solver without the membrane");
        profile_set(*batch, every);
        return SHELL_OK;
    });
}

shell_status_t shell_batch_profile_read(shell_batch_t batch, shell_profile_t* out) {
    return guarded([&]() -> shell_status_t {
        SHELL_CHECK(batch && out, SHELL_E_INVALID_ARG, "bad argument");
        profile_read(batch, out);
        return SHELL_OK;
    });
}

shell_status_t shell_sim_profile(shell_sim_t sim, int32_t every) {
    return guarded([&]() -> shell_status_t {
        SHELL_CHECK(sim && every >= 0, SHELL_E_INVALID_ARG, "bad argument");
        if (sim->solo) profile_set(*sim->solo, every);
        return SHELL_OK;
    });
}

shell_status_t shell_sim_profile_read(shell_sim_t sim, shell_profile_t* out) {
    return guarded([&]() -> shell_status_t {
        SHELL_CHECK(sim && out, SHELL_E_INVALID_ARG, "bad argument");
        profile_read(sim->solo, out);
        return SHELL_OK;
    });
}

void shell_destroy_stencils(shell_stencils_t st) { delete st; }
void shell_destroy_hessian(shell_hessian_t h) { delete h; }
void shell_destroy_sim(shell_sim_t sim) {
    if (!sim) return;
    if (sim->solo) {
        batch_release(*sim->solo);
        delete sim->solo;
    }
    delete sim;
}

shell_status_t shell_batch_create(const shell_sim_t* sims, int32_t n, shell_batch_t* out) {
    return guarded([&]() -> shell_status_t {
        SHELL_CHECK(sims && out && n >= 1, SHELL_E_INVALID_ARG, "bad argument");
        *out = nullptr;
        auto b = std::make_unique<shell_batch_s>();
        for (int32_t m = 0; m < n; ++m) {
            SHELL_CHECK(sims[m], SHELL_E_INVALID_ARG, "null simulation");
            b->sims.push_back(sims[m]);
        }
        try {
            batch_init(*b);
        } catch (...) {
            batch_release(*b);
            throw;
        }
        *out = b.release();
        return SHELL_OK;
    });
}

shell_status_t shell_batch_reset(shell_batch_t batch, const shell_sim_t* sims, int32_t n) {
    return guarded([&]() -> shell_status_t {
        SHELL_CHECK(batch && sims && n >= 1, SHELL_E_INVALID_ARG, "bad argument");
        std::vector<shell_sim_s*> next;
        for (int32_t m = 0; m < n; ++m) {
            SHELL_CHECK(sims[m], SHELL_E_INVALID_ARG, "null simulation");
            next.push_back(sims[m]);
        }
        std::swap(batch->sims, next);
        try {
            batch_init(*batch);
        } catch (...) {
            std::swap(batch->sims, next);
            throw;
        }
        return SHELL_OK;
    });
}

shell_status_t shell_sim_device_bytes(shell_sim_t sim, int64_t* stencil_bytes, int64_t* hessian_bytes,
                                      int64_t* sim_bytes) {
    return guarded([&]() -> shell_status_t {
        SHELL_CHECK(sim, SHELL_E_INVALID_ARG, "null handle");
        const shell_stencils_s& st = *sim->st;
        const shell_hessian_s& h = *sim->h;
        int64_t a = 0, b = 0, c = 0;
        for (size_t v : {st.X.bytes(), st.tris.bytes(), st.perm_d.bytes(), st.idx.bytes(), st.B.bytes(),
                         st.k0.bytes(), st.flags.bytes(), st.boff.bytes(), st.tsrc.bytes(), st.tidx.bytes(),
                         st.trec64.bytes(), st.trec32.bytes(), st.xin.bytes(),
                         st.fout.bytes(), st.epart.bytes(), st.fdesc.bytes(), st.tile_items.bytes(), st.bias.bytes(),
                         st.mtid.bytes(), st.mtrest.bytes(), st.mboff.bytes(), st.mepart.bytes()})
            a += int64_t(v);
        for (size_t v : {h.scol.bytes(), h.width.bytes(), h.sptr.bytes(), h.rowlen.bytes(), h.val.bytes(),
                         h.valf.bytes(), h.kdiag.bytes(), h.pin.bytes(), h.qout.bytes(), h.gptr.bytes(),
                         h.gcols.bytes(), h.lcol.bytes()})
            b += int64_t(v);
        for (size_t v : {sim->x.bytes(), sim->v.bytes(), sim->xt.bytes(), sim->xhat.bytes(), sim->g.bytes(),
                         sim->mass.bytes(), sim->y.bytes(), sim->r.bytes(), sim->f.bytes(), sim->dinv.bytes(), sim->mq.bytes(),
                         sim->pinned.bytes(), sim->p.bytes(), sim->p2.bytes(), sim->z.bytes(), sim->q.bytes(),
                         sim->bins.bytes(), sim->partials.bytes(), sim->y64.bytes(), sim->rq.bytes(),
                         sim->zmass.bytes(), sim->fext.bytes(), sim->ustep.bytes()})
            c += int64_t(v);
        if (sim->ms) c += int64_t(sim->ms->bytes());
        if (stencil_bytes) *stencil_bytes = a;
        if (hessian_bytes) *hessian_bytes = b;
        if (sim_bytes) *sim_bytes = c;
        return SHELL_OK;
    });
}

shell_status_t shell_batch_step(shell_batch_t batch, const shell_step_params_t* params, int32_t nparams,
                                shell_step_stats_t* stats, shell_stream_t stream) {
    return guarded([&]() -> shell_status_t {
        SHELL_CHECK(batch && params && (nparams == 1 || nparams == int32_t(batch->sims.size())),
                    SHELL_E_INVALID_ARG, "params must hold 1 or n entries");
        for (int32_t q = 0; q < nparams; ++q) check_params(params[q]);
        shell_status_t rc = batch_step(*batch, params, nparams, stats, as_stream(stream));
        if (stats) SHELL_HIP(hipStreamSynchronize(as_stream(stream)));
        if (rc == SHELL_E_BUDGET) g_last_error = "PCG iteration budget exhausted in at least one mesh";
        if (rc == SHELL_E_NONFINITE) g_last_error = "non-finite residual in at least one mesh";
        return rc;
    });
}

void shell_destroy_batch(shell_batch_t batch) {
    if (!batch) return;
    batch_release(*batch);
    delete batch;
}

}  // extern "C"
