// Internal declarations of the HIP library behind include/shell.h.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <stdexcept>
#include <string>
#include <memory>
#include <mutex>
#include <vector>

#include "shell.h"

namespace shell {

// ------------------------------------------------------------------ errors

struct Error : std::runtime_error {
    shell_status_t status;
    Error(shell_status_t s, const std::string& m) : std::runtime_error(m), status(s) {}
};

#define SHELL_HIP(call)                                                                                       \
    do {                                                                                                      \
        hipError_t e_ = (call);                                                                               \
        if (e_ != hipSuccess)                                                                                 \
            throw ::shell::Error(e_ == hipErrorOutOfMemory ? SHELL_E_OOM : SHELL_E_HIP,                       \
                                 std::string(#call) + ": " + hipGetErrorString(e_));                          \
    } while (0)

#define SHELL_CHECK(cond, status, msg)                                     \
    do {                                                                   \
        if (!(cond)) throw ::shell::Error((status), (msg));                \
    } while (0)

// ------------------------------------------------------------------ runtime calls against graph capture
//
// While one thread captures a stream into a graph, the HIP runtime refuses some calls from other threads
// (a device-wide synchronisation is one) and the refusal also invalidates that capture.  The library
// makes no device-wide synchronisation; its allocations, releases, stream creation and destruction and
// its own capture sections all take this one process-wide lock, so that handles driven from different
// threads never interleave such a call with a capture.
inline std::recursive_mutex& runtime_mutex() {
    static std::recursive_mutex m;
    return m;
}
using RuntimeLock = std::lock_guard<std::recursive_mutex>;

// ------------------------------------------------------------------ device buffers

template <typename T>
struct DevArray {
    T* p = nullptr;
    size_t n = 0;
    DevArray() = default;
    explicit DevArray(size_t count) { alloc(count); }
    DevArray(const DevArray&) = delete;
    DevArray& operator=(const DevArray&) = delete;
    ~DevArray() { release(); }
    void alloc(size_t count) {
        release();
        n = count;
        if (count) {
            RuntimeLock lk(runtime_mutex());
            SHELL_HIP(hipMalloc(&p, count * sizeof(T)));
        }
    }
    void release() {
        if (p) {
            RuntimeLock lk(runtime_mutex());
            (void)hipFree(p);
        }
        p = nullptr;
        n = 0;
    }
    void upload(const T* h, size_t count, hipStream_t s) {
        if (count) SHELL_HIP(hipMemcpyAsync(p, h, count * sizeof(T), hipMemcpyHostToDevice, s));
    }
    void download(T* h, size_t count, hipStream_t s) const {
        if (count) SHELL_HIP(hipMemcpyAsync(h, p, count * sizeof(T), hipMemcpyDeviceToHost, s));
    }
    size_t bytes() const { return n * sizeof(T); }
};

// ------------------------------------------------------------------ model traits

inline bool model_is_edge(int m) { return m == SHELL_EP || m == SHELL_ES; }
inline bool model_is_shell(int m) { return m == SHELL_ES || m == SHELL_FS || m == SHELL_SS; }
inline bool model_is_fvm(int m) { return m == SHELL_FP || m == SHELL_FS; }
inline int model_k(int m) { return model_is_edge(m) ? 4 : 6; }
inline int model_r(int m) { return model_is_edge(m) ? 1 : 3; }

// ------------------------------------------------------------------ host mesh processing (host_mesh.cpp)

// Boundary bits of a stencil.  Triangle stencils: bit L, flap L+3 missing; bit 3+L, that flap's edge
// clamped.  Edge stencils: kBcEdgeClamped, the stencil (L, M, N, -1) of a clamped boundary edge.
constexpr int32_t kBcEdgeClamped = 1 << 6;
constexpr int32_t kBcClampedAny = (7 << 3) | kBcEdgeClamped;

struct HostTopology {
    int model = 0, k = 4;
    int64_t ns = 0;
    std::vector<int32_t> idx;  // [ns][k] caller ids, -1 = missing flap (or the clamped edge's virtual node)
    std::vector<int32_t> bc;   // [ns] boundary bits
};
// Validates the triangle mesh and enumerates the model's stencils.  clamped [n_clamped][2]: boundary edges
// with the clamped condition (eqs 30-31, 59); a pair that is not a boundary edge is an argument error.
// The edge plate gets one stencil per clamped edge; the edge shell none (measured along its own
// triangle's normal, the folded stencil's transverse displacements all vanish).
HostTopology build_topology(int model, int64_t nv, int64_t nt, const int32_t* tris, int64_t n_clamped,
                            const int32_t* clamped);

// Vertex order: perm[internal] = caller id.  mode 0: the caller's order; 1: recursive coordinate
// bisection into tiles of T vertices (Morton inside a tile); 2: Morton order of the rest positions.
std::vector<int32_t> vertex_order(const double* X, int64_t nv, int mode, int T);

// Tiled stencil streams are stored in blocks of 64 stencils (one wave).  A stream's fields are grouped in
// chunks of 16 bytes (four 32-bit or two 64-bit fields): chunk c of list entry e sits at chunk index
// ((e / 64) * nchunks + c) * 64 + e % 64, so each lane reads a chunk with one 16-byte load and a wave's
// loads of one chunk are one contiguous 1 KB run.  Every tile's list starts at a multiple of 64; the
// slots between a list's end and the next start are padding (vertex 0, zeros) that no kernel reads.
constexpr int kStreamBlock = 64;
__host__ __device__ constexpr int stream_chunks(int nfields, int per_chunk) {
    return (nfields + per_chunk - 1) / per_chunk;
}
// Fields per stencil.  Mixed precision: one 32-bit record of the k vertex ids, the operator's r*(k-1)
// entries other than the origin's column (edge: vertex 1, the hinge's first end; triangle: vertex 0),
// which the kernel takes as minus the sum of the row's other entries (every row of B sums to zero), and
// for shells the r rest curvatures kappa0 = B~ h0 of the float32-rounded operator B~ on the rest heights
// h0, in float64 (as the bit patterns of r doubles), so that the bending strain B~ h - kappa0, summed in
// float64, vanishes at the rest shape to float64 rounding.  The edge plate adds, from field 8 on, the
// float64 coordinates (alpha, beta) of its tip 3 in the basis of the rest edges 0 - 1 and 2 - 1, all three
// projected onto the rest tangent plane, as two doubles.  Plate stencils with a clamped edge set bit 31 of
// the first id.
// FP64: the k ids in one stream and the r*k + r operator entries and rest curvatures in another.
__host__ __device__ constexpr int rec32_fields(int k, int r, bool shell) {
    return (k == 4 && !shell) ? 12 : k + r * (k - 1) + (shell ? 2 * r : 0);
}
constexpr int kRecEdgeAffine = 8;  // first field of the edge plate's (alpha, beta)
constexpr uint32_t kRecClampBit = 0x80000000u;
constexpr uint32_t kRecIdMask = 0x7fffffffu;
__host__ __device__ constexpr int rec64_fields(int k, int r) { return r * k + r; }

struct Tiling {
    int T = 1024;                 // vertices per tile
    int64_t nblocks = 0;
    int64_t count = 0;            // tiled stencils (halo copies included, padding not)
    std::vector<int64_t> boff;    // [2 nblocks]: start (a multiple of 64) and end of each tile's list
    std::vector<int32_t> src;     // [padded length] source stencil of each list slot, -1 for padding
};
// Groups stencils (internal vertex ids) by the vertex tiles they touch; halo stencils repeat.
Tiling build_tiling(const std::vector<int32_t>& idx, int k, int64_t ns, int64_t nv, int T);

// For every vertex, the tuples of a k-tuple list (stencils, triangles) that contain it, in ascending
// tuple order: code = tuple * 8 + position.  Lets the one-time sums over a vertex's stencils (the rows of
// K_s, the lumped mass, the clamp force) be taken per vertex in a fixed order, without atomics.
struct Incidence {
    std::vector<int64_t> ptr;   // [nv + 1]
    std::vector<int64_t> code;  // [ptr[nv]]
};
Incidence build_incidence(const std::vector<int32_t>& idx, int k, int64_t n, int64_t nv);

struct SellPattern {
    int64_t nv = 0, nslices = 0, nnz = 0, nslots = 0;
    std::vector<int64_t> rowptr;  // CSR of the pattern (internal order), sorted columns
    std::vector<int32_t> col;
    std::vector<int32_t> width;   // [nslices]
    std::vector<int64_t> sptr;    // [nslices+1] slot offset of each 64-row slice
    std::vector<int32_t> rowlen;  // [nv]
    std::vector<int32_t> scol;    // [nslots] SELL-64 column ids (padded with the row's last column)
    std::vector<int64_t> csr2sell;  // [nnz] slot of each CSR entry
    std::vector<int64_t> dslot;   // [nv] slot of the diagonal entry (or -1)
    // row groups of kRowGroup rows: the distinct columns of each group, and every slot's column as an
    // index into its group's list (the product stages the group's p entries in LDS)
    std::vector<int32_t> gptr;    // [ngroups+1]
    std::vector<int32_t> gcols;   // distinct columns, sorted per group
    std::vector<uint16_t> lcol;   // [nslots] group-local column index
    int32_t max_gcols = 0;
};
constexpr int kRowGroup = 512;     // rows per work item (and threads per work-group) of the row kernels
constexpr int kMaxGroupCols = 4096;  // largest column set staged in LDS (larger: direct gathers)
// staging: build the row groups' column lists (used when every group fits kMaxGroupCols)
SellPattern build_sell_pattern(const std::vector<int32_t>& idx, int k, int64_t ns, int64_t nv, bool staging);

// ------------------------------------------------------------------ kernel descriptors

// Per-mesh arguments of the force kernel.  Kernels take an array of descriptors and a list of work
// items (mesh, unit): one launch covers any set of meshes, a single mesh being a set of one.
struct ForceDesc {
    const double* x;       // positions [nv][3] (both precisions)
    const double* X;       // rest positions [nv][3] (read by the mixed plate kernels)
    void* f;               // double or float [nv][3]
    double* epart;         // per-tile energy, or null
    const double* bias;    // FP64 plates with clamped edges: constant force [nv][3] added to f, or null
    const int64_t* boff;   // [2 tiles]: start and end of each tile's stencil list
    const int32_t* tidx;   // FP64: vertex id stream
    const void* trec;      // mixed: the 32-bit record stream; FP64: the operator and rest-curvature stream
    int64_t nst, nv;
    int32_t T, model;
    double kb, nu;
    double fscale;         // power-of-two force scale of the tile accumulation (TileAcc)
};

// Per-mesh arguments of the implicit-step kernels.
struct PcgState {
    double rz[3], rr[3], tol2[3], alpha[3], beta[3];
    double gsq;
    int32_t iters[3], target[3], active[3];
    int32_t done, budget, replay, nonfinite;
};

struct SolveDesc {
    double *x, *xhat, *xt, *v, *g, *r;
    const double* fext;             // quasi-static: the applied load F [nv][3] (internal order), or null
    double* ustep;                  // quasi-static with an increment limit: the Newton step's scale, or null
    double eps_u;                   // quasi-static increment limit (max |dx| per Newton iteration)
    void* y;                        // the Newton increment the PCG builds (float in mixed precision: the part
                                    // not yet folded into y64)
    double* y64;                    // mixed precision only: the float64 part of the increment (y = y64 + y)
    const double* X;                // rest positions
    void *f, *p0, *p1, *q, *dinv;   // float in mixed precision; p0/p1 alternate as the search direction
    float* z;                       // mixed precision only: z = D^-1 r as float (null in FP64: recomputed)
    const double *mass, *kdiag;
    const uint8_t* pinned;          // held coordinates per vertex: bit c holds coordinate c, 7 the vertex
    void* mq;                       // the product's mass, in the vector precision; -1 on fixed rows
    const int32_t* scol;
    const void* val;                // SELL values, float in mixed precision
    const int64_t* sptr;
    const int32_t* width;
    const int32_t* gptr;            // group column lists (null: gather p directly)
    const int32_t* gcols;
    const uint16_t* lcol;
    PcgState* st;                   // two states: st[t & 1] enters PCG iteration t
    double* part;                   // reduction partials, quantity-major [q][group]
    double* bins;                   // PCG dot-product partials [parity][set][quantity][work-group slot]
    int32_t pq_lo, pq_hi;           // logical work-groups of the product launch that can touch this mesh
    int32_t rz_lo, rz_hi;           // the same for the update launch (and the solve's first kernel)
    int64_t nv, ngroups;
    double dt, dt2, grav[3], rtol2;
    int32_t replay, target[3];
    int32_t partial_held;           // some vertex has only part of its coordinates held
    double tol2_abs[3];             // > 0: the stop test's bound on r.r as given (a refinement pass keeps
                                    // the first pass's); 0: rtol2 times the initial r.r
    const double* rq;               // mixed refinement: the float64 product (M + dt^2 K_s) y64
};

struct WorkItem {
    int32_t mesh, unit;
};

// ------------------------------------------------------------------ handles

}  // namespace shell

struct shell_stencils_s {
    int model = 0, k = 4, r = 1, precision = 0;
    int64_t nv = 0, nt = 0, ns = 0, ns_tiled = 0, nblocks = 0;
    int64_t nst_pad = 0;  // tiled list length with the per-tile alignment padding
    int T = 1024;
    int cfg_flags = 0;  // SHELL_FLAG_*
    bool reordered = false;
    double young = 0, poisson = 0, thickness = 0, density = 0, kb = 0;
    // power-of-two force scales of the tile accumulation (l the mean rest edge): bending k_b / l 2^-12, the
    // force of a kink at the element scale divided by 4096, so that contributions up to 2^24 times that
    // force are summed exactly, to 2^-51 of it (a few float64 ulps); membrane E h l 2^-12, strains up to
    // 2^24
    double fscale = 1.0, mscale = 1.0;
    std::vector<int32_t> perm, iperm;    // internal -> caller, caller -> internal
    std::vector<int32_t> h_idx;          // [ns][k] internal ids, -1 = missing
    std::vector<int32_t> h_tris;         // [nt][3] internal ids
    std::vector<int64_t> h_boff;
    // device, internal order
    shell::DevArray<double> X;           // [nv][3]
    shell::DevArray<int32_t> tris;       // [nt][3]
    shell::DevArray<int32_t> perm_d;     // [nv]
    shell::DevArray<int32_t> idx;        // SoA [k][ns], a missing flap points at vertex 1
    shell::DevArray<double> B;           // SoA [r*k][ns], scaled by sqrt(stiffness)
    shell::DevArray<double> k0;          // SoA [r][ns]
    shell::DevArray<int32_t> flags;      // [ns]
    // FP64 plates with clamped edges: F0 = -(force of the clamped stencils at the rest shape) [nv][3] and
    // E0 = their energy there, which turn the plain plate force and energy into rest-relative ones
    shell::DevArray<double> bias;
    double bias_e0 = 0.0;
    // SHELL_FLAG_MEMBRANE: the triangles in the force tiles (halo copies repeat): ids [n][4], rest data
    // [n][6] (G = Dm^-1 row-major, area, 0), each tile's list [2 nblocks]; energy partials [nblocks]
    shell::DevArray<int32_t> mtid;
    shell::DevArray<double> mtrest, mepart;
    shell::DevArray<int64_t> mboff;
    shell::DevArray<int64_t> boff;       // [2 nblocks] start, end
    shell::DevArray<int32_t> tsrc;       // [nst_pad]
    // tiled streams, only those of the configured precision: [nst_pad / 64][chunks][64][fields per chunk]
    shell::DevArray<int32_t> tidx;       // FP64: vertex ids
    shell::DevArray<double> trec64;      // FP64: operator entries and rest curvatures
    shell::DevArray<float> trec32;       // mixed: ids (bit patterns), operator, rest curvatures
    // scratch for the caller-order entry point
    shell::DevArray<double> xin;         // [nv][3]
    shell::DevArray<double> fout;        // [nv][3] (float for mixed, sized in doubles)
    shell::DevArray<double> epart;       // [nblocks] energy partials
    shell::DevArray<shell::ForceDesc> fdesc;     // descriptor for the caller-order entry point
    shell::DevArray<shell::WorkItem> tile_items; // (0, tile) for every tile
};

struct shell_hessian_s {
    shell_stencils_s* st = nullptr;
    shell::SellPattern pat;
    shell::DevArray<int32_t> scol;       // [nslots]
    shell::DevArray<int32_t> width;      // [nslices]
    shell::DevArray<int64_t> sptr;       // [nslices+1]
    shell::DevArray<int32_t> rowlen;     // [nv]
    shell::DevArray<int32_t> gptr;       // [ngroups+1], empty when a group's column set is too large
    shell::DevArray<int32_t> gcols;
    shell::DevArray<uint16_t> lcol;      // [nslots]
    shell::DevArray<double> val;         // [nslots]
    shell::DevArray<float> valf;         // [nslots] mixed copy
    shell::DevArray<double> kdiag;       // [nv]
    shell::DevArray<double> pin, qout;   // caller-order scratch for hessian_apply
};


namespace shell {
// The implicit step of a shell with its membrane (SHELL_FLAG_MEMBRANE), float64: K_s as CSR, the membrane
// tangent as 3x3 blocks on the triangle adjacency, one PCG over all coordinates, line search.
struct MembraneSolve {
    DevArray<int64_t> srow;  // K_s CSR (internal order)
    DevArray<int32_t> scol;
    DevArray<double> sval;
    DevArray<int64_t> mrow;  // membrane block pattern: each vertex and its triangle neighbours, sorted
    DevArray<int32_t> mcol;
    // The tangent's 3x3 blocks, component (a, b) of block e at mval[mbase[e] + (3 a + b) mstride]: CSR
    // blocks one after the other (mbase = 9 e, mstride = 1), or, for the staged product, SELL-64 slices of
    // nine component arrays (mbase = the block's slot, mstride = the slot count)
    DevArray<int64_t> mbase;  // [nnz] base index of each CSR block
    DevArray<int64_t> mdiag;  // [nv] base index of the diagonal block
    int64_t mstride = 1;
    DevArray<double> mval;
    // staged product: rows in groups of kRowGroup, the group's directions staged in LDS.  K_s is read from
    // the bending Hessian's SELL slots and the blocks from their own SELL-64 slices (mptr, mwidth), each
    // slot's column an index into its group's list of the distinct columns of both matrices (gptr, gcols,
    // sorted); gself: the list index of the group's first row (its rows follow in order)
    bool staged = false;
    int32_t max_gcols = 0;
    DevArray<int32_t> gptr, gcols, gself, mwidth;
    DevArray<int64_t> mptr;
    DevArray<uint16_t> slcol, mlcol;
    DevArray<int64_t> s2e;  // [slots] the CSR block of each block slot, -1 on padding
    const int64_t* hsptr = nullptr;  // the bending Hessian's SELL slices and values (owned by the Hessian)
    const int32_t* hwidth = nullptr;
    const double* hval = nullptr;
    const float* hvalf = nullptr;
    DevArray<int32_t> brow;   // [nnz] the row of each block
    DevArray<int64_t> btptr;  // [nnz+1] the triangles holding both vertices of each block, ascending
    DevArray<int32_t> bttri;
    DevArray<double> rest;   // [nt][5] G = Dm^-1 and the rest area
    DevArray<double> xtry, ftry, z, p, p2, q, y, r, dinv, part;
    // mixed precision: the force kernels' float32 output (widened into ftry), and the float32 copies of
    // K_s and of the tangent's blocks that the product reads (in difference form)
    bool mixed = false;
    DevArray<float> ff, svalf, mvalf;
    DevArray<double> ppart;      // per-block partials of the PCG product's p.q
    DevArray<double> scal;   // device scalars of the PCG and the energies
    DevArray<double> mepart;     // the membrane tiles' energy partials (this simulation's own)
    DevArray<ForceDesc> fdesc;   // bending force at xtry with energy partials
    DevArray<WorkItem> items;
    int64_t ngroups = 0;
    bool pswap = false;          // which of p, p2 holds the current PCG direction
    // instantiated graphs of PCG chunks, keyed by what their kernel arguments bake in
    struct PcgGraph {
        const double* mass;
        double dt2;
        int count;
        bool parity;
        hipGraphExec_t ex;
    };
    std::vector<PcgGraph> graphs;  // oldest first
    hipStream_t capture = nullptr; // private stream the chunks are captured on
    // the step's host side, made on first use: a pinned copy of scal, the event marking it filled, and
    // the stream the simulation steps on inside a batch
    double* hscal = nullptr;
    hipEvent_t ready = nullptr;
    hipStream_t lane = nullptr;
    // device memory held by the arrays above
    size_t bytes() const {
        size_t n = 0;
        for (size_t v : {srow.bytes(), scol.bytes(), sval.bytes(), mrow.bytes(), mcol.bytes(), mbase.bytes(),
                         mdiag.bytes(), mval.bytes(), gptr.bytes(), gcols.bytes(), gself.bytes(), mwidth.bytes(),
                         mptr.bytes(), slcol.bytes(), mlcol.bytes(), s2e.bytes(), brow.bytes(), btptr.bytes(), bttri.bytes(),
                         rest.bytes(), xtry.bytes(), ftry.bytes(), z.bytes(), p.bytes(), p2.bytes(), q.bytes(),
                         y.bytes(), r.bytes(), dinv.bytes(), part.bytes(), ff.bytes(), svalf.bytes(), mvalf.bytes(),
                         ppart.bytes(), scal.bytes(), mepart.bytes(), fdesc.bytes(), items.bytes()})
            n += v;
        return n;
    }
    MembraneSolve() = default;
    MembraneSolve(const MembraneSolve&) = delete;
    MembraneSolve& operator=(const MembraneSolve&) = delete;
    ~MembraneSolve();
};
}  // namespace shell

struct shell_sim_s {
    shell_stencils_s* st = nullptr;
    shell_hessian_s* h = nullptr;
    int64_t nv = 0;
    int64_t step = 0;
    double dinv_dt = -1.0;               // dt the preconditioner was built for (0: the quasi-static K alone)
    hipStream_t last_stream = nullptr;
    shell::DevArray<double> x, v, xt, xhat, g, mass, y, r;
    shell::DevArray<double> y64;         // mixed only: float64 part of the PCG increment
    shell::DevArray<double> rq;          // mixed only, made on first use: (M + dt^2 K_s) y64 in float64
    shell::DevArray<double> f;           // float64 forces (or float32 in mixed, sized in doubles)
    shell::DevArray<double> dinv;        // [nv] (float in mixed)
    shell::DevArray<double> mq;          // [nv] mass for the product, -1 on fixed rows (float in mixed)
    shell::DevArray<uint8_t> pinned;     // [nv] held coordinates: bit c holds coordinate c, 7 the vertex
    bool partial_held = false;           // some vertex holds only part of its coordinates
    shell::DevArray<double> p, p2, q;    // PCG work vectors (float in mixed; sized in doubles)
    shell::DevArray<float> z;            // mixed only: the preconditioned residual, read by the product
    shell::DevArray<double> bins;        // PCG dot-product bins
    shell::DevArray<double> partials;    // reduction partials
    // quasi-static solves only: zero mass, the applied load (internal order), the Newton step's scale
    shell::DevArray<double> zmass, fext, ustep;
    shell_batch_s* solo = nullptr;       // this simulation alone, as a batch of one
    std::unique_ptr<shell::MembraneSolve> ms;  // stencils built with SHELL_FLAG_MEMBRANE
    shell_step_stats_t stats{};
};

// A set of simulations stepped together: one launch per phase covers all of them.
namespace shell {
// Sampled in-step kernel timing: event pairs recorded on the step's stream around sampled launches,
// read back after the step's own stream synchronisations.
struct StepProfiler {
    int every = 0;
    long counter = 0;
    struct Sample {
        int phase;
        hipEvent_t a, b;
    };
    std::vector<hipEvent_t> pool;
    std::vector<Sample> pending;
    double ms[SHELL_NUM_PHASES] = {};
    int64_t count[SHELL_NUM_PHASES] = {};
    hipEvent_t take();
    bool sample_iteration() { return every > 0 && (counter++ % every) == 0; }
    void drain();  // the stream must be synchronised
    void reset();
    ~StepProfiler();
};
}  // namespace shell

namespace shell {
// Instantiated HIP graphs of PCG chunks, keyed by everything their kernel arguments bake in (the
// buffers' contents are read when a graph runs, so the same key serves any meshes and step).
struct GraphCache {
    struct Key {
        const void* sdesc;
        const void* rows;
        long nrows, grid;
        size_t lds;
        int per, per_u, count, parity, precision;
        bool operator==(const Key& o) const {
            return sdesc == o.sdesc && rows == o.rows && nrows == o.nrows && grid == o.grid && lds == o.lds &&
                   per == o.per && per_u == o.per_u && count == o.count && parity == o.parity &&
                   precision == o.precision;
        }
    };
    std::vector<std::pair<Key, hipGraphExec_t>> entries;  // oldest first
    hipStream_t capture = nullptr;                        // private stream the chunks are captured on
    ~GraphCache();
};
}  // namespace shell

struct shell_batch_s {
    std::vector<shell_sim_s*> sims;
    std::unique_ptr<shell::StepProfiler> prof;  // null unless sampling was requested
    std::unique_ptr<shell::GraphCache> graphs;  // created on first use
    int precision = 0;
    int max_T = 0;
    size_t lds_spmv = 0;                     // staged p bytes per row group, largest over the members
    size_t capacity = 0;                     // meshes the descriptor buffers hold
    bool fdesc_dirty = true;
    shell::DevArray<shell::ForceDesc> fdesc;
    shell::DevArray<shell::SolveDesc> sdesc;
    shell::DevArray<shell::PcgState> state;    // two per mesh
    shell::PcgState* state_host = nullptr;
    shell::SolveDesc* sdesc_host = nullptr;  // pinned staging
    shell::ForceDesc* fdesc_host = nullptr;
    shell::WorkItem* items_host = nullptr;
    int32_t* mlist_host = nullptr;
    size_t items_cap = 0;
    shell::DevArray<shell::WorkItem> items;   // [rows | tiles of each model]
    shell::DevArray<int32_t> mlist;
    bool membrane = false;  // simulations with the membrane: the members' steps interleave on their own streams
};

namespace shell {
// precompute.hip
// bc: device [ns] boundary bits of the stencils (internal order)
void launch_precompute(shell_stencils_s& st, const int32_t* bc, hipStream_t s);
void launch_tile_copy(shell_stencils_s& st, const int32_t* bc, hipStream_t s);
// FP64 plates: st.bias and st.bias_e0 from the clamped stencils (synchronises s)
void launch_clamp_bias(shell_stencils_s& st, const int32_t* bc, hipStream_t s);
// forces.hip
// one launch per model over a list of (mesh, tile) items; lds_T = the largest tile among the meshes
// start/stop: events that receive the kernel's own begin and end times (null: none)
void launch_force_items(int model, int precision, const ForceDesc* descs, const WorkItem* items, long nitems,
                        int lds_T, hipStream_t s, hipEvent_t start = nullptr, hipEvent_t stop = nullptr);
// writes the descriptor *dst = d and the tile items (0, t), t < ntiles, from a kernel
void launch_write_force_desc(const ForceDesc& d, ForceDesc* dst, WorkItem* items, int64_t ntiles, hipStream_t s);
// energy = add + sum of the n partials (+ the m partials of `extra`, when given)
void launch_energy_finalize(const double* epart, int64_t n, double add, double* energy, hipStream_t s,
                            const double* extra = nullptr, int64_t m = 0);
// membrane.hip: rest data of the membrane (SHELL_FLAG_MEMBRANE); its force added into f (internal order,
// double or float per the stencils' precision) from the float64 positions pos
void launch_membrane_rest(shell_stencils_s& st, hipStream_t s);
// epart: where the tiles' energy partials go (the stencils' own array when null)
void launch_membrane_forces(shell_stencils_s& st, const double* pos, void* f, hipStream_t s, double* epart = nullptr);
// the implicit step with the membrane: set-up once per simulation, then one step (float64)
void membrane_sim_init(shell_sim_s& sim, hipStream_t s);
shell_status_t membrane_step(shell_sim_s& sim, const shell_step_params_t& p, shell_step_stats_t& out,
                             hipStream_t s);
// quasi-static Newton-Raphson with the membrane (eq 64): load = device [nv][3] internal order, or null
struct MembraneStatic {
    const double* load = nullptr;
    double eps_f = 0.0, eps_u = 0.0;
};
shell_status_t membrane_static(shell_sim_s& sim, const shell_step_params_t& p, const MembraneStatic& qs,
                               shell_step_stats_t& out, hipStream_t s);
void membrane_time_kernels(shell_sim_s& sim, double dt, int reps, shell_kernel_times_t& out, hipStream_t s);
// one implicit step of every member of a batch of simulations with the membrane (stats: [n])
shell_status_t membrane_batch_step(shell_batch_s& b, const shell_step_params_t* p, int nparams,
                                   shell_step_stats_t* stats, hipStream_t s);
void launch_gather_rows(const double* src, const int32_t* perm, double* dst, int64_t nv, hipStream_t s);
void launch_scatter_rows(const void* src, const int32_t* perm, void* dst, int64_t nv, bool f32, hipStream_t s);
// hessian.hip
void launch_assemble(shell_hessian_s& h, hipStream_t s);
void launch_apply(const shell_hessian_s& h, const double* mass, double dt2, const double* p, double* q,
                  hipStream_t s);
// solver.hip
void sim_alloc(shell_sim_s& sim);
void batch_init(shell_batch_s& b);
void batch_free_host(shell_batch_s& b);
void batch_release(shell_batch_s& b);
// Quasi-static Newton-Raphson (eq 64) in place of a time step: no mass, no predictor motion, the residual
// dPsi/dx - F with F the simulation's fext (when has_load), stop when ||r|| < eps_f, increments capped at
// eps_u (> 0) in the max norm; the velocity and the step counter are left alone.
struct StaticMode {
    double eps_f = 0.0, eps_u = 0.0;
    bool has_load = false;
};
shell_status_t batch_step(shell_batch_s& b, const shell_step_params_t* p, int nparams, shell_step_stats_t* stats,
                          hipStream_t s, const StaticMode* qs = nullptr);
void batch_time_kernels(shell_batch_s& b, double dt, int reps, shell_kernel_times_t& out, hipStream_t s);
void sim_mass(shell_sim_s& sim, hipStream_t s);
}  // namespace shell
