// Host-side mesh processing: validation, stencil enumeration (edge hinge, Sec. 4.3; triangle-centred
// stencil with flap i+3 across the edge opposite vertex i, Secs 4.4-4.5 and App. C), Morton vertex
// order, vertex tiles for the force kernel and the SELL-64 pattern of the constant Hessian.
#include <algorithm>
#include <cstring>
#include <numeric>
#include <thread>

#include "internal.hpp"

namespace shell {

namespace {

inline uint64_t dkey(int32_t from, int32_t to) { return (uint64_t(uint32_t(from)) << 32) | uint32_t(to); }

template <typename F>
void parallel_for(int64_t n, F&& fn) {
    unsigned nt = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
    if (n < 4096 || nt == 1) {
        fn(int64_t(0), n);
        return;
    }
    std::vector<std::thread> th;
    int64_t chunk = (n + nt - 1) / nt;
    for (unsigned t = 0; t < nt; ++t) {
        int64_t a = t * chunk, b = std::min(n, a + chunk);
        if (a < b) th.emplace_back([=, &fn] { fn(a, b); });
    }
    for (auto& t : th) t.join();
}

}  // namespace

HostTopology build_topology(int model, int64_t nv, int64_t nt, const int32_t* tris, int64_t n_clamped,
                            const int32_t* clamped) {
    HostTopology topo;
    topo.model = model;
    topo.k = model_k(model);
    // directed half-edges keyed by (from, to), each carrying the vertex opposite it
    std::vector<std::pair<uint64_t, int32_t>> he(size_t(3 * nt));
    for (int64_t t = 0; t < nt; ++t) {
        const int32_t* v = tris + 3 * t;
        for (int c = 0; c < 3; ++c)
            SHELL_CHECK(v[c] >= 0 && v[c] < nv, SHELL_E_INVALID_ARG, "triangle vertex id out of range");
        SHELL_CHECK(v[0] != v[1] && v[1] != v[2] && v[0] != v[2], SHELL_E_DEGENERATE,
                    "triangle with a repeated vertex");
        he[3 * t + 0] = {dkey(v[0], v[1]), v[2]};
        he[3 * t + 1] = {dkey(v[1], v[2]), v[0]};
        he[3 * t + 2] = {dkey(v[2], v[0]), v[1]};
    }
    std::sort(he.begin(), he.end());
    auto find = [&](int32_t from, int32_t to) -> const std::pair<uint64_t, int32_t>* {
        uint64_t k = dkey(from, to);
        auto it = std::lower_bound(he.begin(), he.end(), std::make_pair(k, INT32_MIN));
        return (it != he.end() && it->first == k) ? &*it : nullptr;
    };
    for (size_t i = 1; i < he.size(); ++i) {
        if (he[i].first == he[i - 1].first) {
            int32_t from = int32_t(he[i].first >> 32), to = int32_t(he[i].first & 0xffffffffu);
            bool fan = find(to, from) != nullptr;
            throw Error(fan ? SHELL_E_NONMANIFOLD : SHELL_E_ORIENTATION,
                        fan ? "edge shared by more than two triangles" : "inconsistently oriented triangles");
        }
    }
    // clamped edges as undirected keys; each must be traversed by exactly one triangle
    std::vector<uint64_t> ckeys(static_cast<size_t>(n_clamped));
    for (int64_t e = 0; e < n_clamped; ++e) {
        const int32_t u = clamped[2 * e], v = clamped[2 * e + 1];
        SHELL_CHECK(u >= 0 && u < nv && v >= 0 && v < nv, SHELL_E_INVALID_ARG, "clamped edge vertex out of range");
        SHELL_CHECK((find(u, v) != nullptr) + (find(v, u) != nullptr) == 1, SHELL_E_INVALID_ARG,
                    "a clamped edge is not a boundary edge of the mesh");
        ckeys[size_t(e)] = dkey(std::min(u, v), std::max(u, v));
    }
    std::sort(ckeys.begin(), ckeys.end());
    auto is_clamped = [&](int32_t u, int32_t v) {
        return std::binary_search(ckeys.begin(), ckeys.end(), dkey(std::min(u, v), std::max(u, v)));
    };
    if (model_is_edge(model)) {
        // one stencil per interior edge; 2->3 is the half-edge with the smaller source id
        for (const auto& h : he) {
            int32_t from = int32_t(h.first >> 32), to = int32_t(h.first & 0xffffffffu);
            if (from > to) continue;
            const auto* twin = find(to, from);
            if (!twin) continue;  // boundary edge: free, no stencil
            topo.idx.insert(topo.idx.end(), {h.second, from, to, twin->second});
        }
        topo.bc.assign(topo.idx.size() / 4, 0);
        if (!model_is_shell(model) && n_clamped > 0) {
            // clamped boundary edge of the plate: (L, M, N, virtual), M->N as its triangle traverses it
            for (const auto& h : he) {
                int32_t from = int32_t(h.first >> 32), to = int32_t(h.first & 0xffffffffu);
                if (find(to, from) || !is_clamped(from, to)) continue;
                topo.idx.insert(topo.idx.end(), {h.second, from, to, -1});
                topo.bc.push_back(kBcEdgeClamped);
            }
        }
        topo.ns = int64_t(topo.idx.size() / 4);
    } else {
        topo.ns = nt;
        topo.idx.resize(size_t(6 * nt));
        topo.bc.assign(size_t(nt), 0);
        for (int64_t t = 0; t < nt; ++t) {
            const int32_t* v = tris + 3 * t;
            int32_t* s = topo.idx.data() + 6 * t;
            s[0] = v[0];
            s[1] = v[1];
            s[2] = v[2];
            int32_t bits = 0;
            for (int i = 0; i < 3; ++i) {
                const auto* nb = find(v[(i + 2) % 3], v[(i + 1) % 3]);
                s[3 + i] = nb ? nb->second : -1;
                if (!nb) bits |= (1 << i) | (is_clamped(v[(i + 1) % 3], v[(i + 2) % 3]) ? 1 << (3 + i) : 0);
            }
            topo.bc[size_t(t)] = bits;
        }
    }
    return topo;
}

namespace {

uint64_t morton3(const double* p, const double* lo, double ext) {
    auto spread = [](uint64_t v) {  // 21 bits -> every third bit
        v &= 0x1fffff;
        v = (v | v << 32) & 0x1f00000000ffffull;
        v = (v | v << 16) & 0x1f0000ff0000ffull;
        v = (v | v << 8) & 0x100f00f00f00f00full;
        v = (v | v << 4) & 0x10c30c30c30c30c3ull;
        v = (v | v << 2) & 0x1249249249249249ull;
        return v;
    };
    uint64_t q[3];
    for (int c = 0; c < 3; ++c) q[c] = uint64_t((p[c] - lo[c]) / ext * 2097151.0);
    return spread(q[0]) | spread(q[1]) << 1 | spread(q[2]) << 2;
}

// Recursive coordinate bisection: split the vertex range along its longest axis so that the left part
// holds a whole number of tiles, until a range fits one tile; tiles come out as compact patches of the
// surface whatever its curvature.  Ties are broken by vertex id, so the order is deterministic.
void rcb(std::vector<int32_t>& perm, int64_t a, int64_t b, const double* X, int T) {
    if (b - a <= T) return;
    double lo[3], hi[3];
    for (int c = 0; c < 3; ++c) lo[c] = hi[c] = X[3 * int64_t(perm[size_t(a)]) + c];
    for (int64_t i = a; i < b; ++i)
        for (int c = 0; c < 3; ++c) {
            double v = X[3 * int64_t(perm[size_t(i)]) + c];
            lo[c] = std::min(lo[c], v);
            hi[c] = std::max(hi[c], v);
        }
    int ax = 0;
    for (int c = 1; c < 3; ++c)
        if (hi[c] - lo[c] > hi[ax] - lo[ax]) ax = c;
    int64_t tiles = (b - a + T - 1) / T;
    int64_t mid = a + ((tiles + 1) / 2) * T;
    std::nth_element(perm.begin() + a, perm.begin() + mid, perm.begin() + b, [&](int32_t u, int32_t v) {
        double pu = X[3 * int64_t(u) + ax], pv = X[3 * int64_t(v) + ax];
        return pu < pv || (pu == pv && u < v);
    });
    rcb(perm, a, mid, X, T);
    rcb(perm, mid, b, X, T);
}

}  // namespace

std::vector<int32_t> vertex_order(const double* X, int64_t nv, int mode, int T) {
    std::vector<int32_t> perm(static_cast<size_t>(nv));
    std::iota(perm.begin(), perm.end(), 0);
    if (mode == 0 || nv < 2) return perm;
    double lo[3], hi[3];
    for (int c = 0; c < 3; ++c) lo[c] = hi[c] = X[c];
    for (int64_t i = 0; i < nv; ++i)
        for (int c = 0; c < 3; ++c) {
            lo[c] = std::min(lo[c], X[3 * i + c]);
            hi[c] = std::max(hi[c], X[3 * i + c]);
        }
    double ext = std::max({hi[0] - lo[0], hi[1] - lo[1], hi[2] - lo[2], 1e-300});
    std::vector<uint64_t> code(static_cast<size_t>(nv));
    for (int64_t i = 0; i < nv; ++i) code[size_t(i)] = morton3(X + 3 * i, lo, ext);
    // Morton order first (it also orders the vertices inside each bisection tile)
    std::stable_sort(perm.begin(), perm.end(), [&](int32_t a, int32_t b) { return code[a] < code[b]; });
    if (mode == 1) {
        rcb(perm, 0, nv, X, T);
        for (int64_t a = 0; a < nv; a += T)
            std::sort(perm.begin() + a, perm.begin() + std::min<int64_t>(nv, a + T),
                      [&](int32_t u, int32_t v) { return code[u] < code[v] || (code[u] == code[v] && u < v); });
    }
    return perm;
}

Tiling build_tiling(const std::vector<int32_t>& idx, int k, int64_t ns, int64_t nv, int T) {
    Tiling t;
    t.T = T;
    t.nblocks = std::max<int64_t>(1, (nv + T - 1) / T);
    std::vector<int64_t> cnt(size_t(t.nblocks + 1), 0);
    auto blocks_of = [&](int64_t s, int32_t* out) {
        int n = 0;
        for (int j = 0; j < k; ++j) {
            int32_t v = idx[size_t(k * s + j)];
            if (v < 0) continue;
            int32_t b = v / T;
            bool seen = false;
            for (int q = 0; q < n; ++q) seen |= out[q] == b;
            if (!seen) out[n++] = b;
        }
        return n;
    };
    int32_t bl[6];
    for (int64_t s = 0; s < ns; ++s) {
        int n = blocks_of(s, bl);
        for (int q = 0; q < n; ++q) cnt[size_t(bl[q]) + 1]++;
    }
    // each tile's list starts on a 64-stencil block
    t.boff.assign(size_t(2 * t.nblocks), 0);
    int64_t at = 0;
    for (int64_t b = 0; b < t.nblocks; ++b) {
        t.boff[size_t(2 * b)] = at;
        t.boff[size_t(2 * b + 1)] = at + cnt[b + 1];
        t.count += cnt[b + 1];
        at = (at + cnt[b + 1] + kStreamBlock - 1) / kStreamBlock * kStreamBlock;
    }
    t.src.assign(size_t(at), -1);
    std::vector<int64_t> fill(size_t(t.nblocks));
    for (int64_t b = 0; b < t.nblocks; ++b) fill[size_t(b)] = t.boff[size_t(2 * b)];
    for (int64_t s = 0; s < ns; ++s) {
        int n = blocks_of(s, bl);
        for (int q = 0; q < n; ++q) t.src[size_t(fill[size_t(bl[q])]++)] = int32_t(s);
    }
    return t;
}

SellPattern build_sell_pattern(const std::vector<int32_t>& idx, int k, int64_t ns, int64_t nv, bool staging) {
    SellPattern P;
    P.nv = nv;
    // vertex -> incident stencils
    std::vector<int64_t> vptr(size_t(nv + 1), 0);
    for (int64_t s = 0; s < ns; ++s)
        for (int j = 0; j < k; ++j)
            if (idx[size_t(k * s + j)] >= 0) vptr[size_t(idx[size_t(k * s + j)]) + 1]++;
    for (int64_t v = 0; v < nv; ++v) vptr[v + 1] += vptr[v];
    std::vector<int32_t> vst(static_cast<size_t>(vptr[nv]));
    {
        std::vector<int64_t> fill(vptr.begin(), vptr.end() - 1);
        for (int64_t s = 0; s < ns; ++s)
            for (int j = 0; j < k; ++j) {
                int32_t v = idx[size_t(k * s + j)];
                if (v >= 0) vst[size_t(fill[v]++)] = int32_t(s);
            }
    }
    // row patterns: the union of the incident stencils' vertices
    std::vector<int32_t> len(size_t(nv), 0);
    parallel_for(nv, [&](int64_t a, int64_t b) {
        std::vector<int32_t> buf;
        for (int64_t v = a; v < b; ++v) {
            buf.clear();
            for (int64_t e = vptr[v]; e < vptr[v + 1]; ++e)
                for (int j = 0; j < k; ++j) {
                    int32_t u = idx[size_t(k * vst[size_t(e)] + j)];
                    if (u >= 0) buf.push_back(u);
                }
            std::sort(buf.begin(), buf.end());
            len[size_t(v)] = int32_t(std::unique(buf.begin(), buf.end()) - buf.begin());
        }
    });
    P.rowptr.assign(size_t(nv + 1), 0);
    for (int64_t v = 0; v < nv; ++v) P.rowptr[v + 1] = P.rowptr[v] + len[size_t(v)];
    P.nnz = P.rowptr[nv];
    P.col.resize(size_t(P.nnz));
    parallel_for(nv, [&](int64_t a, int64_t b) {
        std::vector<int32_t> buf;
        for (int64_t v = a; v < b; ++v) {
            buf.clear();
            for (int64_t e = vptr[v]; e < vptr[v + 1]; ++e)
                for (int j = 0; j < k; ++j) {
                    int32_t u = idx[size_t(k * vst[size_t(e)] + j)];
                    if (u >= 0) buf.push_back(u);
                }
            std::sort(buf.begin(), buf.end());
            buf.erase(std::unique(buf.begin(), buf.end()), buf.end());
            std::copy(buf.begin(), buf.end(), P.col.begin() + P.rowptr[v]);
        }
    });
    // SELL-64: slice s holds rows 64s..64s+63, entry q of row i at sptr[s] + 64 q + (i mod 64)
    P.nslices = (nv + 63) / 64;
    P.width.assign(size_t(P.nslices), 0);
    P.sptr.assign(size_t(P.nslices + 1), 0);
    P.rowlen = len;
    for (int64_t s = 0; s < P.nslices; ++s) {
        int w = 0;
        for (int64_t i = 64 * s; i < std::min(nv, 64 * s + 64); ++i) w = std::max(w, len[size_t(i)]);
        P.width[size_t(s)] = std::max(w, 1);
        P.sptr[s + 1] = P.sptr[s] + 64 * int64_t(P.width[size_t(s)]);
    }
    P.nslots = P.sptr[P.nslices];
    P.scol.assign(size_t(P.nslots), 0);
    P.csr2sell.resize(size_t(P.nnz));
    P.dslot.assign(size_t(nv), -1);
    for (int64_t s = 0; s < P.nslices; ++s) {
        for (int lane = 0; lane < 64; ++lane) {
            int64_t i = 64 * s + lane;
            int32_t last = i < nv ? int32_t(i) : 0;
            for (int q = 0; q < P.width[size_t(s)]; ++q) {
                int64_t slot = P.sptr[s] + 64 * q + lane;
                if (i < nv && q < len[size_t(i)]) {
                    int64_t e = P.rowptr[i] + q;
                    last = P.col[size_t(e)];
                    P.csr2sell[size_t(e)] = slot;
                    if (last == i) P.dslot[size_t(i)] = slot;
                }
                P.scol[size_t(slot)] = last;  // padding repeats the last column with a zero value
            }
        }
    }
    // distinct columns of each row group, and each slot's index into its group's list
    const int64_t ng = (nv + kRowGroup - 1) / kRowGroup;
    P.gptr.assign(size_t(ng + 1), 0);
    std::vector<std::vector<int32_t>> gl(static_cast<size_t>(ng));
    parallel_for(ng, [&](int64_t a, int64_t b) {
        for (int64_t g = a; g < b; ++g) {
            auto& v = gl[size_t(g)];
            for (int64_t i = g * kRowGroup; i < std::min(nv, (g + 1) * kRowGroup); ++i) {
                v.insert(v.end(), P.col.begin() + P.rowptr[i], P.col.begin() + P.rowptr[i + 1]);
                if (P.rowptr[i] == P.rowptr[i + 1]) v.push_back(int32_t(i));  // an empty row pads with itself
            }
            std::sort(v.begin(), v.end());
            v.erase(std::unique(v.begin(), v.end()), v.end());
        }
    });
    for (int64_t g = 0; g < ng; ++g) {
        P.gptr[size_t(g + 1)] = P.gptr[size_t(g)] + int32_t(gl[size_t(g)].size());
        P.max_gcols = std::max<int32_t>(P.max_gcols, int32_t(gl[size_t(g)].size()));
    }
    if (staging && P.max_gcols <= kMaxGroupCols) {
        P.gcols.reserve(size_t(P.gptr[size_t(ng)]));
        for (const auto& v : gl) P.gcols.insert(P.gcols.end(), v.begin(), v.end());
        P.lcol.assign(size_t(P.nslots), 0);
        parallel_for(P.nslices, [&](int64_t a, int64_t b) {
            for (int64_t sl = a; sl < b; ++sl) {
                const auto& v = gl[size_t((64 * sl) / kRowGroup)];
                for (int64_t slot = P.sptr[sl]; slot < P.sptr[sl + 1]; ++slot) {
                    int32_t c = P.scol[size_t(slot)];
                    auto it = std::lower_bound(v.begin(), v.end(), c);
                    // rows past nv in the last slice pad with column 0, which may be absent: use entry 0
                    P.lcol[size_t(slot)] = (it != v.end() && *it == c) ? uint16_t(it - v.begin()) : uint16_t(0);
                }
            }
        });
    } else {
        P.gptr.clear();
    }
    return P;
}

Incidence build_incidence(const std::vector<int32_t>& idx, int k, int64_t n, int64_t nv) {
    Incidence inc;
    inc.ptr.assign(size_t(nv + 1), 0);
    for (int64_t t = 0; t < n; ++t)
        for (int j = 0; j < k; ++j) {
            const int32_t v = idx[size_t(k * t + j)];
            if (v >= 0) ++inc.ptr[size_t(v) + 1];
        }
    for (int64_t v = 0; v < nv; ++v) inc.ptr[size_t(v + 1)] += inc.ptr[size_t(v)];
    inc.code.resize(size_t(inc.ptr[size_t(nv)]));
    std::vector<int64_t> fill(inc.ptr.begin(), inc.ptr.end() - 1);
    for (int64_t t = 0; t < n; ++t)
        for (int j = 0; j < k; ++j) {
            const int32_t v = idx[size_t(k * t + j)];
            if (v >= 0) inc.code[size_t(fill[size_t(v)]++)] = t * 8 + j;
        }
    return inc;
}

}  // namespace shell
