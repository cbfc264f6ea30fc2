// Constant bending Hessian K = K_s (x) I3 (eqs 21, 41, 53; the shell models reuse it), assembled once,
// and its product inside the implicit step.
//
// K_s = sum over stencils of P^T G P with G = B^T D B (k x k): every stencil block of the paper's
// Hessian is G (x) I3, so only the scalar K_s is stored.  Storage is SELL-64: slice s holds rows
// 64s..64s+63 and entry q of row i sits at sptr[s] + 64 q + (i mod 64), so the 64 lanes of a wave read
// 64 consecutive values and column ids per step (fully coalesced), one row per lane, no reduction.
#include "devmath.hpp"
#include "internal.hpp"
#include "spmv.hpp"

namespace shell {

namespace {

// slot of column c in row i (columns sorted within the row's rowlen entries)
__device__ __forceinline__ long find_slot(const int32_t* __restrict__ scol, const int64_t* __restrict__ sptr,
                                          const int32_t* __restrict__ rowlen, long i, int c) {
    long s0 = sptr[i >> 6] + (i & 63);
    int lo = 0, hi = rowlen[i] - 1;
    while (lo < hi) {
        int mid = (lo + hi) >> 1;
        if (scol[s0 + 64L * mid] < c)
            lo = mid + 1;
        else
            hi = mid;
    }
    return s0 + 64L * lo;
}

// Row i of K_s: over the stencils that contain vertex i (as local vertex j), in ascending order, row j of
// the stencil's block B^T D B.  One thread per row writes only its own slots, so the sums take the same
// order in every run.
template <int K, int R>
__global__ void assemble_rows(const int64_t* __restrict__ inc_ptr, const int64_t* __restrict__ inc,
                              const int32_t* __restrict__ idx, const double* __restrict__ B, long ns,
                              const int32_t* __restrict__ missing, double kb, double nu,
                              const int32_t* __restrict__ scol, const int64_t* __restrict__ sptr,
                              const int32_t* __restrict__ rowlen, long nv, double* __restrict__ val) {
    const long i = blockIdx.x * long(blockDim.x) + threadIdx.x;
    if (i >= nv) return;
    for (int64_t e = inc_ptr[i]; e < inc_ptr[i + 1]; ++e) {
        const long s = long(inc[e] >> 3);
        const int j = int(inc[e] & 7);
        int v[K];
        double Bm[R][K];
        for (int l = 0; l < K; ++l) v[l] = idx[l * ns + s];
        for (int r = 0; r < R; ++r)
            for (int l = 0; l < K; ++l) Bm[r][l] = B[(r * K + l) * ns + s];
        const int miss = missing ? missing[s] : 0;
        // D B (the stiffness is already folded into B for edges; triangles carry D_b)
        double DB[R][K];
        if constexpr (R == 1) {
            for (int l = 0; l < K; ++l) DB[0][l] = Bm[0][l];
        } else {
            const double t = 0.5 * (1.0 - nu);
            for (int l = 0; l < K; ++l) {
                DB[0][l] = kb * (Bm[0][l] + nu * Bm[1][l]);
                DB[1][l] = kb * (nu * Bm[0][l] + Bm[1][l]);
                DB[2][l] = kb * t * Bm[2][l];
            }
        }
        for (int l = 0; l < K; ++l) {
            if (l >= 3 && (miss & (1 << (l - 3)))) continue;
            double g = 0.0;
            for (int r = 0; r < R; ++r) g += Bm[r][j] * DB[r][l];
            val[find_slot(scol, sptr, rowlen, i, v[l])] += g;
        }
    }
}

__global__ void fill_zero(double* __restrict__ p, long n) {
    long i = blockIdx.x * long(blockDim.x) + threadIdx.x;
    if (i < n) p[i] = 0.0;
}

__global__ void extract_diag(const double* __restrict__ val, const int64_t* __restrict__ dslot, long nv,
                             double* __restrict__ kdiag) {
    long i = blockIdx.x * long(blockDim.x) + threadIdx.x;
    if (i < nv) kdiag[i] = dslot[i] >= 0 ? val[dslot[i]] : 0.0;
}

__global__ void to_float(const double* __restrict__ a, float* __restrict__ b, long n) {
    long i = blockIdx.x * long(blockDim.x) + threadIdx.x;
    if (i < n) b[i] = float(a[i]);
}

// q = diag(mass) p + dt2 K_s p over 3 columns (caller order handled by the host wrapper)
__global__ void apply_sell(const int32_t* __restrict__ scol, const double* __restrict__ val,
                           const int64_t* __restrict__ sptr, const int32_t* __restrict__ width,
                           const int32_t* __restrict__ gptr, const int32_t* __restrict__ gcols,
                           const uint16_t* __restrict__ lcol, long nv, const double* __restrict__ mass, double dt2,
                           const double* __restrict__ p, double* __restrict__ q) {
    long i = blockIdx.x * long(blockDim.x) + threadIdx.x;
    extern __shared__ unsigned char smem_raw[];
    double* ps = reinterpret_cast<double*>(smem_raw);
    if (gptr) {
        stage_group_columns<double>(gptr, gcols, blockIdx.x, p, ps);
        __syncthreads();
    }
    if (i >= nv) return;
    double ax, ay, az;
    if (gptr)
        sell_row_product_staged<double, double>(lcol, val, sptr, width, i, ps, ax, ay, az);
    else
        sell_row_product<double, double>(scol, val, sptr, width, i, p, ax, ay, az);
    double m = mass ? mass[i] : 0.0;
    q[3 * i] = fma(m, p[3 * i], dt2 * ax);
    q[3 * i + 1] = fma(m, p[3 * i + 1], dt2 * ay);
    q[3 * i + 2] = fma(m, p[3 * i + 2], dt2 * az);
}

}  // namespace

void launch_assemble(shell_hessian_s& h, hipStream_t s) {
    shell_stencils_s& st = *h.st;
    const long nslots = h.pat.nslots;
    fill_zero<<<(nslots + 255) / 256, 256, 0, s>>>(h.val.p, nslots);
    SHELL_HIP(hipGetLastError());
    const long ns = st.ns;
    DevArray<int32_t> md;
    if (!model_is_edge(st.model) && ns) {
        std::vector<int32_t> mask(size_t(ns), 0);
        for (long q = 0; q < ns; ++q)
            for (int L = 0; L < 3; ++L)
                if (st.h_idx[size_t(6 * q + 3 + L)] < 0) mask[size_t(q)] |= 1 << L;
        md.alloc(size_t(ns));
        md.upload(mask.data(), size_t(ns), s);
    }
    if (ns) {
        const Incidence inc = build_incidence(st.h_idx, st.k, ns, st.nv);
        DevArray<int64_t> iptr(inc.ptr.size()), icode(std::max<size_t>(inc.code.size(), 1));
        iptr.upload(inc.ptr.data(), inc.ptr.size(), s);
        icode.upload(inc.code.data(), inc.code.size(), s);
        const long grid = (st.nv + 255) / 256;
        if (model_is_edge(st.model))
            assemble_rows<4, 1><<<grid, 256, 0, s>>>(iptr.p, icode.p, st.idx.p, st.B.p, ns, nullptr, st.kb,
                                                     st.poisson, h.scol.p, h.sptr.p, h.rowlen.p, st.nv, h.val.p);
        else
            assemble_rows<6, 3><<<grid, 256, 0, s>>>(iptr.p, icode.p, st.idx.p, st.B.p, ns, md.p, st.kb,
                                                     st.poisson, h.scol.p, h.sptr.p, h.rowlen.p, st.nv, h.val.p);
        SHELL_HIP(hipGetLastError());
        SHELL_HIP(hipStreamSynchronize(s));  // the incidence lists are released on return
    }
    DevArray<int64_t> dslot(static_cast<size_t>(st.nv));
    dslot.upload(h.pat.dslot.data(), size_t(st.nv), s);
    if (st.nv) {
        extract_diag<<<(st.nv + 255) / 256, 256, 0, s>>>(h.val.p, dslot.p, st.nv, h.kdiag.p);
        SHELL_HIP(hipGetLastError());
    }
    if (h.valf.p) {
        to_float<<<(nslots + 255) / 256, 256, 0, s>>>(h.val.p, h.valf.p, nslots);
        SHELL_HIP(hipGetLastError());
    }
    SHELL_HIP(hipStreamSynchronize(s));  // temporaries are released on return
}

void launch_apply(const shell_hessian_s& h, const double* mass, double dt2, const double* p, double* q,
                  hipStream_t s) {
    const long nv = h.pat.nv;
    if (!nv) return;
    size_t lds = h.gptr.p ? size_t(h.pat.max_gcols) * 3 * sizeof(double) : 0;
    apply_sell<<<(nv + kRowGroup - 1) / kRowGroup, kRowGroup, lds, s>>>(h.scol.p, h.val.p, h.sptr.p, h.width.p,
                                                                      h.gptr.p, h.gcols.p, h.lcol.p, nv, mass, dt2,
                                                                      p, q);
    SHELL_HIP(hipGetLastError());
}

}  // namespace shell
