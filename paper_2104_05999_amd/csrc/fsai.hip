// Factored sparse approximate inverse (Kolotilina-Yeremin FSAI), used where
// the paper uses hypre's ParaSails sparse approximate inverse (Section 2.3).
//
// G is lower triangular with the static pattern S_i = {j <= i : A_ij stored}
// (the lower half of L's pattern, zero entries included).  Row i of G is
// y / sqrt(y_i) with A[S_i, S_i] y = e_i, so that G A G^T has a unit
// diagonal; with A[S_i, S_i] = L L^T (Cholesky) that row is L^-T e_i.
// The preconditioner is M^-1 = G^T G.  G^T is stored as its own CSR: by the
// symmetry of the pattern, row j of G^T has the columns of row j of A that
// are >= j.  The dense per-row systems live in a global workspace (packed
// lower triangles), so the pattern size is not limited.
#include "solver.h"

namespace {

__global__ void k_fsai_lengths(int64_t V, const int32_t* __restrict__ row_ptr, const int32_t* __restrict__ diag_pos,
                               int32_t* __restrict__ glen, int32_t* __restrict__ gtlen, int32_t* __restrict__ wlen) {
    GRID_STRIDE_LOOP(i, V) {
        const int32_t m = diag_pos[i] - row_ptr[i] + 1;
        glen[i] = m;
        gtlen[i] = row_ptr[i + 1] - diag_pos[i];
        wlen[i] = m * (m + 1) / 2;
    }
}

__global__ void k_fsai_pattern(int64_t V, const int32_t* __restrict__ row_ptr, const int32_t* __restrict__ col,
                               const int32_t* __restrict__ diag_pos, const int64_t* __restrict__ g_ptr,
                               const int64_t* __restrict__ gt_ptr, int32_t* __restrict__ g_col,
                               int32_t* __restrict__ gt_col, int32_t* __restrict__ gt_src) {
    GRID_STRIDE_LOOP(i, V) {
        const int32_t b = row_ptr[i], d = diag_pos[i], e = row_ptr[i + 1];
        for (int32_t k = b; k <= d; ++k) g_col[g_ptr[i] + (k - b)] = col[k];
        for (int32_t k = d; k < e; ++k) {
            const int32_t c = col[k];  // entry (i, c) of G^T is G[c][i]
            gt_col[gt_ptr[i] + (k - d)] = c;
            int32_t lo = row_ptr[c], hi = diag_pos[c], pos = -1;
            while (lo <= hi) {
                const int32_t mid = (lo + hi) >> 1;
                const int32_t cm = col[mid];
                if (cm == (int32_t)i) {
                    pos = mid;
                    break;
                }
                if (cm < (int32_t)i)
                    lo = mid + 1;
                else
                    hi = mid - 1;
            }
            gt_src[gt_ptr[i] + (k - d)] = pos < 0 ? -1 : (int32_t)(g_ptr[c] + (pos - row_ptr[c]));
        }
    }
}

__device__ __forceinline__ double lookup(const int32_t* __restrict__ row_ptr, const int32_t* __restrict__ col,
                                         const double* __restrict__ val, int32_t r, int32_t c) {
    int32_t lo = row_ptr[r], hi = row_ptr[r + 1] - 1;
    while (lo <= hi) {
        const int32_t mid = (lo + hi) >> 1;
        const int32_t cm = col[mid];
        if (cm == c) return val[mid];
        if (cm < c)
            lo = mid + 1;
        else
            hi = mid - 1;
    }
    return 0.0;
}

// packed lower triangle: element (a, b), b <= a, at a(a+1)/2 + b
__device__ __forceinline__ int64_t tri(int a, int b) { return (int64_t)a * (a + 1) / 2 + b; }

__global__ void k_fsai_values(int64_t V, const int32_t* __restrict__ row_ptr, const int32_t* __restrict__ col,
                              const double* __restrict__ val, const int32_t* __restrict__ diag_pos,
                              const int64_t* __restrict__ g_ptr, const int64_t* __restrict__ w_ptr,
                              double* __restrict__ work, double* __restrict__ g64, float* __restrict__ g32,
                              unsigned* __restrict__ err) {
    GRID_STRIDE_LOOP(i, V) {
        const int32_t b = row_ptr[i];
        const int m = diag_pos[i] - b + 1;
        const int32_t* S = col + b;
        double* Lw = work + w_ptr[i];
        // A[S, S], lower triangle
        for (int a = 0; a < m; ++a)
            for (int c = 0; c <= a; ++c) Lw[tri(a, c)] = lookup(row_ptr, col, val, S[a], S[c]);
        // Cholesky, in place
        bool ok = true;
        for (int j = 0; j < m && ok; ++j) {
            double d = Lw[tri(j, j)];
            for (int k = 0; k < j; ++k) d -= Lw[tri(j, k)] * Lw[tri(j, k)];
            if (!(d > 0.0)) {
                ok = false;
                break;
            }
            const double ljj = sqrt(d);
            Lw[tri(j, j)] = ljj;
            for (int a = j + 1; a < m; ++a) {
                double s = Lw[tri(a, j)];
                for (int k = 0; k < j; ++k) s -= Lw[tri(a, k)] * Lw[tri(j, k)];
                Lw[tri(a, j)] = s / ljj;
            }
        }
        double* g = g64 + g_ptr[i];
        if (!ok) {
            atomicOr(err, 1u);
            for (int a = 0; a < m; ++a) g[a] = 0.0;
            continue;
        }
        // L^T g = e_m, back substitution (g written in place, last entry first)
        for (int a = m - 1; a >= 0; --a) {
            double s = (a == m - 1) ? 1.0 : 0.0;
            for (int c = a + 1; c < m; ++c) s -= Lw[tri(c, a)] * g[c];
            g[a] = s / Lw[tri(a, a)];
        }
        for (int a = 0; a < m; ++a) g32[g_ptr[i] + a] = static_cast<float>(g[a]);
    }
}

__global__ void k_fsai_transpose_values(int64_t n, const int32_t* __restrict__ src, const double* __restrict__ g64,
                                        double* __restrict__ gt64, float* __restrict__ gt32) {
    GRID_STRIDE_LOOP(k, n) {
        const int32_t s = src[k];
        const double v = s >= 0 ? g64[s] : 0.0;
        gt64[k] = v;
        gt32[k] = static_cast<float>(v);
    }
}

// Sliced-ELL copy of a CSR matrix: per-slice width (one wavefront per slice,
// the maximum of its 64 row lengths), then the entries of each row in CSR
// order, column-major inside the slice; padding repeats the row's own column
// with value 0.
__global__ __launch_bounds__(BLOCK) void k_csr_sell_width(int64_t V, int64_t nslices, const int32_t* __restrict__ ptr,
                                                          int32_t* __restrict__ width64) {
    static_assert(SELL_C == 64, "one slice per wavefront");
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    int64_t s0, s1;
    block_range(nslices, &s0, &s1);
    for (int64_t s = s0 + w; s < s1; s += BLOCK / 64) {
        const int64_t r = s * SELL_C + lane;
        int wmax = r < V ? ptr[r + 1] - ptr[r] : 0;
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) wmax = max(wmax, __shfl_xor(wmax, off, 64));
        if (lane == 0) width64[s] = wmax * SELL_C;
    }
}

__global__ void k_csr_sell_fill(int64_t V, int64_t nslices, const int32_t* __restrict__ ptr,
                                const int32_t* __restrict__ col, const double* __restrict__ v64,
                                const float* __restrict__ v32, const int64_t* __restrict__ sptr,
                                int32_t* __restrict__ scol, double* __restrict__ s64, float* __restrict__ s32) {
    RANGE_LOOP(r, nslices * SELL_C) {
        const int64_t s = r / SELL_C;
        const int lane = static_cast<int>(r % SELL_C);
        const int width = static_cast<int>((sptr[s + 1] - sptr[s]) / SELL_C);
        const int32_t pad = static_cast<int32_t>(r < V ? r : V - 1);
        int j = 0;
        if (r < V) {
            for (int32_t k = ptr[r]; k < ptr[r + 1]; ++k, ++j) {
                const int64_t idx = sell_index(sptr[s], width, j, lane);
                scol[idx] = col[k];
                s64[idx] = v64[k];
                s32[idx] = v32[k];
            }
        }
        for (; j < width; ++j) {
            const int64_t idx = sell_index(sptr[s], width, j, lane);
            scol[idx] = pad;
            s64[idx] = 0.0;
            s32[idx] = 0.0f;
        }
    }
}

}  // namespace

// Sliced-ELL copy of a CSR matrix (also used for the tet systems).
void build_sell_copy(dec_ctx* ctx, int64_t V, int64_t nnz, const int32_t* ptr, const int32_t* col, const double* v64,
                     const float* v32, SellMatrix& S) {
    hipStream_t s = ctx->stream;
    S.nslices = (V + SELL_C - 1) / SELL_C;
    DBuf<int32_t> w;
    w.alloc(ctx, S.nslices);
    hipLaunchKernelGGL(k_csr_sell_width, dim3(grid_xcd(S.nslices, BLOCK / 64)), dim3(BLOCK), 0, s, V, S.nslices, ptr,
                       w.p);
    S.ptr.alloc(ctx, S.nslices + 1);
    S.entries = scan_exclusive_i32_to_i64(ctx, w.p, S.ptr.p, S.nslices, true);
    S.kept = nnz;
    S.col.alloc(ctx, S.entries);
    S.val64.alloc(ctx, S.entries);
    S.val32.alloc(ctx, S.entries);
    hipLaunchKernelGGL(k_csr_sell_fill, dim3(grid_xcd(S.nslices * SELL_C)), dim3(BLOCK), 0, s, V, S.nslices, ptr, col,
                       v64, v32, S.ptr.p, S.col.p, S.val64.p, S.val32.p);
    HIP_CHECK(hipGetLastError());
    build_sell_offsets(ctx, S, V);
}

void fsai_setup(dec_mesh* m) {
    FsaiFactor& F = m->fsai;
    if (F.ready) return;
    dec_ctx* ctx = m->ctx;
    hipStream_t s = ctx->stream;
    const int64_t V = m->V;
    DEC_REQUIRE(m->bc_ready, DEC_ESTATE, "FSAI needs dec_apply_bc first");
    DBuf<int32_t> glen, gtlen, wlen;
    glen.alloc(ctx, V);
    gtlen.alloc(ctx, V);
    wlen.alloc(ctx, V);
    hipLaunchKernelGGL(k_fsai_lengths, dim3(grid_for(V)), dim3(BLOCK), 0, s, V, m->row_ptr.p, m->diag_pos.p, glen.p,
                       gtlen.p, wlen.p);
    DBuf<int64_t> g_ptr64, gt_ptr64, w_ptr;
    g_ptr64.alloc(ctx, V + 1);
    gt_ptr64.alloc(ctx, V + 1);
    w_ptr.alloc(ctx, V + 1);
    const int64_t ng = scan_exclusive_i32_to_i64(ctx, glen.p, g_ptr64.p, V, true);
    const int64_t ngt = scan_exclusive_i32_to_i64(ctx, gtlen.p, gt_ptr64.p, V, true);
    const int64_t nw = scan_exclusive_i32_to_i64(ctx, wlen.p, w_ptr.p, V, true);
    DEC_REQUIRE(ng == ngt, DEC_EINVAL, "internal: FSAI pattern is not symmetric");
    F.nnz = ng;
    F.g_ptr.alloc(ctx, V + 1);
    F.gt_ptr.alloc(ctx, V + 1);
    copy_i64_to_i32(ctx, g_ptr64.p, F.g_ptr.p, V + 1);
    copy_i64_to_i32(ctx, gt_ptr64.p, F.gt_ptr.p, V + 1);
    F.g_col.alloc(ctx, ng);
    F.gt_col.alloc(ctx, ng);
    F.gt_src.alloc(ctx, ng);
    hipLaunchKernelGGL(k_fsai_pattern, dim3(grid_for(V)), dim3(BLOCK), 0, s, V, m->row_ptr.p, m->col.p, m->diag_pos.p,
                       g_ptr64.p, gt_ptr64.p, F.g_col.p, F.gt_col.p, F.gt_src.p);
    F.g_val64.alloc(ctx, ng);
    F.g_val32.alloc(ctx, ng);
    F.gt_val64.alloc(ctx, ng);
    F.gt_val32.alloc(ctx, ng);
    DBuf<double> work;
    work.alloc(ctx, nw);
    DBuf<unsigned> err;
    err.alloc(ctx, 1);
    err.zero();
    hipLaunchKernelGGL(k_fsai_values, dim3(grid_for(V)), dim3(BLOCK), 0, s, V, m->row_ptr.p, m->col.p, m->val64.p,
                       m->diag_pos.p, g_ptr64.p, w_ptr.p, work.p, F.g_val64.p, F.g_val32.p, err.p);
    hipLaunchKernelGGL(k_fsai_transpose_values, dim3(grid_for(ng)), dim3(BLOCK), 0, s, ng, F.gt_src.p, F.g_val64.p,
                       F.gt_val64.p, F.gt_val32.p);
    HIP_CHECK(hipGetLastError());
    const unsigned e = *static_cast<unsigned*>(ctx->readback(err.p, sizeof(unsigned)));
    DEC_REQUIRE(e == 0, DEC_EBREAKDOWN, "FSAI: a local system is not positive definite");
    F.g_sell = SellMatrix();
    F.gt_sell = SellMatrix();
    build_sell_copy(ctx, V, ng, F.g_ptr.p, F.g_col.p, F.g_val64.p, F.g_val32.p, F.g_sell);
    build_sell_copy(ctx, V, ng, F.gt_ptr.p, F.gt_col.p, F.gt_val64.p, F.gt_val32.p, F.gt_sell);
    ctx->sync();  // the width scratch is released on return
    F.ready = true;
    if (m->solve) clear_graphs(m->solve);
}

extern "C" int dec_get_fsai(dec_mesh* m, int64_t* nnz_out, int32_t* g_ptr, int32_t* g_col, double* g_val) {
    if (!m) return DEC_EINVAL;
    try {
        m->ctx->set_device();
        fsai_setup(m);
        if (nnz_out) *nnz_out = m->fsai.nnz;
        hipStream_t s = m->ctx->stream;
        if (g_ptr)
            HIP_CHECK(hipMemcpyAsync(g_ptr, m->fsai.g_ptr.p, (m->V + 1) * sizeof(int32_t), hipMemcpyDeviceToDevice, s));
        if (g_col)
            HIP_CHECK(hipMemcpyAsync(g_col, m->fsai.g_col.p, m->fsai.nnz * sizeof(int32_t), hipMemcpyDeviceToDevice, s));
        if (g_val)
            HIP_CHECK(hipMemcpyAsync(g_val, m->fsai.g_val64.p, m->fsai.nnz * sizeof(double), hipMemcpyDeviceToDevice, s));
    } catch (const DecError& e) {
        m->ctx->last_error = e.msg;
        return e.code;
    }
    return DEC_OK;
}
