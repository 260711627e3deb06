// Assembly of L = d0^T *1 d0 on the static pattern (Section 2.1; the paper
// keeps the system matrix's form fixed when cracks are inserted, Section
// 2.3): L_ij = -*1_e, L_ii = sum of *1_e over the row's edges in ascending
// column order.  One thread per row, no atomics, so the values are
// deterministic.  The FP32 copy and the sliced-ELL copies are refreshed
// from the FP64 CSR values.
#include "common.h"

namespace {

__global__ void k_assemble_values(int64_t V, const int32_t* __restrict__ row_ptr, const int32_t* __restrict__ nz_edge,
                                  const int32_t* __restrict__ diag_pos, const double* __restrict__ star1,
                                  double* __restrict__ val64, float* __restrict__ val32) {
    GRID_STRIDE_LOOP(v, V) {
        double sum = 0.0;
        for (int32_t k = row_ptr[v]; k < row_ptr[v + 1]; ++k) {
            const int32_t e = nz_edge[k];
            if (e < 0) continue;
            const double s = star1[e];
            val64[k] = -s;
            val32[k] = static_cast<float>(-s);
            sum += s;
        }
        const int32_t d = diag_pos[v];
        val64[d] = sum;
        val32[d] = static_cast<float>(sum);
    }
}

__global__ void k_sell_width(int64_t V, int64_t nslices, const int32_t* __restrict__ row_ptr,
                             int32_t* __restrict__ width64) {
    GRID_STRIDE_LOOP(s, nslices) {
        int w = 0;
        const int64_t r0 = s * SELL_C;
        for (int64_t r = r0; r < r0 + SELL_C && r < V; ++r) w = max(w, row_ptr[r + 1] - row_ptr[r]);
        width64[s] = w * SELL_C;  // entries in the slice
    }
}

__global__ void k_sell_fill(int64_t V, int64_t nslices, const int32_t* __restrict__ row_ptr,
                            const int32_t* __restrict__ col, const int64_t* __restrict__ sptr,
                            int32_t* __restrict__ scol, int32_t* __restrict__ ssrc) {
    GRID_STRIDE_LOOP(i, nslices * SELL_C) {
        const int64_t s = i / SELL_C;
        const int lane = static_cast<int>(i % SELL_C);
        const int64_t row = i;
        const int width = static_cast<int>((sptr[s + 1] - sptr[s]) / SELL_C);
        const int32_t b = row < V ? row_ptr[row] : 0;
        const int len = row < V ? row_ptr[row + 1] - b : 0;
        const int32_t pad_col = static_cast<int32_t>(row < V ? row : V - 1);
        for (int j = 0; j < width; ++j) {
            const int64_t idx = sptr[s] + static_cast<int64_t>(j) * SELL_C + lane;
            if (j < len) {
                scol[idx] = col[b + j];
                ssrc[idx] = b + j;
            } else {
                scol[idx] = pad_col;
                ssrc[idx] = -1;
            }
        }
    }
}

__global__ void k_sell_values(int64_t n, const int32_t* __restrict__ ssrc, const double* __restrict__ v64,
                              double* __restrict__ s64, float* __restrict__ s32) {
    GRID_STRIDE_LOOP(i, n) {
        const int32_t k = ssrc[i];
        const double v = k >= 0 ? v64[k] : 0.0;
        s64[i] = v;
        s32[i] = static_cast<float>(v);
    }
}

void build_sell_pattern(dec_mesh* m) {
    dec_ctx* ctx = m->ctx;
    SellMatrix& S = m->sell;
    if (S.nslices) return;
    S.nslices = (m->V + SELL_C - 1) / SELL_C;
    DBuf<int32_t> w;
    w.alloc(ctx, S.nslices);
    hipLaunchKernelGGL(k_sell_width, dim3(grid_for(S.nslices)), dim3(BLOCK), 0, ctx->stream, m->V, S.nslices,
                       m->row_ptr.p, w.p);
    S.ptr.alloc(ctx, S.nslices + 1);
    S.entries = scan_exclusive_i32_to_i64(ctx, w.p, S.ptr.p, S.nslices, true);
    S.col.alloc(ctx, S.entries);
    S.src.alloc(ctx, S.entries);
    S.val64.alloc(ctx, S.entries);
    S.val32.alloc(ctx, S.entries);
    hipLaunchKernelGGL(k_sell_fill, dim3(grid_for(S.nslices * SELL_C)), dim3(BLOCK), 0, ctx->stream, m->V,
                       S.nslices, m->row_ptr.p, m->col.p, S.ptr.p, S.col.p, S.src.p);
    HIP_CHECK(hipGetLastError());
}

}  // namespace

// Copy the CSR values into the sliced-ELL layout (after assembly or boundary edits).
void refresh_sell_values(dec_mesh* m) {
    SellMatrix& S = m->sell;
    hipLaunchKernelGGL(k_sell_values, dim3(grid_for(S.entries)), dim3(BLOCK), 0, m->ctx->stream, S.entries,
                       S.src.p, m->val64.p, S.val64.p, S.val32.p);
    HIP_CHECK(hipGetLastError());
}

void assemble_device(dec_mesh* m) {
    dec_ctx* ctx = m->ctx;
    DEC_REQUIRE(m->star_ready, DEC_ESTATE, "dec_assemble needs dec_hodge1 first");
    m->val64.alloc(ctx, m->nnz);
    m->val32.alloc(ctx, m->nnz);
    hipLaunchKernelGGL(k_assemble_values, dim3(grid_for(m->V)), dim3(BLOCK), 0, ctx->stream, m->V, m->row_ptr.p,
                       m->nz_edge.p, m->diag_pos.p, m->star1.p, m->val64.p, m->val32.p);
    HIP_CHECK(hipGetLastError());
    build_sell_pattern(m);
    refresh_sell_values(m);
    m->assembled = true;
    m->bc_ready = false;
    m->fsai.ready = false;
}

extern "C" int dec_assemble(dec_mesh* m, uint32_t flags) {
    if (!m) return DEC_EINVAL;
    try {
        DEC_REQUIRE(flags == DEC_ASM_DEFAULT, DEC_EINVAL, "unknown assembly flags");
        m->ctx->set_device();
        assemble_device(m);
    } catch (const DecError& e) {
        m->ctx->last_error = e.msg;
        return e.code;
    }
    return DEC_OK;
}

extern "C" int dec_get_csr(const dec_mesh* m, int32_t* row_ptr, int32_t* col, double* val64, float* val32) {
    if (!m) return DEC_EINVAL;
    try {
        hipStream_t s = m->ctx->stream;
        if (row_ptr)
            HIP_CHECK(hipMemcpyAsync(row_ptr, m->row_ptr.p, (m->V + 1) * sizeof(int32_t), hipMemcpyDeviceToDevice, s));
        if (col) HIP_CHECK(hipMemcpyAsync(col, m->col.p, m->nnz * sizeof(int32_t), hipMemcpyDeviceToDevice, s));
        if (val64 || val32) DEC_REQUIRE(m->assembled, DEC_ESTATE, "values need dec_assemble first");
        if (val64) HIP_CHECK(hipMemcpyAsync(val64, m->val64.p, m->nnz * sizeof(double), hipMemcpyDeviceToDevice, s));
        if (val32) HIP_CHECK(hipMemcpyAsync(val32, m->val32.p, m->nnz * sizeof(float), hipMemcpyDeviceToDevice, s));
    } catch (const DecError& e) {
        m->ctx->last_error = e.msg;
        return e.code;
    }
    return DEC_OK;
}
