// Assembly of L = d0^T *1 d0 on the static pattern (Section 2.1; the paper
// keeps the system matrix's form fixed when cracks are inserted, Section
// 2.3): L_ij = -*1_e, L_ii = sum of *1_e over the row's edges in ascending
// column order.  No atomics, so the values are deterministic.  The FP32 copy and the sliced-ELL copies are refreshed
// from the FP64 CSR values.
#include <climits>
#include <cstdio>
#include <cstdlib>
#include <cstring>

#include "group_front.h"
#include "row_scan.h"
#include "sell.h"

struct SolveCache;
void clear_graphs(SolveCache* c);

namespace {

// One ROWG-lane group per row: the group loads a run of ROWG entries at a
// time (coalesced), writes the off-diagonal values, and adds the run's *1
// values to the diagonal in ascending column order (row_seq_sum), so the
// diagonal is the same sequential sum as a one-thread-per-row loop.
constexpr int ROWG = 16;

__global__ void k_assemble_values(int64_t V, const int32_t* __restrict__ row_ptr, const int32_t* __restrict__ nz_edge,
                                  const int32_t* __restrict__ diag_pos, const double* __restrict__ star1,
                                  double* __restrict__ val64, float* __restrict__ val32) {
    const int g = threadIdx.x & (ROWG - 1);
    GROUP_FRONT_LOOP(v, V, ROWG) {
        const int32_t b = row_ptr[v], n = row_ptr[v + 1] - b;
        double sum = 0.0;  // lane 0's
        for (int32_t k0 = 0; k0 < n; k0 += ROWG) {
            const int32_t k = k0 + g;
            const int32_t e = k < n ? nz_edge[b + k] : -1;
            const double s = e >= 0 ? star1[e] : 0.0;
            if (e >= 0) {
                val64[b + k] = -s;
                val32[b + k] = static_cast<float>(-s);
            }
            sum = row_seq_sum(sum, s, e >= 0, g);
        }
        if (g == 0) {
            const int32_t d = diag_pos[v];
            val64[d] = sum;
            val32[d] = static_cast<float>(sum);
        }
    }
}

// Entries kept in the sliced-ELL copy: the diagonal and every edge whose
// geometric factor |*e| / |e| is not exactly zero.  An edge with zero dual
// area has L_ij = -kappa * 0 = -0 for every conductivity and crack set, and
// adding its product to a row sum changes nothing, so the product y = A x is
// bit-for-bit that of the full static pattern (which the CSR keeps).
//
// Kept flags (bit u) of entries k .. k + 7 of a row that ends before k1
// (entries past the row: not kept); the eight loads of each kind are issued
// together.
__device__ __forceinline__ unsigned kept8(int32_t k, int32_t k1, const int32_t* __restrict__ nz_edge,
                                          const double* __restrict__ geo) {
    int32_t e[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) e[u] = k + u < k1 ? nz_edge[k + u] : -1;
    unsigned mask = 0;
#pragma unroll
    for (int u = 0; u < 8; ++u) {
        const bool in = k + u < k1;
        const double g = (in && e[u] >= 0 && geo != nullptr) ? geo[e[u]] : 1.0;
        mask |= (in && g != 0.0) ? 1u << u : 0u;
    }
    return mask;
}

constexpr int KEPT_SPREAD = 64;

// Stored entries per slice: one wavefront per slice, each lane counts its
// row's kept entries and the wavefront takes the maximum.  Also the number of
// kept entries, per block.
__global__ __launch_bounds__(BLOCK) void k_sell_width(int64_t V, int64_t nslices, const int32_t* __restrict__ row_ptr,
                                                      const int32_t* __restrict__ nz_edge,
                                                      const double* __restrict__ geo, int32_t* __restrict__ width64,
                                                      unsigned long long* __restrict__ kept_count) {
    static_assert(SELL_C == 64, "one slice per wavefront");
    __shared__ unsigned long long lds[BLOCK / 64];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    unsigned long long total = 0;
    int64_t s0, s1;
    block_range(nslices, &s0, &s1);
    for (int64_t s = s0 + w; s < s1; s += BLOCK / 64) {
        const int64_t r = s * SELL_C + lane;
        int len = 0;
        if (r < V) {
            const int32_t k1 = row_ptr[r + 1];
            for (int32_t k = row_ptr[r]; k < k1; k += 8) len += __popc(kept8(k, k1, nz_edge, geo));
        }
        total += len;
        int wmax = len;
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) wmax = max(wmax, __shfl_xor(wmax, off, 64));
        if (lane == 0) width64[s] = wmax * SELL_C;  // entries in the slice
    }
    total = block_sum(total, lds);
    // one of KEPT_SPREAD counters per block (summed on the host): thousands
    // of blocks adding to one address would wait on each other
    if (threadIdx.x == 0 && total) atomicAdd(kept_count + blockIdx.x % KEPT_SPREAD, total);
}

__global__ void k_sell_fill(int64_t V, int64_t nslices, const int32_t* __restrict__ row_ptr,
                            const int32_t* __restrict__ col, const int32_t* __restrict__ nz_edge,
                            const double* __restrict__ geo, const int64_t* __restrict__ sptr,
                            int32_t* __restrict__ scol, int32_t* __restrict__ ssrc) {
    GROUP_FRONT_LOOP(i, nslices * SELL_C, 1) {
        const int64_t s = i / SELL_C;
        const int lane = static_cast<int>(i % SELL_C);
        const int64_t row = i;
        const int width = static_cast<int>((sptr[s + 1] - sptr[s]) / SELL_C);
        const int32_t pad_col = static_cast<int32_t>(row < V ? row : V - 1);
        int j = 0;
        if (row < V) {
            const int32_t k1 = row_ptr[row + 1];
            for (int32_t k = row_ptr[row]; k < k1; k += 8) {
                const unsigned mask = kept8(k, k1, nz_edge, geo);
                int32_t c[8];
#pragma unroll
                for (int u = 0; u < 8; ++u) c[u] = (mask >> u) & 1u ? col[k + u] : 0;
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    if (!((mask >> u) & 1u)) continue;
                    const int64_t idx = sell_index(sptr[s], width, j, lane);
                    scol[idx] = c[u];
                    ssrc[idx] = k + u;
                    ++j;
                }
            }
        }
        for (; j < width; ++j) {
            const int64_t idx = sell_index(sptr[s], width, j, lane);
            scol[idx] = pad_col;
            ssrc[idx] = -1;
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

// The column offsets col - row of a sliced-ELL matrix (rows past V count as
// offset 0), in one pass: as int16 in the same slots (with a flag when one
// does not fit), and as the set of distinct values, collected in an
// open-addressing hash set of OSET_CAP slots: each workgroup first gathers
// its own in LDS, then adds them to the global set, so the global atomics
// number (workgroups x distinct offsets).  flags: [0] an offset beyond 16 bits,
// [1] distinct offsets, [2] more than OTAB_MAX of them (in one workgroup or
// in all), [3] the largest |offset| (written with the table).
constexpr int OSET_CAP = 1024;
constexpr int32_t OSET_EMPTY = INT32_MIN;

__device__ __forceinline__ uint32_t oset_hash(int32_t d) { return (static_cast<uint32_t>(d) * 2654435761u) >> 22; }

// insert d into a set of OSET_CAP slots; returns 1 when this call added it, 0 when present,
// -1 when the set is full
template <bool SHARED>
__device__ __forceinline__ int oset_insert(int32_t* set, int32_t d) {
    uint32_t h = oset_hash(d);
    for (int probe = 0; probe < OSET_CAP; ++probe, h = (h + 1) & (OSET_CAP - 1)) {
        int32_t cur = SHARED ? set[h] : coherent_load(set + h);
        if (cur == d) return 0;
        if (cur == OSET_EMPTY) {
            cur = atomicCAS(set + h, OSET_EMPTY, d);
            if (cur == OSET_EMPTY) return 1;
            if (cur == d) return 0;
        }
    }
    return -1;
}

__global__ __launch_bounds__(BLOCK) void k_sell_offsets(int64_t V, int64_t nslices, const int64_t* __restrict__ sptr,
                                                        const int32_t* __restrict__ scol, int16_t* __restrict__ dcol,
                                                        int32_t* __restrict__ gset, unsigned* __restrict__ flags) {
    __shared__ int32_t lset[OSET_CAP];
    __shared__ int lcount;
    for (int t = threadIdx.x; t < OSET_CAP; t += BLOCK) lset[t] = OSET_EMPTY;
    if (threadIdx.x == 0) lcount = 0;
    __syncthreads();
    bool over16 = false;
    RANGE_LOOP(i, nslices * SELL_C) {
        const int64_t s = i / SELL_C;
        const int lane = static_cast<int>(i % SELL_C);
        const int width = static_cast<int>((sptr[s + 1] - sptr[s]) / SELL_C);
        for (int j = 0; j < width; ++j) {
            const int64_t idx = sell_index(sptr[s], width, j, lane);
            const int64_t d = static_cast<int64_t>(scol[idx]) - i;  // row i = s * SELL_C + lane
            over16 |= d < INT16_MIN || d > INT16_MAX;
            dcol[idx] = static_cast<int16_t>(d);  // unused when any offset is out of range
            if (lcount > OTAB_MAX) continue;  // too many for a table already
            const int r = oset_insert<true>(lset, i < V ? static_cast<int32_t>(d) : 0);
            if (r != 0) atomicAdd(&lcount, r > 0 ? 1 : OTAB_MAX + 1);
        }
    }
    if (over16) atomicOr(flags, 1u);
    __syncthreads();
    if (lcount > OTAB_MAX) {
        if (threadIdx.x == 0) atomicOr(flags + 2, 1u);
        return;
    }
    for (int t = threadIdx.x; t < OSET_CAP; t += BLOCK) {
        if (lset[t] == OSET_EMPTY) continue;
        const int r = oset_insert<false>(gset, lset[t]);
        if (r > 0) atomicAdd(flags + 1, 1u);
        if (r < 0) atomicOr(flags + 2, 1u);
    }
}

// One workgroup of OSET_CAP threads: the set's values in ascending order into
// otab (bitonic sort in LDS; the empty slots, INT32_MIN, sort first), when
// there are at most OTAB_MAX of them.
__global__ __launch_bounds__(OSET_CAP) void k_offset_sort(const int32_t* __restrict__ gset,
                                                          unsigned* __restrict__ flags,
                                                          int32_t* __restrict__ otab) {
    __shared__ int32_t v[OSET_CAP];
    const unsigned count = flags[1];
    if (flags[2] || count > (unsigned)OTAB_MAX) return;
    const int t = threadIdx.x;
    v[t] = gset[t];
    __syncthreads();
    for (int k = 2; k <= OSET_CAP; k <<= 1)
        for (int j = k >> 1; j > 0; j >>= 1) {
            const int p = t ^ j;
            if (p > t) {
                const bool up = (t & k) == 0;
                const int32_t a = v[t], b = v[p];
                if ((a > b) == up) {
                    v[t] = b;
                    v[p] = a;
                }
            }
            __syncthreads();
        }
    if (t < (int)count) otab[t] = v[OSET_CAP - count + t];
    if (t == 0 && count > 0) {
        const int64_t lo = v[OSET_CAP - count], hi = v[OSET_CAP - 1];
        flags[3] = static_cast<unsigned>(-lo > hi ? -lo : hi);
    }
}

// The index of col - row in the ascending offset table (staged in LDS), per
// stored entry, when the table was built.
__global__ __launch_bounds__(BLOCK) void k_offset_index(int64_t V, int64_t nslices, const int64_t* __restrict__ sptr,
                                                        const int32_t* __restrict__ scol, const int32_t* __restrict__ otab,
                                                        const unsigned* __restrict__ flags, uint8_t* __restrict__ tcol) {
    __shared__ int32_t tab[OTAB_MAX];
    const unsigned count = flags[1];
    if (flags[2] || count > (unsigned)OTAB_MAX) return;
    const int ntab = static_cast<int>(count);
    stage_offsets(otab, ntab, tab);
    RANGE_LOOP(i, nslices * SELL_C) {
        const int64_t s = i / SELL_C;
        const int lane = static_cast<int>(i % SELL_C);
        const int width = static_cast<int>((sptr[s + 1] - sptr[s]) / SELL_C);
        for (int j = 0; j < width; ++j) {
            const int64_t idx = sell_index(sptr[s], width, j, lane);
            const int32_t d = i < V ? scol[idx] - static_cast<int32_t>(i) : 0;
            int lo = 0, hi = ntab - 1;  // d is in the table
            while (lo < hi) {
                const int mid = (lo + hi) >> 1;
                if (tab[mid] < d)
                    lo = mid + 1;
                else
                    hi = mid;
            }
            tcol[idx] = static_cast<uint8_t>(lo);
        }
    }
}

__global__ void k_fill_i32(int64_t n, int32_t v, int32_t* __restrict__ out) { GRID_STRIDE_LOOP(i, n) out[i] = v; }

void build_sell_pattern(dec_mesh* m) {
    dec_ctx* ctx = m->ctx;
    SellMatrix& S = m->sell;
    if (S.nslices) return;
    S.nslices = (m->V + SELL_C - 1) / SELL_C;
    DBuf<int32_t> w;
    w.alloc(ctx, S.nslices);
    DBuf<unsigned long long> cnt;
    cnt.alloc(ctx, KEPT_SPREAD);
    cnt.zero();
    const double* geo = m->prune_geometric_zeros ? m->geo.p : nullptr;
    hipLaunchKernelGGL(k_sell_width, dim3(grid_xcd(S.nslices, BLOCK / 64)), dim3(BLOCK), 0, ctx->stream, m->V,
                       S.nslices, m->row_ptr.p, m->nz_edge.p, geo, w.p, cnt.p);
    S.ptr.alloc(ctx, S.nslices + 1);
    S.entries = scan_exclusive_i32_to_i64(ctx, w.p, S.ptr.p, S.nslices, true);
    const unsigned long long* kc =
        static_cast<const unsigned long long*>(ctx->readback(cnt.p, KEPT_SPREAD * sizeof(unsigned long long)));
    S.kept = 0;
    for (int k = 0; k < KEPT_SPREAD; ++k) S.kept += (int64_t)kc[k];
    S.col.alloc(ctx, S.entries);
    S.src.alloc(ctx, S.entries);
    S.val64.alloc(ctx, S.entries);
    S.val32.alloc(ctx, S.entries);
    hipLaunchKernelGGL(k_sell_fill, dim3(grid_xcd(S.nslices * SELL_C)), dim3(BLOCK), 0, ctx->stream, m->V,
                       S.nslices, m->row_ptr.p, m->col.p, m->nz_edge.p, geo, S.ptr.p, S.col.p, S.src.p);
    HIP_CHECK(hipGetLastError());
    build_sell_offsets(ctx, S, m->V);
}

}  // namespace

void build_sell_offsets(dec_ctx* ctx, SellMatrix& S, int64_t V) {
    S.dcol = DBuf<int16_t>();
    S.tcol = DBuf<uint8_t>();
    S.otab = DBuf<int32_t>();
    S.ntab = 0;
    S.far = -1;
    S.band_plane = S.band = 0;
    if (S.entries == 0) return;
    hipStream_t st = ctx->stream;
    DBuf<int16_t> d;
    d.alloc(ctx, S.entries);
    DBuf<uint8_t> t;
    t.alloc(ctx, S.entries);
    DBuf<int32_t> tab, gset;
    tab.alloc(ctx, OTAB_MAX);
    gset.alloc(ctx, OSET_CAP);
    DBuf<unsigned> flags;  // see k_sell_offsets
    flags.alloc(ctx, 4);
    flags.zero();
    hipLaunchKernelGGL(k_fill_i32, dim3(grid_for(OSET_CAP)), dim3(BLOCK), 0, st, (int64_t)OSET_CAP, OSET_EMPTY, gset.p);
    const unsigned g = grid_xcd(S.nslices * SELL_C);
    hipLaunchKernelGGL(k_sell_offsets, dim3(g), dim3(BLOCK), 0, st, V, S.nslices, S.ptr.p, S.col.p, d.p, gset.p,
                       flags.p);
    hipLaunchKernelGGL(k_offset_sort, dim3(1), dim3(OSET_CAP), 0, st, gset.p, flags.p, tab.p);
    hipLaunchKernelGGL(k_offset_index, dim3(g), dim3(BLOCK), 0, st, V, S.nslices, S.ptr.p, S.col.p, tab.p, flags.p,
                       t.p);
    HIP_CHECK(hipGetLastError());
    unsigned h[4];
    std::memcpy(h, ctx->readback(flags.p, sizeof(h)), sizeof(h));  // the one synchronisation
    if (h[0] == 0) S.dcol = std::move(d);
    if (h[2] == 0 && h[1] <= (unsigned)OTAB_MAX) {
        S.tcol = std::move(t);
        S.otab = std::move(tab);
        S.ntab = (int32_t)h[1];
        S.far = (int32_t)h[3];
    }
    choose_band(S, V);
}

// The product's slice order (sell.h banded_slice), plain unless
// DEC_SELL_BAND asks for bands: "plane,band" sets them for every matrix,
// "auto" applies this rule.  Between reading x_j for row j and gathering it
// for row j + far, an XCD streams about far times the bytes one row costs the
// FP64 product with one-byte columns; above BAND_REUSE_BYTES the order is
// banded, with planes of far / 64 slices (rounded) and bands of about
// BAND_BYTES of matrix.  On gfx950 the rule removes the repeated fetches of
// those gathers from L2 but not their time (the Infinity Cache serves them),
// so plain order is the default.
void choose_band(SellMatrix& S, int64_t V) {
    S.band_plane = S.band = 0;
    const char* env = getenv("DEC_SELL_BAND");
    if (!env) return;
    unsigned p = 0, b = 0;
    if (sscanf(env, "%u,%u", &p, &b) == 2 && p > 0 && b > 0) {
        S.band_plane = p;
        S.band = b;
        return;
    }
    if (strcmp(env, "auto") != 0) return;
    if (S.far < 0 || V == 0) return;
    const double row_bytes = (9.0 * (double)S.entries + 20.0 * (double)V) / (double)V;
    if ((double)S.far * row_bytes <= BAND_REUSE_BYTES) return;
    const uint32_t plane = (uint32_t)((S.far + SELL_C / 2) / SELL_C);
    double w = BAND_BYTES / (SELL_C * row_bytes);
    if (w < 16.0) w = 16.0;
    S.band_plane = plane;
    S.band = (uint32_t)w < plane ? (uint32_t)w : plane;
}

// Copy the CSR values into the sliced-ELL layout (after assembly or boundary edits).
void refresh_sell_values(dec_mesh* m) {
    SellMatrix& S = m->sell;
    hipLaunchKernelGGL(k_sell_values, dim3(grid_for(S.entries)), dim3(BLOCK), 0, m->ctx->stream, S.entries,
                       S.src.p, m->val64.p, S.val64.p, S.val32.p);
    HIP_CHECK(hipGetLastError());
}

// L = d0^T *1 d0 into the CSR values (FP64 and FP32) from the current *1.
void assemble_values(dec_mesh* m) {
    hipLaunchKernelGGL(k_assemble_values, dim3(grid_xcd(m->V, BLOCK / ROWG)), dim3(BLOCK), 0, m->ctx->stream, m->V,
                       m->row_ptr.p, m->nz_edge.p, m->diag_pos.p, m->star1.p, m->val64.p, m->val32.p);
    HIP_CHECK(hipGetLastError());
}

void assemble_device(dec_mesh* m) {
    dec_ctx* ctx = m->ctx;
    DEC_REQUIRE(m->star_ready, DEC_ESTATE, "dec_assemble needs dec_hodge1 first");
    m->val64.alloc(ctx, m->nnz);
    m->val32.alloc(ctx, m->nnz);
    assemble_values(m);
    build_sell_pattern(m);
    refresh_sell_values(m);
    m->assembled = true;
    m->bc_ready = false;
    m->fsai.ready = false;
    m->jsplit.ready = false;
}

extern "C" int dec_assemble(dec_mesh* m, uint32_t flags) {
    if (!m) return DEC_EINVAL;
    try {
        DEC_REQUIRE(!m->dual, DEC_ESTATE, "dec_assemble is for meshes of vertex unknowns");
        DEC_REQUIRE((flags & ~DEC_ASM_FULL_PATTERN) == 0, DEC_EINVAL, "unknown assembly flags");
        m->ctx->set_device();
        const bool prune = !(flags & DEC_ASM_FULL_PATTERN);
        if (m->sell.nslices && prune != m->prune_geometric_zeros) {
            m->sell = SellMatrix();  // rebuild the sliced-ELL pattern for the other choice
            if (m->solve) clear_graphs(m->solve);
        }
        m->prune_geometric_zeros = prune;
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
