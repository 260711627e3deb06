// Internal runtime of the DEC library: context, device buffers, the mesh
// object, error handling and the device-side reduction/scan building blocks
// shared by the kernels.  Nothing here is visible through the C ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstring>
#include <array>
#include <map>
#include <string>
#include <utility>
#include <vector>

#include "dec.h"

// ---------------------------------------------------------------- errors
struct DecError {
    int code;
    std::string msg;
};

[[noreturn]] inline void dec_fail(int code, const std::string& msg) { throw DecError{code, msg}; }

// Message of the last failed call that takes no context (this thread); dec_last_error(NULL).
std::string& free_error();

#define HIP_CHECK(expr)                                                                    \
    do {                                                                                   \
        hipError_t e_ = (expr);                                                            \
        if (e_ != hipSuccess)                                                              \
            dec_fail(DEC_EHIP, std::string(#expr) + " failed: " + hipGetErrorString(e_)); \
    } while (0)

#define DEC_REQUIRE(cond, code, msg) \
    do {                             \
        if (!(cond)) dec_fail((code), (msg)); \
    } while (0)

// ---------------------------------------------------------------- context
struct dec_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    dec_alloc_fn alloc = nullptr;
    dec_free_fn free_fn = nullptr;
    void* user = nullptr;
    std::string last_error;
    int num_cus = 256;
    int num_xcds = 8;
    int live_children = 0;  // meshes and servers created on this context and not yet destroyed
    // SpMV variant (unroll, non-temporal loads, column format) chosen per (kind of matrix and
    // precision, V, slices, stored entries)
    std::map<std::array<int64_t, 4>, std::array<int, 4>> spmv_tune;
    // small pinned staging area for scalar read-backs
    void* pinned = nullptr;
    size_t pinned_bytes = 0;

    void* dalloc(size_t bytes);
    void dfree(void* p);
    void set_device() const { HIP_CHECK(hipSetDevice(device)); }
    void sync() const { HIP_CHECK(hipStreamSynchronize(stream)); }
    // copy `bytes` from device to the pinned area and wait; returns the pinned pointer
    void* readback(const void* dptr, size_t bytes);
};

// A required pointer argument was NULL: record which call on the context (when
// one is reachable) and return DEC_EINVAL.
inline int null_argument(dec_ctx* ctx, const char* call) {
    if (ctx) ctx->last_error = std::string(call) + ": a required pointer argument is NULL";
    return DEC_EINVAL;
}

// Device buffer owned through the context's allocator.
template <class T>
struct DBuf {
    dec_ctx* ctx = nullptr;
    T* p = nullptr;
    size_t n = 0;

    DBuf() = default;
    DBuf(const DBuf&) = delete;
    DBuf& operator=(const DBuf&) = delete;
    DBuf(DBuf&& o) noexcept { swap(o); }
    DBuf& operator=(DBuf&& o) noexcept {
        release();
        swap(o);
        return *this;
    }
    ~DBuf() { release(); }
    void swap(DBuf& o) noexcept {
        std::swap(ctx, o.ctx);
        std::swap(p, o.p);
        std::swap(n, o.n);
    }
    void alloc(dec_ctx* c, size_t count) {
        if (p && n >= count && ctx == c) return;
        release();
        ctx = c;
        n = count;
        p = count ? static_cast<T*>(c->dalloc(count * sizeof(T))) : nullptr;
    }
    void release() {
        if (p && ctx) ctx->dfree(p);
        p = nullptr;
        n = 0;
    }
    size_t bytes() const { return n * sizeof(T); }
    void zero() const {
        if (p) HIP_CHECK(hipMemsetAsync(p, 0, n * sizeof(T), ctx->stream));
    }
};

// ---------------------------------------------------------------- matrices
// Sliced ELLPACK with slice height SELL_C (one row per lane of a wavefront)
// and `width` stored entries per row in the slice, paired: entries 2t and
// 2t + 1 of lane l sit side by side at ptr[s] + 2 SELL_C t + 2 l (+1), and an
// odd last entry at ptr[s] + 2 SELL_C (width / 2) + l.  A wavefront then
// reads two entries of every row with one 8 B (column) or 16 B (FP64 value)
// load per lane, over one contiguous segment.  Padding entries repeat the
// row's own column with value 0.
constexpr int SELL_C = 64;

__host__ __device__ inline int64_t sell_index(int64_t base, int width, int j, int lane) {
    const int np = width >> 1;
    return j < 2 * np ? base + static_cast<int64_t>(j >> 1) * (2 * SELL_C) + 2 * lane + (j & 1)
                      : base + static_cast<int64_t>(np) * (2 * SELL_C) + lane;
}

struct SellMatrix {
    int64_t nslices = 0;
    int64_t entries = 0;  // stored entries, padding included
    int64_t kept = 0;     // entries of the pattern the product uses
    DBuf<int64_t> ptr;   // [nslices + 1]
    DBuf<int32_t> col;   // [entries]
    DBuf<int32_t> src;   // [entries]: CSR entry index, -1 for padding
    DBuf<double> val64;  // [entries]
    DBuf<float> val32;   // [entries]
    DBuf<double> excess64;  // [V] row excess for the difference-form product (empty: plain form)
    DBuf<float> excess32;   // [V]
    DBuf<int16_t> dcol;     // [entries] col - row, kept only when every offset fits in 16 bits
    DBuf<uint8_t> tcol;     // [entries] index into otab of col - row (0 past the last row), kept only
                            // when the entries take at most 256 distinct offsets
    DBuf<int32_t> otab;     // [ntab] those offsets, ascending
    int32_t ntab = 0;
    int32_t far = -1;        // largest |col - row| over the entries when otab exists, else -1
    uint32_t band_plane = 0;  // the product's banded slice order (sell.h banded_slice), 0: plain order
    uint32_t band = 0;
};

// Fill S.dcol from S.col (rows of V, padding included), or leave it empty when
// some column lies 2^15 or more from its row; and S.tcol / S.otab when the
// offsets take at most 256 distinct values (rows past V count as offset 0).
// Then the product's slice order (choose_band): plain, or banded
// (S.band_plane, S.band) on request through DEC_SELL_BAND.
// Synchronises the stream.
constexpr double BAND_REUSE_BYTES = 2.0 * (1 << 20);  // half an XCD's 4 MiB L2
constexpr double BAND_BYTES = 1.0 * (1 << 20);
void build_sell_offsets(dec_ctx* ctx, SellMatrix& S, int64_t V);
void choose_band(SellMatrix& S, int64_t V);

// Lower-triangular FSAI factor G (CSR) and its transpose (CSR of G^T).
struct FsaiFactor {
    bool ready = false;
    int64_t nnz = 0;
    DBuf<int32_t> g_ptr, g_col, gt_ptr, gt_col, gt_src;
    DBuf<double> g_val64, gt_val64;
    DBuf<float> g_val32, gt_val32;
    SellMatrix g_sell, gt_sell;  // sliced-ELL copies that the solver applies (same entry order per row)
};

// Jacobi in split form: CG on D^-1/2 A D^-1/2 with x = D^-1/2 x^, the same
// iterates as Jacobi-preconditioned CG on A, one vector fewer per iteration.
// Built by the solver from the sliced-ELL copy when every diagonal entry is
// positive; stale after assembly or new boundary data.
struct JacobiSplit {
    bool ready = false;   // built for the current values
    DBuf<double> v64;     // [entries] a_ij s_i s_j, s = D^-1/2
    DBuf<float> v32;      // [entries]
    DBuf<double> s64;     // [V] s
    DBuf<double> b64;     // [V] s * b
    DBuf<double> d64;     // [V] a_ii (r.r of the unscaled residual is sum d r^2)
    DBuf<float> d32;      // [V]
};

// The paper's own unknowns: a system whose rows are the tets of a mesh, with
// the face data its flux and queries need (see dual.hip).
struct DualData {
    int64_t F = 0;
    DBuf<int32_t> t1, k1, t2, k2;  // [F] owner tet, local face index, other tet (-1), its index (-1)
    DBuf<double> W;                // [F] kappa_f / *_f on interior and Dirichlet faces, else 0
    DBuf<double> T0;               // [F] Dirichlet value (0 elsewhere)
    DBuf<int8_t> kind;             // [F] 0 interior, 1 Dirichlet, 2 insulated boundary
    DBuf<int8_t> side;             // [F] 1 inflow, 2 outflow, 0 other
    DBuf<uint8_t> cut;             // [F] cut by a disc
    DBuf<uint8_t> limited;         // [F] *_f set by the limiter
    int64_t n_limited = 0;         // limited faces
    int64_t n_blocks = 0;          // clusters of >= 2 tets inverted as one block
    int64_t max_block = 0;         // largest such cluster
};

struct SolveCache;  // Krylov vectors, reduction scratch and captured graphs

// ---------------------------------------------------------------- mesh
struct dec_mesh {
    dec_ctx* ctx = nullptr;
    dec_ctx* owner = nullptr;  // the context counted in live_children (servers re-point ctx)
    int64_t V = 0, T = 0, E = 0, F = 0, Fb = 0, nnz = 0;

    DBuf<double> xyz;        // [V*3]
    DBuf<int32_t> tets;      // [T*4]
    DBuf<int64_t> vt_ptr;    // [V+1]   vertex -> tets (ascending)
    DBuf<int32_t> vt_list;   // [4T]
    DBuf<int32_t> edges;     // [E*2]   (lo, hi), lexicographic
    DBuf<int64_t> up_ptr;    // [V+1]   edges with lo = v are up_ptr[v] .. up_ptr[v+1]-1
    DBuf<int64_t> et_ptr;    // [E+1]   edge -> (tet*6 + local edge), ascending tet
    DBuf<int32_t> et_inc;    // [6T]
    DBuf<uint8_t> tet_bface; // [T]     bit k: face opposite local vertex k is on the boundary

    // CSR pattern of L (static) and values
    DBuf<int32_t> row_ptr;   // [V+1]
    DBuf<int32_t> col;       // [nnz]
    DBuf<int32_t> nz_edge;   // [nnz]  edge of the entry, -1 on the diagonal
    DBuf<int32_t> diag_pos;  // [V]
    DBuf<double> val64;      // [nnz]
    DBuf<float> val32;       // [nnz]
    SellMatrix sell;
    bool prune_geometric_zeros = true;  // sliced-ELL drops edges with |*e| = 0

    // Hodge star
    bool geo_ready = false;
    double extent[7] = {0, 0, 0, 0, 0, 0, 0};  // bounding box (min xyz, max xyz) and longest half edge
    DBuf<double> geo;        // [E]  |*e| / |e| after the snap
    DBuf<double> star1;      // [E]
    DBuf<uint8_t> cut;       // [E]
    bool star_ready = false;
    bool assembled = false;

    // boundary data
    bool bc_ready = false;
    DBuf<uint8_t> fixed;     // [V] 1 Dirichlet, 2 pinned, 0 free
    DBuf<double> rhs;        // [V]
    DBuf<double> bc_value;   // [V] Dirichlet values (0 elsewhere)
    DBuf<double> invdiag64;  // [V]
    DBuf<float> invdiag32;   // [V]
    int64_t n_pinned = 0;
    bool neumann = false;    // the boundary data carry a Neumann load (neumann_f0 given)

    FsaiFactor fsai;
    JacobiSplit jsplit;
    bool diag_positive = false;  // every diagonal entry positive and finite (set with the boundary data)
    SolveCache* solve = nullptr;
    DualData* dual = nullptr;  // set for a system of tet unknowns (dec_dual_build)
    SellMatrix blockinv;       // tet systems: inverse of the diagonal blocks over the
                               // clusters of tets joined by limited faces (block Jacobi)

    ~dec_mesh();
};

// ---------------------------------------------------------------- launch helpers
constexpr int BLOCK = 256;

inline unsigned grid_for(int64_t n, int block = BLOCK, int64_t cap = 1 << 20) {
    int64_t g = (n + block - 1) / block;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return static_cast<unsigned>(g);
}

// Workgroups are dispatched round-robin over the 8 XCDs (each with its own
// L2).  Renumber them so that XCD x owns the contiguous x-th eighth of the
// work: neighbouring items, which gather the same data, then share an L2.
// gridDim.x must be a multiple of 8 (grid_xcd).
__device__ __forceinline__ int logical_block() {
    const int G = gridDim.x, b = blockIdx.x;
    return (b & 7) * (G >> 3) + (b >> 3);
}

// This block's contiguous share [b0, b1) of n items.
__device__ __forceinline__ void block_range(int64_t n, int64_t* b0, int64_t* b1) {
    const int64_t L = logical_block(), G = gridDim.x;
    *b0 = n * L / G;
    *b1 = n * (L + 1) / G;
}

// Front order for streaming kernels: XCD x owns the contiguous x-th eighth
// [x0, x1) of n items, and its blocks sweep it together, block j taking rows
// x0 + (j + k * per) * blockDim.x + threadIdx.x, k = 0, 1, ... (per = blocks
// of one XCD), so that at any moment an XCD streams one contiguous stretch of
// memory.  gridDim.x must be a multiple of 8.
struct FrontRange {
    int64_t first, step, end;
};

__device__ __forceinline__ FrontRange front_range(int64_t n) {
    const int64_t xcd = blockIdx.x & 7, j = blockIdx.x >> 3, per = gridDim.x >> 3;
    FrontRange r;
    r.first = n * xcd / 8 + j * blockDim.x + threadIdx.x;
    r.step = per * blockDim.x;
    r.end = n * (xcd + 1) / 8;
    return r;
}

// The same range in unsigned 32-bit row numbers (n < 2^31, so every row and
// every row plus a few strides fits): kernels that index several vectors with
// it address them as a uniform base plus a 32-bit offset per lane.
struct FrontRange32 {
    uint32_t first, step, end;
};

__device__ __forceinline__ FrontRange32 front_range32(int64_t n) {
    const FrontRange r = front_range(n);
    return FrontRange32{static_cast<uint32_t>(r.first), static_cast<uint32_t>(r.step), static_cast<uint32_t>(r.end)};
}

// Grid for block_range: about `per_block` items per block, at most `cap`
// blocks (32 per CU on 256 CUs: long-lived blocks, each walking a
// contiguous range), a multiple of 8.
inline unsigned grid_xcd(int64_t n, int64_t per_block = BLOCK, int64_t cap = 8192) {
    int64_t g = (n + per_block - 1) / per_block;
    if (g > cap) g = cap;
    g = (g + 7) / 8 * 8;
    if (g < 8) g = 8;
    return static_cast<unsigned>(g);
}

// Loop over this block's contiguous share of n items (launch with grid_xcd).
#define RANGE_LOOP(i, n)                                      \
    int64_t i##_lo, i##_hi;                                   \
    block_range((n), &i##_lo, &i##_hi);                       \
    for (int64_t i = i##_lo + threadIdx.x; i < i##_hi; i += blockDim.x)

#define GRID_STRIDE_LOOP(i, n)                                                     \
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; \
         i < (n); i += static_cast<int64_t>(gridDim.x) * blockDim.x)

// ---------------------------------------------------------------- device reductions
// Butterfly sum across a 64-lane wavefront (fixed pattern: deterministic).
template <class T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Sum over a block of BLOCK threads; the result is valid in thread 0.
template <class T>
__device__ __forceinline__ T block_sum(T v, T* lds) {
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    v = wave_sum(v);
    __syncthreads();
    if (lane == 0) lds[wid] = v;
    __syncthreads();
    T r = 0;
    if (threadIdx.x == 0) {
        const int nw = blockDim.x >> 6;
        for (int w = 0; w < nw; ++w) r += lds[w];
    }
    return r;
}

// Called by every thread of a block after thread 0 has stored the block's
// partial results.  Returns true in the block that finishes last; its loads
// after this point see every other block's partials.  (Used only where one
// launch per call is made; the solver's per-iteration kernels instead reduce
// the previous kernel's partials redundantly, see reduce_bcast.)
__device__ __forceinline__ bool last_block_arrived(unsigned* counter) {
    __shared__ int am_last;
    __syncthreads();
    if (threadIdx.x == 0) {
        __threadfence();
        unsigned prev = atomicAdd(counter, 1u);
        am_last = (prev == gridDim.x - 1);
    }
    __syncthreads();
    if (am_last) __threadfence();
    return am_last != 0;
}

template <class T>
__device__ __forceinline__ T coherent_load(const T* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Deterministic sum of `n` partials by one block (fixed order, independent
// of which block arrived last).  Result valid in thread 0.
template <class T>
__device__ __forceinline__ T reduce_partials(const T* partials, int n, T* lds) {
    T acc = 0;
    for (int i = threadIdx.x; i < n; i += blockDim.x) acc += coherent_load(partials + i);
    return block_sum(acc, lds);
}

// Thread t's share of a fixed-order sum of n partials: p[t] + p[t + BLOCK] +
// ... in that order.  The loads of a batch are issued together, so a block
// waits for one memory latency per FOLD_BATCH * BLOCK partials, not one per
// BLOCK (every block of a solver kernel folds the same partials at its start).
constexpr int FOLD_BATCH = 8;

struct FoldBatch {
    double v[FOLD_BATCH];
};

__device__ __forceinline__ FoldBatch fold_load(const double* __restrict__ p, int n, int base) {
    FoldBatch b;
#pragma unroll
    for (int k = 0; k < FOLD_BATCH; ++k) {
        const int i = base + k * BLOCK + static_cast<int>(threadIdx.x);
        b.v[k] = i < n ? p[i] : 0.0;
    }
    return b;
}

__device__ __forceinline__ double fold_add(double acc, const FoldBatch& b) {
#pragma unroll
    for (int k = 0; k < FOLD_BATCH; ++k) acc += b.v[k];
    return acc;
}

__device__ __forceinline__ double thread_fold(const double* __restrict__ p, int n) {
    double acc = 0.0;
    for (int base = 0; base < n; base += FOLD_BATCH * BLOCK) acc = fold_add(acc, fold_load(p, n, base));
    return acc;
}

// The block's sum of thread values t, returned to every thread.  lds holds
// BLOCK/64 + 1 doubles.
__device__ __forceinline__ double bcast_sum(double t, double* lds) {
    t = block_sum(t, lds);
    __syncthreads();
    if (threadIdx.x == 0) lds[BLOCK / 64] = t;
    __syncthreads();
    return lds[BLOCK / 64];
}

// Fixed-order sum of `n` partials written by an earlier kernel, returned to
// every thread of the block.  lds holds BLOCK/64 + 1 doubles.
__device__ __forceinline__ double reduce_bcast(const double* __restrict__ partials, int n, double* lds) {
    return bcast_sum(thread_fold(partials, n), lds);
}

// Two fixed-order sums (each as reduce_bcast computes it) with the loads of
// both in flight together and one set of barriers.  lds holds
// 2 * (BLOCK/64 + 1) doubles.
__device__ __forceinline__ void reduce_bcast2(const double* __restrict__ a, int na, const double* __restrict__ b,
                                              int nb, double* lds, double* ra, double* rb) {
    constexpr int NW = BLOCK / 64;
    const FoldBatch la = fold_load(a, na, 0), lb = fold_load(b, nb, 0);
    double sa = fold_add(0.0, la), sb = fold_add(0.0, lb);
    for (int base = FOLD_BATCH * BLOCK; base < na; base += FOLD_BATCH * BLOCK) sa = fold_add(sa, fold_load(a, na, base));
    for (int base = FOLD_BATCH * BLOCK; base < nb; base += FOLD_BATCH * BLOCK) sb = fold_add(sb, fold_load(b, nb, base));
    sa = wave_sum(sa);
    sb = wave_sum(sb);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) {
        lds[wid] = sa;
        lds[NW + wid] = sb;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double ta = 0, tb = 0;
        for (int w = 0; w < NW; ++w) ta += lds[w];
        for (int w = 0; w < NW; ++w) tb += lds[NW + w];
        lds[2 * NW] = ta;
        lds[2 * NW + 1] = tb;
    }
    __syncthreads();
    *ra = lds[2 * NW];
    *rb = lds[2 * NW + 1];
}

// Three fixed-order sums (each as reduce_bcast computes it) with the loads of
// all three in flight together and one set of barriers.  lds holds
// 3 * (BLOCK/64 + 1) doubles.
__device__ __forceinline__ void reduce_bcast3(const double* __restrict__ a, int na, const double* __restrict__ b,
                                              int nb, const double* __restrict__ c, int nc, double* lds,
                                              double* ra, double* rb, double* rc) {
    constexpr int NW = BLOCK / 64;
    const FoldBatch la = fold_load(a, na, 0), lb = fold_load(b, nb, 0), lc = fold_load(c, nc, 0);
    double sa = fold_add(0.0, la), sb = fold_add(0.0, lb), sc = fold_add(0.0, lc);
    for (int base = FOLD_BATCH * BLOCK; base < na; base += FOLD_BATCH * BLOCK) sa = fold_add(sa, fold_load(a, na, base));
    for (int base = FOLD_BATCH * BLOCK; base < nb; base += FOLD_BATCH * BLOCK) sb = fold_add(sb, fold_load(b, nb, base));
    for (int base = FOLD_BATCH * BLOCK; base < nc; base += FOLD_BATCH * BLOCK) sc = fold_add(sc, fold_load(c, nc, base));
    sa = wave_sum(sa);
    sb = wave_sum(sb);
    sc = wave_sum(sc);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) {
        lds[wid] = sa;
        lds[NW + wid] = sb;
        lds[2 * NW + wid] = sc;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double ta = 0, tb = 0, tc = 0;
        for (int w = 0; w < NW; ++w) ta += lds[w];
        for (int w = 0; w < NW; ++w) tb += lds[NW + w];
        for (int w = 0; w < NW; ++w) tc += lds[2 * NW + w];
        lds[3 * NW] = ta;
        lds[3 * NW + 1] = tb;
        lds[3 * NW + 2] = tc;
    }
    __syncthreads();
    *ra = lds[3 * NW];
    *rb = lds[3 * NW + 1];
    *rc = lds[3 * NW + 2];
}

// ---------------------------------------------------------------- host primitives
// out[0] = 0, out[i+1] = in[0] + ... + in[i]; returns out[n] (synchronises) when want_total.
int64_t scan_exclusive_i32_to_i64(dec_ctx* ctx, const int32_t* in, int64_t* out, int64_t n,
                                  bool want_total);
void copy_i64_to_i32(dec_ctx* ctx, const int64_t* in, int32_t* out, int64_t n);
