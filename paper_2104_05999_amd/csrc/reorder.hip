// Spatial numbering of a mesh (Section 2.2: a pre-processing step numbers the
// Delaunay nodes by their location in space, z first, then y, then x, so that
// blocks of consecutive nodes are compact; here it also makes the gathers of
// the SpMV and the assembly local).  For points off a lattice the sort is
// taken on cells: the bounding box is cut into B^3 cells, B^3 the first cube >= V,
// a point's cell on each axis is floor((x - lo) * (B / (hi - lo))) clamped to
// [0, B-1], and points are ordered by (x cell, y cell, z cell) with the z cell
// fastest, ties by original index.  Tets are then ordered by their smallest
// new vertex number, ties by original index, and keep their vertex order.
// Both orders come from a stable radix sort of (key, original index) pairs
// with the indices in ascending order (sort_indices, written here), so the
// result is unique, and its cost is linear however unevenly the points fill
// the cells.
// The Z (Morton) order is offered beside it: cells by the interleaved bits of
// (x cell, y cell, z cell) (z in the lowest bit), which keeps neighbours in
// all three directions close in memory.
#include <cmath>
#include <cstring>

#include "common.h"

namespace {

__global__ void k_bbox(int64_t V, const double* __restrict__ xyz, double* __restrict__ part) {
    __shared__ double red[6][BLOCK];
    double mn[3] = {INFINITY, INFINITY, INFINITY}, mx[3] = {-INFINITY, -INFINITY, -INFINITY};
    GRID_STRIDE_LOOP(i, V) {
        for (int a = 0; a < 3; ++a) {
            const double v = xyz[3 * i + a];
            mn[a] = fmin(mn[a], v);
            mx[a] = fmax(mx[a], v);
        }
    }
    for (int a = 0; a < 3; ++a) {
        red[a][threadIdx.x] = mn[a];
        red[3 + a][threadIdx.x] = mx[a];
    }
    __syncthreads();
    if (threadIdx.x < 6) {
        double r = red[threadIdx.x][0];
        for (int t = 1; t < BLOCK; ++t) r = threadIdx.x < 3 ? fmin(r, red[threadIdx.x][t]) : fmax(r, red[threadIdx.x][t]);
        part[6 * blockIdx.x + threadIdx.x] = r;
    }
}

__global__ void k_bbox_fold(int nb, const double* __restrict__ part, double* __restrict__ out) {
    if (threadIdx.x < 6) {
        double r = part[threadIdx.x];
        for (int b = 1; b < nb; ++b)
            r = threadIdx.x < 3 ? fmin(r, part[6 * b + threadIdx.x]) : fmax(r, part[6 * b + threadIdx.x]);
        out[threadIdx.x] = r;
    }
}

struct Grid {
    double lo[3], s[3];
    int64_t B;
};

__device__ __forceinline__ int64_t axis_cell(double x, double lo, double s, int64_t B) {
    const double c = floor((x - lo) * s);
    if (!(c > 0.0)) return 0;  // also NaN
    return c >= static_cast<double>(B - 1) ? B - 1 : static_cast<int64_t>(c);
}

// the bits of v (< 2^21) spread to every third position
__device__ __forceinline__ uint64_t spread3(uint64_t v) {
    v &= 0x1fffff;
    v = (v | (v << 32)) & 0x1f00000000ffffull;
    v = (v | (v << 16)) & 0x1f0000ff0000ffull;
    v = (v | (v << 8)) & 0x100f00f00f00f00full;
    v = (v | (v << 4)) & 0x10c30c30c30c30c3ull;
    v = (v | (v << 2)) & 0x1249249249249249ull;
    return v;
}

__global__ void k_point_cell(int64_t V, const double* __restrict__ xyz, Grid g, int morton,
                             uint64_t* __restrict__ cell, unsigned* __restrict__ err) {
    GRID_STRIDE_LOOP(i, V) {
        // the box ignores NaN (fmin / fmax), so a NaN coordinate is caught here
        if (!(isfinite(xyz[3 * i]) && isfinite(xyz[3 * i + 1]) && isfinite(xyz[3 * i + 2]))) atomicOr(err, 1u);
        const int64_t bx = axis_cell(xyz[3 * i], g.lo[0], g.s[0], g.B);
        const int64_t by = axis_cell(xyz[3 * i + 1], g.lo[1], g.s[1], g.B);
        const int64_t bz = axis_cell(xyz[3 * i + 2], g.lo[2], g.s[2], g.B);
        cell[i] = morton ? (spread3(bx) << 2) | (spread3(by) << 1) | spread3(bz)
                         : static_cast<uint64_t>((bx * g.B + by) * g.B + bz);
    }
}

__global__ void k_apply_vperm(int64_t V, const int32_t* __restrict__ perm, const double* __restrict__ xyz,
                              double* __restrict__ xyz_out, int32_t* __restrict__ inv) {
    GRID_STRIDE_LOOP(i, V) {
        const int32_t o = perm[i];
        inv[o] = (int32_t)i;
        xyz_out[3 * i] = xyz[3 * (int64_t)o];
        xyz_out[3 * i + 1] = xyz[3 * (int64_t)o + 1];
        xyz_out[3 * i + 2] = xyz[3 * (int64_t)o + 2];
    }
}

// tet key: its smallest new vertex number; flags a vertex index out of range
__global__ void k_tet_key(int64_t T, int64_t V, const int32_t* __restrict__ tets, const int32_t* __restrict__ inv,
                          uint32_t* __restrict__ key, unsigned* __restrict__ err) {
    GRID_STRIDE_LOOP(t, T) {
        int32_t m = INT32_MAX;
        bool ok = true;
        for (int k = 0; k < 4; ++k) {
            const int32_t v = tets[4 * t + k];
            if (v < 0 || v >= V) {
                ok = false;
                break;
            }
            m = min(m, inv[v]);
        }
        if (!ok) {
            atomicOr(err, 1u);
            m = 0;
        }
        key[t] = static_cast<uint32_t>(m);
    }
}

__global__ void k_apply_tperm(int64_t T, const int32_t* __restrict__ tperm, const int32_t* __restrict__ tets,
                              const int32_t* __restrict__ inv, int32_t* __restrict__ tets_out) {
    GRID_STRIDE_LOOP(i, T) {
        const int64_t o = tperm[i];
        for (int k = 0; k < 4; ++k) tets_out[4 * i + k] = inv[tets[4 * o + k]];
    }
}

// ---------------------------------------------------------------- stable radix sort
// A least-significant-digit radix sort of (key, index) pairs, 8 bits a pass.
// Block b owns the contiguous tile [b * tile, (b + 1) * tile) of the input.
// A pass counts each block's digits (k_radix_count, digit-major: count[d * G
// + b]), scans the counts (so block b's run of digit d starts after every
// element of a smaller digit and after blocks 0..b-1's elements of digit d),
// and scatters (k_radix_scatter): the block walks its tile in order, one
// element per thread, BLOCK elements at a time; an element's place is its
// run's start, plus the block's elements of its digit in earlier rounds,
// plus those before it in this round (earlier waves, then earlier lanes of
// its own wave, found with ballots on the digit's bits).  Every element
// keeps its order among equal digits, so after the last pass the pairs are
// ordered by key with ties in index order.
constexpr int RADIX_BITS = 8;
constexpr int RADIX = 1 << RADIX_BITS;
static_assert(BLOCK == RADIX, "one thread per digit in the block-wide steps");

__global__ void k_iota(int64_t n, int32_t* __restrict__ out) {
    GRID_STRIDE_LOOP(i, n) out[i] = static_cast<int32_t>(i);
}

template <class K>
__global__ void k_radix_count(const K* __restrict__ key, int64_t n, int shift, int64_t tile,
                              int32_t* __restrict__ count) {
    __shared__ int32_t h[RADIX];
    h[threadIdx.x] = 0;
    __syncthreads();
    const int64_t t0 = (int64_t)blockIdx.x * tile;
    const int64_t t1 = t0 + tile < n ? t0 + tile : n;
    for (int64_t i = t0 + threadIdx.x; i < t1; i += BLOCK)
        atomicAdd(&h[static_cast<int>((key[i] >> shift) & (RADIX - 1))], 1);
    __syncthreads();
    count[(int64_t)threadIdx.x * gridDim.x + blockIdx.x] = h[threadIdx.x];
}

template <class K>
__global__ void k_radix_scatter(const K* __restrict__ key, const int32_t* __restrict__ val, int64_t n, int shift,
                                int64_t tile, const int64_t* __restrict__ start, K* __restrict__ key_out,
                                int32_t* __restrict__ val_out) {
    constexpr int WAVES = BLOCK / 64;
    __shared__ int64_t run[RADIX];            // where the block's next element of each digit goes
    __shared__ int32_t wave_n[WAVES][RADIX];  // this round's elements of each digit per wave
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    run[threadIdx.x] = start[(int64_t)threadIdx.x * gridDim.x + blockIdx.x];
    const int64_t t0 = (int64_t)blockIdx.x * tile;
    const int64_t t1 = t0 + tile < n ? t0 + tile : n;
    const uint64_t lower = (uint64_t(1) << lane) - 1;
    for (int64_t r0 = t0; r0 < t1; r0 += BLOCK) {
#pragma unroll
        for (int k = 0; k < WAVES; ++k) wave_n[k][threadIdx.x] = 0;
        __syncthreads();
        const int64_t i = r0 + threadIdx.x;
        const bool in = i < t1;
        const K kv = in ? key[i] : K(0);
        const int d = static_cast<int>((kv >> shift) & (RADIX - 1));
        // lanes of this wave holding the same digit
        uint64_t same = __ballot(in);
#pragma unroll
        for (int bit = 0; bit < RADIX_BITS; ++bit) {
            const uint64_t ones = __ballot((d >> bit) & 1);
            same &= (d >> bit) & 1 ? ones : ~ones;
        }
        const int before = __popcll(same & lower);
        if (in && before == 0) wave_n[w][d] = __popcll(same);
        __syncthreads();
        if (in) {
            int64_t pos = run[d] + before;
            for (int k = 0; k < w; ++k) pos += wave_n[k][d];
            key_out[pos] = kv;
            val_out[pos] = val[i];
        }
        __syncthreads();
        int32_t add = 0;
#pragma unroll
        for (int k = 0; k < WAVES; ++k) add += wave_n[k][threadIdx.x];
        run[threadIdx.x] += add;
        __syncthreads();
    }
}

// perm = the indices 0..n-1 ordered by key, ties in index order, over the
// low `bits` bits of the keys (key is overwritten).
template <class K>
void sort_indices(dec_ctx* ctx, DBuf<K>& key, int64_t n, int bits, DBuf<int32_t>& perm) {
    hipStream_t s = ctx->stream;
    perm.alloc(ctx, n);
    hipLaunchKernelGGL(k_iota, dim3(grid_for(n)), dim3(BLOCK), 0, s, n, perm.p);
    DBuf<K> key2;
    DBuf<int32_t> val2;
    key2.alloc(ctx, n);
    val2.alloc(ctx, n);
    // tiles of at least 16 rounds, so that a block's fixed costs are spread
    const int64_t per_block = 16 * (int64_t)BLOCK;
    int64_t G = (n + per_block - 1) / per_block;
    const int64_t cap = 8 * (int64_t)ctx->num_cus;
    if (G > cap) G = cap;
    if (G < 1) G = 1;
    const int64_t tile = ((n + G - 1) / G + BLOCK - 1) / BLOCK * BLOCK;
    DBuf<int32_t> count;
    DBuf<int64_t> start;
    count.alloc(ctx, RADIX * G);
    start.alloc(ctx, RADIX * G + 1);
    for (int shift = 0; shift < bits; shift += RADIX_BITS) {
        hipLaunchKernelGGL(k_radix_count<K>, dim3(G), dim3(BLOCK), 0, s, key.p, n, shift, tile, count.p);
        scan_exclusive_i32_to_i64(ctx, count.p, start.p, RADIX * G, false);
        hipLaunchKernelGGL(k_radix_scatter<K>, dim3(G), dim3(BLOCK), 0, s, key.p, perm.p, n, shift, tile, start.p,
                           key2.p, val2.p);
        HIP_CHECK(hipGetLastError());
        key.swap(key2);
        perm.swap(val2);
    }
    ctx->sync();  // the second buffers are released on return
}

int bits_for(uint64_t n) {  // bits of the largest key below n
    int b = 1;
    while (b < 64 && (uint64_t(1) << b) < n) ++b;
    return b;
}

}  // namespace

extern "C" int dec_reorder(dec_ctx* ctx, int32_t order, int64_t V, const double* xyz, int64_t T,
                           const int32_t* tets, double* xyz_out, int32_t* tets_out, int32_t* vperm_out,
                           int32_t* tperm_out) {
    if (!ctx) return DEC_EINVAL;
    try {
        DEC_REQUIRE(order == DEC_ORDER_LEXICOGRAPHIC || order == DEC_ORDER_MORTON, DEC_EINVAL, "unknown order");
        DEC_REQUIRE(V > 0 && T > 0 && V < (int64_t(1) << 31) && T < (int64_t(1) << 31), DEC_EINVAL, "bad sizes");
        DEC_REQUIRE(xyz && tets && xyz_out && tets_out, DEC_EINVAL, "NULL array");
        DEC_REQUIRE(xyz_out != xyz && tets_out != tets, DEC_EINVAL, "outputs must not alias the inputs");
        ctx->set_device();
        hipStream_t s = ctx->stream;
        // bounding box and the cell grid
        const unsigned nb = grid_for(V, BLOCK, 1024);
        DBuf<double> part, box;
        part.alloc(ctx, 6 * (int64_t)nb);
        box.alloc(ctx, 6);
        hipLaunchKernelGGL(k_bbox, dim3(nb), dim3(BLOCK), 0, s, V, xyz, part.p);
        hipLaunchKernelGGL(k_bbox_fold, dim3(1), dim3(64), 0, s, (int)nb, part.p, box.p);
        double bb[6];
        std::memcpy(bb, ctx->readback(box.p, sizeof(bb)), sizeof(bb));
        for (int a = 0; a < 3; ++a)
            DEC_REQUIRE(std::isfinite(bb[a]) && std::isfinite(bb[3 + a]), DEC_EINVAL, "non-finite coordinates");
        Grid g;
        // B = the smallest integer with B^3 >= V (found exactly, whatever cbrt rounds to)
        g.B = std::llround(std::cbrt(static_cast<double>(V)));
        if (g.B < 1) g.B = 1;
        while (g.B * g.B * g.B < V) ++g.B;
        while (g.B > 1 && (g.B - 1) * (g.B - 1) * (g.B - 1) >= V) --g.B;
        for (int a = 0; a < 3; ++a) {
            g.lo[a] = bb[a];
            const double ext = bb[3 + a] - bb[a];
            g.s[a] = ext > 0.0 ? static_cast<double>(g.B) / ext : 0.0;
        }
        // cell keys: lexicographic in [0, B^3), or Morton in [0, 2^(3k)) with 2^k >= B
        int kbits = 0;
        while ((int64_t(1) << kbits) < g.B) ++kbits;
        const int cbits = order == DEC_ORDER_MORTON ? (3 * kbits > 0 ? 3 * kbits : 1)
                                                    : bits_for(static_cast<uint64_t>(g.B * g.B * g.B));
        // vertices: by cell, then original index
        DBuf<uint64_t> cell;
        DBuf<int32_t> perm, inv;
        DBuf<unsigned> bad;
        cell.alloc(ctx, V);
        bad.alloc(ctx, 1);
        bad.zero();
        hipLaunchKernelGGL(k_point_cell, dim3(grid_for(V)), dim3(BLOCK), 0, s, V, xyz, g,
                           (int)(order == DEC_ORDER_MORTON), cell.p, bad.p);
        DEC_REQUIRE(*static_cast<unsigned*>(ctx->readback(bad.p, sizeof(unsigned))) == 0, DEC_EINVAL,
                    "non-finite coordinates");
        sort_indices(ctx, cell, V, cbits, perm);
        inv.alloc(ctx, V);
        hipLaunchKernelGGL(k_apply_vperm, dim3(grid_for(V)), dim3(BLOCK), 0, s, V, perm.p, xyz, xyz_out, inv.p);
        // tets: by smallest new vertex, then original index
        DBuf<uint32_t> tkey;
        DBuf<int32_t> tperm;
        DBuf<unsigned> err;
        tkey.alloc(ctx, T);
        err.alloc(ctx, 1);
        err.zero();
        hipLaunchKernelGGL(k_tet_key, dim3(grid_for(T)), dim3(BLOCK), 0, s, T, V, tets, inv.p, tkey.p, err.p);
        const unsigned e = *static_cast<unsigned*>(ctx->readback(err.p, sizeof(unsigned)));
        DEC_REQUIRE(e == 0, DEC_ETOPO, "tet vertex index out of range");
        sort_indices(ctx, tkey, T, bits_for(static_cast<uint64_t>(V)), tperm);
        hipLaunchKernelGGL(k_apply_tperm, dim3(grid_for(T)), dim3(BLOCK), 0, s, T, tperm.p, tets, inv.p, tets_out);
        HIP_CHECK(hipGetLastError());
        if (vperm_out) HIP_CHECK(hipMemcpyAsync(vperm_out, perm.p, V * sizeof(int32_t), hipMemcpyDeviceToDevice, s));
        if (tperm_out) HIP_CHECK(hipMemcpyAsync(tperm_out, tperm.p, T * sizeof(int32_t), hipMemcpyDeviceToDevice, s));
        ctx->sync();  // the temporaries are released on return
    } catch (const DecError& e) {
        ctx->last_error = e.msg;
        return e.code;
    }
    return DEC_OK;
}
