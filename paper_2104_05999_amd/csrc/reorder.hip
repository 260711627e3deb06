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
// with the indices in ascending order, so the result is unique, and its cost
// is linear however unevenly the points fill the cells.
// The Z (Morton) order is offered beside it: cells by the interleaved bits of
// (x cell, y cell, z cell) (z in the lowest bit), which keeps neighbours in
// all three directions close in memory.
#include <cmath>
#include <cstring>

#include <rocprim/device/device_radix_sort.hpp>
#include <rocprim/iterator/counting_iterator.hpp>

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

// perm = the indices 0..n-1 ordered by key, ties in index order (a stable
// radix sort over the low `bits` bits of the keys); keys are left sorted.
template <class K>
void sort_indices(dec_ctx* ctx, DBuf<K>& key, int64_t n, int bits, DBuf<int32_t>& perm) {
    DBuf<K> key_out;
    key_out.alloc(ctx, n);
    perm.alloc(ctx, n);
    const rocprim::counting_iterator<int32_t> idx(0);
    size_t bytes = 0;
    HIP_CHECK(rocprim::radix_sort_pairs(nullptr, bytes, key.p, key_out.p, idx, perm.p, static_cast<size_t>(n), 0,
                                        static_cast<unsigned>(bits), ctx->stream));
    DBuf<uint8_t> tmp;
    tmp.alloc(ctx, bytes ? bytes : 1);
    HIP_CHECK(rocprim::radix_sort_pairs(tmp.p, bytes, key.p, key_out.p, idx, perm.p, static_cast<size_t>(n), 0,
                                        static_cast<unsigned>(bits), ctx->stream));
    ctx->sync();  // tmp and key_out are released on return
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
