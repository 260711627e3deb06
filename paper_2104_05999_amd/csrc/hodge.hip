// Circumcentric Hodge star *1 with conductivity and cracks (Sections 2.1, 2.5).
//
// Geometry (once per mesh): every tet computes the signed area of the part
// of each of its six edges' dual 2-cells that it holds -- the planar
// quadrilateral (edge midpoint, circumcentre of face 1, tet circumcentre,
// circumcentre of face 2) in the edge's bisector plane, in a closed form
// (cotangent of the face angles, distance of the tet circumcentre to the
// face planes) -- then every edge
// gathers its pieces in ascending tet order (no atomics), snaps near-zero
// areas (|*e| <= 1e-12 |e|^2) to zero and stores |*e| / |e|.
//
// Per call: the crack predicate marks the edges whose segment passes
// through a penny disc, and *1_e = kappa_e * (|*e| / |e|), zero when cut.
//
// This file is compiled without floating-point contraction and follows a
// fixed operation order, so that integer decisions taken from floating
// point (the cut mask, the snap) match an FP64 reference evaluated in the
// same order.
#include "common.h"

namespace {

struct d3 {
    double x, y, z;
};
__device__ __forceinline__ d3 sub(d3 a, d3 b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
__device__ __forceinline__ double dot(d3 a, d3 b) { return (a.x * b.x + a.y * b.y) + a.z * b.z; }
__device__ __forceinline__ d3 cross(d3 a, d3 b) {
    return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}
__device__ __forceinline__ d3 scale(double s, d3 a) { return {s * a.x, s * a.y, s * a.z}; }
__device__ __forceinline__ d3 load3(const double* p) { return {p[0], p[1], p[2]}; }

// c_T = p0 + (|a|^2 (b x c) + |b|^2 (c x a) + |c|^2 (a x b)) / (2 a.(b x c))
__device__ d3 tet_circumcentre(d3 p0, d3 p1, d3 p2, d3 p3) {
    const d3 a = sub(p1, p0), b = sub(p2, p0), c = sub(p3, p0);
    const d3 bc = cross(b, c), ca = cross(c, a), ab = cross(a, b);
    const double sa = dot(a, a), sb = dot(b, b), sc = dot(c, c);
    const d3 num = {(sa * bc.x + sb * ca.x) + sc * ab.x, (sa * bc.y + sb * ca.y) + sc * ab.y,
                    (sa * bc.z + sb * ca.z) + sc * ab.z};
    const double den = 2.0 * dot(a, bc);
    return {p0.x + num.x / den, p0.y + num.y / den, p0.z + num.z / den};
}

// Signed elementary dual area of edge (i, j) inside a tet with other vertices
// k, l: the quad (edge midpoint, circumcentre of face ijk, tet circumcentre,
// circumcentre of face ijl) in the edge's bisector plane has area
//     A = 1/2 [ h(e -> f_ijk) h(f_ijk -> T) + h(e -> f_ijl) h(f_ijl -> T) ],
// with h(e -> f) the in-plane signed distance from the edge midpoint to the
// face circumcentre (positive toward the face's third vertex) and h(f -> T)
// the signed distance from the face to the tet circumcentre along the face
// normal (positive toward the opposite vertex).  Evaluated as:
//  * h(e -> f_ijk) = |e|/2 cot(angle at k) = |e|/2 (p_i - p_k).(p_j - p_k) / |n_f|,
//    |n_f| = twice the face area (the circumcentre sits |e|/2 cot from the
//    edge midpoint on its perpendicular bisector);
//  * h(f -> T) = sgn (c_T - p_a).n_f / |n_f| for any face vertex p_a (the face
//    circumcentre lies in the face plane, so only the tet circumcentre's
//    distance to that plane enters);
// so A = |e|/4 [ dot_k H_l + dot_l H_k ] with H_f = sgn (c_T - p_a).n_f / |n_f|^2
// for the face opposite vertex f.  Seven divisions and six square roots per
// tet.
__global__ void k_elementary_areas(int64_t T, const int32_t* __restrict__ tets, const double* __restrict__ xyz,
                                   double* __restrict__ elem) {
    constexpr int FA[4] = {1, 0, 0, 0}, FB[4] = {2, 2, 1, 1}, FC[4] = {3, 3, 3, 2};  // face opposite vertex f
    constexpr int EI[6] = {0, 0, 0, 1, 1, 2}, EJ[6] = {1, 2, 3, 2, 3, 3};
    constexpr int EK[6] = {2, 1, 1, 0, 0, 0}, EL[6] = {3, 3, 2, 3, 2, 1};
    GRID_STRIDE_LOOP(t, T) {
        const int4 q = reinterpret_cast<const int4*>(tets)[t];
        const d3 p[4] = {load3(xyz + 3 * (int64_t)q.x), load3(xyz + 3 * (int64_t)q.y),
                         load3(xyz + 3 * (int64_t)q.z), load3(xyz + 3 * (int64_t)q.w)};
        const d3 ct = tet_circumcentre(p[0], p[1], p[2], p[3]);
        double H[4];
#pragma unroll
        for (int f = 0; f < 4; ++f) {
            const d3 pa = p[FA[f]];
            const d3 n = cross(sub(p[FB[f]], pa), sub(p[FC[f]], pa));
            const double sgn = dot(n, sub(p[f], pa)) < 0.0 ? -1.0 : 1.0;
            H[f] = sgn * dot(sub(ct, pa), n) / dot(n, n);
        }
#pragma unroll
        for (int e = 0; e < 6; ++e) {
            const d3 pi = p[EI[e]], pj = p[EJ[e]], pk = p[EK[e]], pl = p[EL[e]];
            const d3 d = sub(pj, pi);
            const double le = sqrt(dot(d, d));
            const double dk = dot(sub(pi, pk), sub(pj, pk));
            const double dl = dot(sub(pi, pl), sub(pj, pl));
            elem[e * T + t] = 0.25 * le * (dk * H[EL[e]] + dl * H[EK[e]]);
        }
    }
}

// |*e| in ascending tet order, snapped, over |e|.  Up to RING incidences are
// loaded at once (their loads do not wait on each other), then added in order.
// The elementary areas sit local edge by local edge (elem[e * T + t]): the
// gathers of neighbouring edges then share more cache lines than with a
// tet's six areas side by side.
constexpr int RING = 8;

__global__ void k_edge_geometry(int64_t E, int64_t T, const int32_t* __restrict__ edges,
                                const double* __restrict__ xyz, const int64_t* __restrict__ et_ptr,
                                const int32_t* __restrict__ et_inc,
                                const double* __restrict__ elem, double* __restrict__ geo) {
    // incidence tet * 6 + local edge e -> elem[e * T + tet]
    auto at = [&](int32_t sl) { return elem[(int64_t)(sl % 6) * T + sl / 6]; };
    const FrontRange fr = front_range(E);
    for (int64_t e = fr.first; e < fr.end; e += fr.step) {
        const int64_t i0 = et_ptr[e];
        const int m = static_cast<int>(et_ptr[e + 1] - i0);
        double area = 0.0;
        if (m <= RING) {
            double a[RING];
#pragma unroll
            for (int r = 0; r < RING; ++r) a[r] = r < m ? at(et_inc[i0 + r]) : 0.0;
#pragma unroll
            for (int r = 0; r < RING; ++r)
                if (r < m) area += a[r];
        } else {
            for (int r = 0; r < m; ++r) area += at(et_inc[i0 + r]);
        }
        const d3 d = sub(load3(xyz + 3 * (int64_t)edges[2 * e + 1]), load3(xyz + 3 * (int64_t)edges[2 * e]));
        const double len = sqrt(dot(d, d));
        if (fabs(area) <= 1e-12 * len * len) area = 0.0;
        geo[e] = area / len;
    }
}

constexpr int kMaxDiscsLds = 256;  // 256 * 7 doubles = 14 KiB of LDS per block
constexpr int kBinnedFrom = 64;    // more discs than this: spatially binned cut

__global__ void k_crack_cut(int64_t E, const int32_t* __restrict__ edges, const double* __restrict__ xyz,
                            int32_t n_discs, const double* __restrict__ discs, uint8_t* __restrict__ cut) {
    __shared__ double sd[kMaxDiscsLds * 7];
    for (int32_t base = 0; base < n_discs || base == 0; base += kMaxDiscsLds) {
        const int32_t nd = min(kMaxDiscsLds, n_discs - base);
        __syncthreads();
        for (int i = threadIdx.x; i < nd * 7; i += blockDim.x) sd[i] = discs[(int64_t)base * 7 + i];
        __syncthreads();
        for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < E;
             e += (int64_t)gridDim.x * blockDim.x) {
            const d3 p0 = load3(xyz + 3 * (int64_t)edges[2 * e]);
            const d3 p1 = load3(xyz + 3 * (int64_t)edges[2 * e + 1]);
            uint8_t hit = base == 0 ? 0 : cut[e];
            for (int i = 0; i < nd && !hit; ++i) {
                const double* d = sd + 7 * i;
                const double cx = d[0], cy = d[1], cz = d[2], nx = d[3], ny = d[4], nz = d[5], r = d[6];
                const double s0 = ((p0.x - cx) * nx + (p0.y - cy) * ny) + (p0.z - cz) * nz;
                const double s1 = ((p1.x - cx) * nx + (p1.y - cy) * ny) + (p1.z - cz) * nz;
                if ((s0 < 0.0) == (s1 < 0.0)) continue;
                const double t = s0 / (s0 - s1);
                const double qx = p0.x + t * (p1.x - p0.x);
                const double qy = p0.y + t * (p1.y - p0.y);
                const double qz = p0.z + t * (p1.z - p0.z);
                const double d2 = ((qx - cx) * (qx - cx) + (qy - cy) * (qy - cy)) + (qz - cz) * (qz - cz);
                if (d2 <= r * r) hit = 1;
            }
            cut[e] = hit;
        }
        if (n_discs == 0) break;
    }
}

// ---- spatially binned cut for many discs
// The mesh's bounding box is split into kBins^3 cells.  A disc is listed in
// every cell its bounding box, inflated by the longest half edge, overlaps;
// an edge can only cross a disc if its midpoint lies in that inflated box,
// so each edge tests the discs of its midpoint's cell only.  The decision
// per (edge, disc) is the same predicate, so the mask is unchanged.
constexpr int kBins = 32;

struct Bins {
    double lo[3];
    double inv[3];  // cells per unit length
};

// cell index along one axis, clamped to [0, kBins); NaN maps to 0
__device__ __forceinline__ int bin_of(double x, double lo, double inv) {
    const double t = (x - lo) * inv;
    if (!(t > 0.0)) return 0;
    if (!(t < (double)(kBins - 1))) return kBins - 1;
    return (int)t;
}

// per-block partial extents: [block][7] = min xyz, max xyz, longest half edge
__global__ void k_geom_extent(int64_t V, const double* __restrict__ xyz, int64_t E, const int32_t* __restrict__ edges,
                              double* __restrict__ part) {
    __shared__ double red[7][BLOCK];
    double mn[3] = {INFINITY, INFINITY, INFINITY}, mx[3] = {-INFINITY, -INFINITY, -INFINITY}, he = 0.0;
    GRID_STRIDE_LOOP(i, V) {
        for (int a = 0; a < 3; ++a) {
            const double v = xyz[3 * i + a];
            mn[a] = fmin(mn[a], v);
            mx[a] = fmax(mx[a], v);
        }
    }
    GRID_STRIDE_LOOP(e, E) {
        const d3 d = sub(load3(xyz + 3 * (int64_t)edges[2 * e + 1]), load3(xyz + 3 * (int64_t)edges[2 * e]));
        he = fmax(he, 0.5 * sqrt(dot(d, d)));
    }
    for (int a = 0; a < 3; ++a) {
        red[a][threadIdx.x] = mn[a];
        red[3 + a][threadIdx.x] = mx[a];
    }
    red[6][threadIdx.x] = he;
    __syncthreads();
    if (threadIdx.x < 7) {
        double r = red[threadIdx.x][0];
        for (int t = 1; t < BLOCK; ++t)
            r = threadIdx.x < 3 ? fmin(r, red[threadIdx.x][t]) : fmax(r, red[threadIdx.x][t]);
        part[7 * blockIdx.x + threadIdx.x] = r;
    }
}

// min / max are exact, so the fold order does not matter
__global__ __launch_bounds__(BLOCK) void k_geom_extent_fold(int nblocks, const double* __restrict__ part,
                                                            double* __restrict__ out) {
    __shared__ double red[7][BLOCK];
    double r[7];
    for (int a = 0; a < 7; ++a) r[a] = a < 3 ? INFINITY : -INFINITY;
    for (int b = threadIdx.x; b < nblocks; b += BLOCK)
        for (int a = 0; a < 7; ++a) r[a] = a < 3 ? fmin(r[a], part[7 * b + a]) : fmax(r[a], part[7 * b + a]);
    for (int a = 0; a < 7; ++a) red[a][threadIdx.x] = r[a];
    __syncthreads();
    for (int w = BLOCK / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w)
            for (int a = 0; a < 7; ++a)
                red[a][threadIdx.x] = a < 3 ? fmin(red[a][threadIdx.x], red[a][threadIdx.x + w])
                                            : fmax(red[a][threadIdx.x], red[a][threadIdx.x + w]);
        __syncthreads();
    }
    if (threadIdx.x < 7) out[threadIdx.x] = red[threadIdx.x][0];
}

__device__ __forceinline__ void disc_cells(const double* d, double reach, const Bins& B, int lo[3], int hi[3]) {
    const double R = fabs(d[6]) + reach;
    for (int a = 0; a < 3; ++a) {
        lo[a] = bin_of(d[a] - R, B.lo[a], B.inv[a]);
        hi[a] = bin_of(d[a] + R, B.lo[a], B.inv[a]);
    }
}

// One block per disc (grid-stride over discs), its threads over the disc's
// cells.  Counts are order-free; the order inside a cell's list is not
// fixed, which the cut (an "any disc" test) does not see.
__global__ void k_bin_count(int32_t n, const double* __restrict__ discs, double reach, Bins B, int32_t* __restrict__ cnt) {
    for (int32_t i = blockIdx.x; i < n; i += gridDim.x) {
        int lo[3], hi[3];
        disc_cells(discs + 7 * (int64_t)i, reach, B, lo, hi);
        const int nx = hi[0] - lo[0] + 1, ny = hi[1] - lo[1] + 1, nz = hi[2] - lo[2] + 1;
        for (int k = threadIdx.x; k < nx * ny * nz; k += blockDim.x) {
            const int x = lo[0] + k / (ny * nz), y = lo[1] + (k / nz) % ny, z = lo[2] + k % nz;
            atomicAdd(&cnt[(x * kBins + y) * kBins + z], 1);
        }
    }
}

__global__ void k_bin_fill(int32_t n, const double* __restrict__ discs, double reach, Bins B,
                           const int64_t* __restrict__ off, int32_t* __restrict__ fill, int32_t* __restrict__ list) {
    for (int32_t i = blockIdx.x; i < n; i += gridDim.x) {
        int lo[3], hi[3];
        disc_cells(discs + 7 * (int64_t)i, reach, B, lo, hi);
        const int nx = hi[0] - lo[0] + 1, ny = hi[1] - lo[1] + 1, nz = hi[2] - lo[2] + 1;
        for (int k = threadIdx.x; k < nx * ny * nz; k += blockDim.x) {
            const int x = lo[0] + k / (ny * nz), y = lo[1] + (k / nz) % ny, z = lo[2] + k % nz;
            const int c = (x * kBins + y) * kBins + z;
            list[off[c] + atomicAdd(&fill[c], 1)] = i;
        }
    }
}

__global__ void k_crack_cut_binned(int64_t E, const int32_t* __restrict__ edges, const double* __restrict__ xyz,
                                   const double* __restrict__ discs, Bins B, const int64_t* __restrict__ off,
                                   const int32_t* __restrict__ list, uint8_t* __restrict__ cut) {
    RANGE_LOOP(e, E) {
        const d3 p0 = load3(xyz + 3 * (int64_t)edges[2 * e]);
        const d3 p1 = load3(xyz + 3 * (int64_t)edges[2 * e + 1]);
        const int bx = bin_of(0.5 * (p0.x + p1.x), B.lo[0], B.inv[0]);
        const int by = bin_of(0.5 * (p0.y + p1.y), B.lo[1], B.inv[1]);
        const int bz = bin_of(0.5 * (p0.z + p1.z), B.lo[2], B.inv[2]);
        const int c = (bx * kBins + by) * kBins + bz;
        uint8_t hit = 0;
        for (int64_t k = off[c]; k < off[c + 1] && !hit; ++k) {
            const double* d = discs + 7 * (int64_t)list[k];
            const double cx = d[0], cy = d[1], cz = d[2], nx = d[3], ny = d[4], nz = d[5], r = d[6];
            const double s0 = ((p0.x - cx) * nx + (p0.y - cy) * ny) + (p0.z - cz) * nz;
            const double s1 = ((p1.x - cx) * nx + (p1.y - cy) * ny) + (p1.z - cz) * nz;
            if ((s0 < 0.0) == (s1 < 0.0)) continue;
            const double t = s0 / (s0 - s1);
            const double qx = p0.x + t * (p1.x - p0.x);
            const double qy = p0.y + t * (p1.y - p0.y);
            const double qz = p0.z + t * (p1.z - p0.z);
            const double d2 = ((qx - cx) * (qx - cx) + (qy - cy) * (qy - cy)) + (qz - cz) * (qz - cz);
            if (d2 <= r * r) hit = 1;
        }
        cut[e] = hit;
    }
}

__global__ void k_star1(int64_t E, const double* __restrict__ geo, const double* __restrict__ kappa,
                        const uint8_t* __restrict__ cut, double* __restrict__ star1) {
    GRID_STRIDE_LOOP(e, E) {
        const double k = kappa ? kappa[e] : 1.0;
        star1[e] = cut[e] ? 0.0 : k * geo[e];
    }
}

void ensure_geometry(dec_mesh* m) {
    if (m->geo_ready) return;
    dec_ctx* ctx = m->ctx;
    DBuf<double> ext, part;
    const int nb = (int)grid_for(m->E, BLOCK, 1024);
    ext.alloc(ctx, 7);
    part.alloc(ctx, 7 * (int64_t)nb);
    hipLaunchKernelGGL(k_geom_extent, dim3(nb), dim3(BLOCK), 0, ctx->stream, m->V, m->xyz.p, m->E, m->edges.p, part.p);
    hipLaunchKernelGGL(k_geom_extent_fold, dim3(1), dim3(BLOCK), 0, ctx->stream, nb, part.p, ext.p);
    std::memcpy(m->extent, ctx->readback(ext.p, 7 * sizeof(double)), sizeof(m->extent));
    DBuf<double> elem;
    elem.alloc(ctx, 6 * m->T);
    hipLaunchKernelGGL(k_elementary_areas, dim3(grid_for(m->T)), dim3(BLOCK), 0, ctx->stream, m->T, m->tets.p,
                       m->xyz.p, elem.p);
    m->geo.alloc(ctx, m->E);
    hipLaunchKernelGGL(k_edge_geometry, dim3(grid_xcd(m->E, BLOCK, 1 << 20)), dim3(BLOCK), 0, ctx->stream, m->E, m->T,
                       m->edges.p, m->xyz.p, m->et_ptr.p, m->et_inc.p, elem.p, m->geo.p);
    HIP_CHECK(hipGetLastError());
    ctx->sync();  // elem is released on return
    m->geo_ready = true;
}

}  // namespace

// Used by the crack-growth and serving paths as well as dec_hodge1.
void hodge1_device(dec_mesh* m, const double* kappa, int32_t n_cracks, const double* cracks) {
    dec_ctx* ctx = m->ctx;
    ensure_geometry(m);
    m->cut.alloc(ctx, m->E);
    m->star1.alloc(ctx, m->E);
    if (n_cracks <= kBinnedFrom) {
        const unsigned g = grid_for(m->E, BLOCK, 8 * (int64_t)ctx->num_cus);
        hipLaunchKernelGGL(k_crack_cut, dim3(g), dim3(BLOCK), 0, ctx->stream, m->E, m->edges.p, m->xyz.p,
                           n_cracks, cracks, m->cut.p);
    } else {
        Bins B;
        for (int a = 0; a < 3; ++a) {
            const double ext = m->extent[3 + a] - m->extent[a];
            B.lo[a] = m->extent[a];
            B.inv[a] = ext > 0.0 ? kBins / ext : 1.0;
        }
        // longest half edge, with a relative margin for the rounding of midpoints and cells
        const double reach = m->extent[6] * (1.0 + 1e-9) + 1e-12;
        const int64_t ncell = (int64_t)kBins * kBins * kBins;
        DBuf<int32_t> cnt, fill, list;
        DBuf<int64_t> off;
        cnt.alloc(ctx, ncell);
        cnt.zero();
        const dim3 disc_grid(n_cracks < 65536 ? n_cracks : 65536);
        hipLaunchKernelGGL(k_bin_count, disc_grid, dim3(64), 0, ctx->stream, n_cracks, cracks, reach, B, cnt.p);
        off.alloc(ctx, ncell + 1);
        const int64_t total = scan_exclusive_i32_to_i64(ctx, cnt.p, off.p, ncell, true);
        list.alloc(ctx, total > 0 ? total : 1);
        cnt.zero();
        hipLaunchKernelGGL(k_bin_fill, disc_grid, dim3(64), 0, ctx->stream, n_cracks, cracks, reach, B, off.p, cnt.p,
                           list.p);
        hipLaunchKernelGGL(k_crack_cut_binned, dim3(grid_xcd(m->E)), dim3(BLOCK), 0, ctx->stream, m->E, m->edges.p,
                           m->xyz.p, cracks, B, off.p, list.p, m->cut.p);
        HIP_CHECK(hipGetLastError());
        ctx->sync();  // the bins are released on return
    }
    hipLaunchKernelGGL(k_star1, dim3(grid_for(m->E)), dim3(BLOCK), 0, ctx->stream, m->E, m->geo.p, kappa,
                       m->cut.p, m->star1.p);
    HIP_CHECK(hipGetLastError());
    m->star_ready = true;
    m->assembled = false;
    m->bc_ready = false;
}

extern "C" int dec_hodge1(dec_mesh* m, const double* kappa, int32_t n_cracks, const double* cracks,
                          uint8_t* cut_out, double* star1_out) {
    if (!m) return DEC_EINVAL;
    dec_ctx* ctx = m->ctx;
    try {
        DEC_REQUIRE(!m->dual, DEC_ESTATE, "dec_hodge1 is for meshes of vertex unknowns");
        DEC_REQUIRE(n_cracks >= 0, DEC_EINVAL, "negative crack count");
        DEC_REQUIRE(n_cracks == 0 || cracks, DEC_EINVAL, "NULL crack array");
        ctx->set_device();
        hodge1_device(m, kappa, n_cracks, cracks);
        if (cut_out)
            HIP_CHECK(hipMemcpyAsync(cut_out, m->cut.p, m->E, hipMemcpyDeviceToDevice, ctx->stream));
        if (star1_out)
            HIP_CHECK(hipMemcpyAsync(star1_out, m->star1.p, m->E * sizeof(double), hipMemcpyDeviceToDevice,
                                     ctx->stream));
    } catch (const DecError& e) {
        ctx->last_error = e.msg;
        return e.code;
    }
    return DEC_OK;
}
