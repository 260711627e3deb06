// Topology of the tetrahedral complex (Section 2.1: cells, incidence, d0):
// vertex -> tet lists, the edge set in lexicographic (lo, hi) order, the
// edge -> tet incidence in ascending tet order, the static CSR pattern of
// L = d0^T *1 d0 (full edge graph plus diagonal) and the boundary faces.
//
// Every list is built per vertex from that vertex's sorted tet list, so the
// result is independent of thread scheduling: integer atomics only count
// (deterministic totals) or claim slots whose order the per-vertex sort then
// fixes.  Compiled without floating-point contraction: the zero-volume test
// must take the same decision as the FP64 reference.
#include <climits>

#include "common.h"
#include "wave_atomic.h"

namespace {

// local edge index of the local vertex pair (a, b), a < b:
// (0,1) (0,2) (0,3) (1,2) (1,3) (2,3)
__device__ __forceinline__ int local_edge(int a, int b) {
    return a == 0 ? b - 1 : (a == 1 ? b + 1 : 5);
}

__device__ __forceinline__ int vget(const int4& q, int k) {
    return k == 0 ? q.x : (k == 1 ? q.y : (k == 2 ? q.z : q.w));
}

__global__ void k_tet_check(const int4* __restrict__ tets, int64_t T, int64_t V, const double* __restrict__ xyz,
                            unsigned* __restrict__ err) {
    GRID_STRIDE_LOOP(t, T) {
        const int4 q = tets[t];
        const int a[4] = {q.x, q.y, q.z, q.w};
        bool oob = false;
        for (int k = 0; k < 4; ++k) oob |= (a[k] < 0) | (static_cast<int64_t>(a[k]) >= V);
        if (oob) {
            atomicOr(err, 1u);
            continue;
        }
        if (a[0] == a[1] || a[0] == a[2] || a[0] == a[3] || a[1] == a[2] || a[1] == a[3] || a[2] == a[3]) {
            atomicOr(err, 2u);
            continue;
        }
        const double* p0 = xyz + 3 * (int64_t)a[0];
        const double* p1 = xyz + 3 * (int64_t)a[1];
        const double* p2 = xyz + 3 * (int64_t)a[2];
        const double* p3 = xyz + 3 * (int64_t)a[3];
        const double ax = p1[0] - p0[0], ay = p1[1] - p0[1], az = p1[2] - p0[2];
        const double bx = p2[0] - p0[0], by = p2[1] - p0[1], bz = p2[2] - p0[2];
        const double cx = p3[0] - p0[0], cy = p3[1] - p0[1], cz = p3[2] - p0[2];
        const double det = (ax * (by * cz - bz * cy) + ay * (bz * cx - bx * cz)) + az * (bx * cy - by * cx);
        if (det == 0.0) atomicOr(err, 4u);
        if (!isfinite(det)) atomicOr(err, 32u);  // a NaN or infinite coordinate
    }
}

// Vertex-to-tet counts and slots, one atomic per distinct vertex of a
// wavefront (wave_claim): the 16 tets of a wavefront share most vertices.
__global__ void k_vt_count(const int32_t* __restrict__ tets, int64_t n4, int32_t* __restrict__ cnt) {
    GRID_STRIDE_LOOP(i, n4) (void)wave_claim(cnt, tets[i]);
}

__global__ void k_vt_fill(const int32_t* __restrict__ tets, int64_t n4, const int64_t* __restrict__ vt_ptr,
                          int32_t* __restrict__ fill, int32_t* __restrict__ vt_list) {
    GRID_STRIDE_LOOP(i, n4) {
        const int v = tets[i];
        const int pos = wave_claim(fill, v);
        vt_list[vt_ptr[v] + pos] = static_cast<int32_t>(i >> 2);
    }
}

// Sort each vertex's tet list (ascending tet id).  One 32-lane group per
// vertex: a list of at most 32 distinct ids is ranked in registers (rank =
// number of smaller ids) and written back; longer lists are insertion-sorted
// by the group's first lane.
__global__ void k_vt_sort(const int64_t* __restrict__ vt_ptr, int32_t* __restrict__ vt_list, int64_t V) {
    constexpr int W = 32;
    const int lane = threadIdx.x & (W - 1);
    int64_t v0, v1;
    block_range(V, &v0, &v1);
    for (int64_t v = v0 + threadIdx.x / W; v < v1; v += blockDim.x / W) {
        const int64_t b = vt_ptr[v];
        const int d = (int)(vt_ptr[v + 1] - b);
        if (d <= W) {
            const int key = lane < d ? vt_list[b + lane] : INT_MAX;
            int rank = 0;
#pragma unroll
            for (int k = 0; k < W; ++k) rank += __shfl(key, k, W) < key;
            if (lane < d) vt_list[b + rank] = key;
        } else if (lane == 0) {
            for (int64_t i = b + 1; i < b + d; ++i) {
                const int32_t key = vt_list[i];
                int64_t j = i - 1;
                while (j >= b && vt_list[j] > key) {
                    vt_list[j + 1] = vt_list[j];
                    --j;
                }
                vt_list[j + 1] = key;
            }
        }
    }
}

// Neighbour enumeration with one 16-lane group per vertex (four vertices per
// wavefront, so the group reductions stay inside a row of 16 lanes): lane g
// of the group holds tets g and g + 16 of the vertex's sorted tet list in
// registers (entries -1 past the end), tets g + 32, g + 48, ... are read as
// needed.  Each round finds the smallest neighbour w > cur (group minimum)
// and the tets holding it (ballot; each tet holds w at most once).
// INT_MAX: no neighbour left.
constexpr int NG = 16;

__device__ __forceinline__ int group_min(int v) {
#pragma unroll
    for (int off = NG / 2; off > 0; off >>= 1) v = min(v, __shfl_xor(v, off, NG));
    return v;
}

__device__ __forceinline__ int group_sum(int v) {
#pragma unroll
    for (int off = NG / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, NG);
    return v;
}

__device__ __forceinline__ int tet_pos(const int4& q, int w) {
    return q.x == w ? 0 : (q.y == w ? 1 : (q.z == w ? 2 : (q.w == w ? 3 : -1)));
}

// vertices of q above v (-1 entries never are)
__device__ __forceinline__ int above(const int4& q, int v) {
    return (q.x > v) + (q.y > v) + (q.z > v) + (q.w > v);
}

struct GroupTets {
    int4 q0, q1;  // tets g and g + NG of the list
    int t0, t1;   // their ids
};

__device__ __forceinline__ GroupTets load_group_tets(const int4* __restrict__ tets, const int32_t* __restrict__ list,
                                                     int64_t b, int d, int g) {
    GroupTets t;
    const int4 none = make_int4(-1, -1, -1, -1);
    t.t0 = g < d ? list[b + g] : -1;
    t.t1 = g + NG < d ? list[b + g + NG] : -1;
    t.q0 = t.t0 >= 0 ? tets[t.t0] : none;
    t.q1 = t.t1 >= 0 ? tets[t.t1] : none;
    return t;
}

__device__ __forceinline__ void scan_tet(const int4& q, int v, int cur, int* best) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int w = vget(q, r);
        if (w != v && w > cur && w < *best) *best = w;
    }
}

__device__ __forceinline__ int group_next(const int4* __restrict__ tets, const int32_t* __restrict__ list, int64_t b,
                                          int d, int v, int cur, int g, const GroupTets& gt) {
    int best = INT_MAX;
    scan_tet(gt.q0, v, cur, &best);
    scan_tet(gt.q1, v, cur, &best);
    for (int k = g + 2 * NG; k < d; k += NG) scan_tet(tets[list[b + k]], v, cur, &best);
    return group_min(best);
}

// Per vertex: upper neighbours (edges it is the low end of), pattern row
// length, and the incidences of its upper edges -- each tet of v adds one per
// vertex above v, so that count needs no enumeration.
__global__ void k_nbr_count(const int4* __restrict__ tets, const int64_t* __restrict__ vt_ptr,
                            const int32_t* __restrict__ vt_list, int64_t V, int32_t* __restrict__ n_up,
                            int32_t* __restrict__ row_len, int32_t* __restrict__ n_inc) {
    const int g = threadIdx.x & (NG - 1);
    const int64_t ngroups = ((int64_t)gridDim.x * blockDim.x) / NG;
    for (int64_t v = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / NG; v < V; v += ngroups) {
        const int64_t b = vt_ptr[v];
        const int d = (int)(vt_ptr[v + 1] - b);
        const GroupTets gt = load_group_tets(tets, vt_list, b, d, g);
        int inc = above(gt.q0, (int)v) + above(gt.q1, (int)v);
        for (int k = g + 2 * NG; k < d; k += NG) inc += above(tets[vt_list[b + k]], (int)v);
        inc = group_sum(inc);
        int cur = -1, up = 0, all = 0;
        while (true) {
            const int w = group_next(tets, vt_list, b, d, (int)v, cur, g, gt);
            if (w == INT_MAX) break;
            cur = w;
            ++all;
            up += w > v;
        }
        if (g == 0) {
            n_up[v] = up;
            row_len[v] = all + 1;
            n_inc[v] = inc;
        }
    }
}

// Row v of the pattern (lower neighbours, the diagonal, upper neighbours,
// ascending).  Upper neighbours w define the edges (v, w), numbered from
// up_ptr[v] in ascending w -- lexicographic (lo, hi) order overall -- and
// their incidence lists: the tets of v holding w, in ascending tet order, as
// tet * 6 + local edge, from inc_ptr[v] on.  Also the tet -> edge map.
__global__ void k_nbr_fill(const int4* __restrict__ tets, const int64_t* __restrict__ vt_ptr,
                           const int32_t* __restrict__ vt_list, int64_t V, const int64_t* __restrict__ up_ptr,
                           const int64_t* __restrict__ row_ptr, const int64_t* __restrict__ inc_ptr,
                           int32_t* __restrict__ edges, int64_t* __restrict__ et_ptr, int32_t* __restrict__ et_inc,
                           int32_t* __restrict__ tet_edge, int32_t* __restrict__ col, int32_t* __restrict__ nz_edge,
                           int32_t* __restrict__ diag_pos) {
    const int lane = threadIdx.x & 63;
    const int g = threadIdx.x & (NG - 1);
    const int gbase = lane & ~(NG - 1);  // first lane of this group in the wavefront
    const uint64_t below = ((uint64_t)1 << g) - 1;
    const int64_t ngroups = ((int64_t)gridDim.x * blockDim.x) / NG;
    for (int64_t v = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / NG; v < V; v += ngroups) {
        const int64_t b = vt_ptr[v];
        const int d = (int)(vt_ptr[v + 1] - b);
        const GroupTets gt = load_group_tets(tets, vt_list, b, d, g);
        int64_t pos = row_ptr[v], ep = up_ptr[v], ip = inc_ptr[v];
        bool diag = false;
        int cur = -1;
        while (true) {
            const int w = group_next(tets, vt_list, b, d, (int)v, cur, g, gt);
            if (w == INT_MAX) break;
            cur = w;
            if (w > v && !diag) {
                if (g == 0) {
                    col[pos] = (int32_t)v;
                    nz_edge[pos] = -1;
                    diag_pos[v] = (int32_t)pos;
                }
                ++pos;
                diag = true;
            }
            if (g == 0) {
                col[pos] = w;
                nz_edge[pos] = w < v ? -2 : (int32_t)ep;  // lower entries: k_lower_edge_ids
            }
            ++pos;
            if (w < v) continue;
            if (g == 0) {
                edges[2 * ep] = (int32_t)v;
                edges[2 * ep + 1] = w;
                et_ptr[ep] = ip;
            }
            // incidences in ascending tet order: blocks of NG tets, lane order inside a block
            for (int k0 = 0; k0 < d; k0 += NG) {
                const int k = k0 + g;
                int4 q = make_int4(-1, -1, -1, -1);
                int t = -1;
                if (k0 == 0) {
                    q = gt.q0;
                    t = gt.t0;
                } else if (k0 == NG) {
                    q = gt.q1;
                    t = gt.t1;
                } else if (k < d) {
                    t = vt_list[b + k];
                    q = tets[t];
                }
                const int pw = tet_pos(q, w);
                const uint64_t ball = (__ballot(pw >= 0) >> gbase) & ((uint64_t(1) << NG) - 1);
                if (pw >= 0) {
                    const int pv = tet_pos(q, (int)v);
                    const int slot = t * 6 + local_edge(pv < pw ? pv : pw, pv < pw ? pw : pv);
                    et_inc[ip + __popcll(ball & below)] = slot;
                    tet_edge[slot] = (int32_t)ep;
                }
                ip += __popcll(ball);
            }
            ++ep;
        }
        if (!diag && g == 0) {
            col[pos] = (int32_t)v;
            nz_edge[pos] = -1;
            diag_pos[v] = (int32_t)pos;
        }
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) et_ptr[up_ptr[V]] = inc_ptr[V];
}

// Entries (v, w) with w < v belong to edge (w, v), found by binary search in
// w's upper edges (sorted by hi).
__global__ void k_lower_edge_ids(int64_t V, const int64_t* __restrict__ row_ptr, const int32_t* __restrict__ col,
                                 const int64_t* __restrict__ up_ptr, const int32_t* __restrict__ edges,
                                 int32_t* __restrict__ nz_edge, unsigned* __restrict__ err) {
    RANGE_LOOP(v, V) {
        for (int64_t k = row_ptr[v]; k < row_ptr[v + 1]; ++k) {
            const int w = col[k];
            if (w >= v) break;
            int64_t lo = up_ptr[w], hi = up_ptr[w + 1] - 1, found = -1;
            while (lo <= hi) {
                const int64_t mid = (lo + hi) >> 1;
                const int h = edges[2 * mid + 1];
                if (h == v) {
                    found = mid;
                    break;
                }
                if (h < v)
                    lo = mid + 1;
                else
                    hi = mid - 1;
            }
            if (found < 0) atomicOr(err, 8u);
            nz_edge[k] = (int32_t)found;
        }
    }
}

// Faces: face k of tet t is opposite local vertex k.  The tets holding face
// (a, b, c) are those holding both edges (a, b) and (a, c): the intersection
// of two incidence lists, both in ascending tet order (a merge over ~10
// contiguous integers).  The first such tet owns the face.  Four lanes take
// the four faces of a tet (their merges are independent chains of loads) and
// combine their boundary bits with shuffles.
__global__ void k_faces(int64_t T, const int32_t* __restrict__ tet_edge, const int64_t* __restrict__ et_ptr,
                        const int32_t* __restrict__ et_inc, uint8_t* __restrict__ bface,
                        unsigned long long* __restrict__ counts, unsigned* __restrict__ err) {
    __shared__ unsigned long long lds[BLOCK / 64];
    unsigned long long owned = 0, bnd = 0;
    const int k = threadIdx.x & 3;
    const int la = k == 0 ? 1 : 0, lb = k <= 1 ? 2 : 1, lc = k == 3 ? 2 : 3;
    const int ea = local_edge(la, lb), eb = local_edge(la, lc);
    int64_t t_lo, t_hi;
    block_range(T, &t_lo, &t_hi);
    for (int64_t t = t_lo + threadIdx.x / 4; t < t_hi; t += blockDim.x / 4) {
        const int e1 = tet_edge[6 * t + ea];
        const int e2 = tet_edge[6 * t + eb];
        int64_t i = et_ptr[e1], j = et_ptr[e2];
        const int64_t i1 = et_ptr[e1 + 1], j1 = et_ptr[e2 + 1];
        int cnt = 0, first = -1;
        while (i < i1 && j < j1) {
            const int u = et_inc[i] / 6, w = et_inc[j] / 6;
            if (u == w) {
                if (first < 0) first = u;
                ++cnt;
                ++i;
                ++j;
            } else if (u < w) {
                ++i;
            } else {
                ++j;
            }
        }
        if (cnt > 2) atomicOr(err, 16u);
        unsigned mask = cnt == 1 ? 1u << k : 0u;
        bnd += cnt == 1;
        owned += first == t;
        mask |= __shfl_xor(mask, 1);
        mask |= __shfl_xor(mask, 2);
        if (k == 0) bface[t] = static_cast<uint8_t>(mask);
    }
    owned = block_sum(owned, lds);
    bnd = block_sum(bnd, lds);
    if (threadIdx.x == 0) {
        if (owned) atomicAdd(&counts[0], owned);
        if (bnd) atomicAdd(&counts[1], bnd);
    }
}

std::string topo_message(unsigned err) {
    if (err & 1u) return "tet vertex index out of range";
    if (err & 2u) return "tet repeats a vertex";
    if (err & 32u) return "non-finite vertex coordinate";
    if (err & 4u) return "tet of zero volume";
    if (err & 16u) return "face shared by more than two tets";
    if (err & 8u) return "internal: lower edge not found";
    return "invalid mesh";
}

}  // namespace

// m (1 to 3) exclusive scans of int32 arrays of the same length in one set
// of launches, as scan_exclusive_i32_to_i64 does one; totals (when given)
// receives their m totals with one synchronisation (api.hip).
void scan_exclusive_multi(dec_ctx* ctx, int m, const int32_t* const* in, int64_t* const* out, int64_t n,
                          int64_t* totals);

// Build every topology array of m (V, T set) from device xyz / tets.
void build_topology_device(dec_mesh* m, const double* xyz, const int32_t* tets) {
    dec_ctx* ctx = m->ctx;
    hipStream_t s = ctx->stream;
    const int64_t V = m->V, T = m->T;
    m->xyz.alloc(ctx, 3 * V);
    m->tets.alloc(ctx, 4 * T);
    HIP_CHECK(hipMemcpyAsync(m->xyz.p, xyz, 3 * V * sizeof(double), hipMemcpyDeviceToDevice, s));
    HIP_CHECK(hipMemcpyAsync(m->tets.p, tets, 4 * T * sizeof(int32_t), hipMemcpyDeviceToDevice, s));
    const int4* tq = reinterpret_cast<const int4*>(m->tets.p);

    DBuf<unsigned> err;
    err.alloc(ctx, 1);
    err.zero();
    hipLaunchKernelGGL(k_tet_check, dim3(grid_for(T)), dim3(BLOCK), 0, s, tq, T, V, m->xyz.p, err.p);
    HIP_CHECK(hipGetLastError());
    unsigned e0 = *static_cast<unsigned*>(ctx->readback(err.p, sizeof(unsigned)));
    if (e0) dec_fail(DEC_ETOPO, topo_message(e0));

    // vertex -> tets
    DBuf<int32_t> cnt;
    cnt.alloc(ctx, V);
    cnt.zero();
    hipLaunchKernelGGL(k_vt_count, dim3(grid_for(4 * T)), dim3(BLOCK), 0, s, m->tets.p, 4 * T, cnt.p);
    m->vt_ptr.alloc(ctx, V + 1);
    scan_exclusive_i32_to_i64(ctx, cnt.p, m->vt_ptr.p, V, false);
    m->vt_list.alloc(ctx, 4 * T);
    cnt.zero();
    hipLaunchKernelGGL(k_vt_fill, dim3(grid_for(4 * T)), dim3(BLOCK), 0, s, m->tets.p, 4 * T, m->vt_ptr.p, cnt.p,
                       m->vt_list.p);
    hipLaunchKernelGGL(k_vt_sort, dim3(grid_xcd(V, BLOCK / 32)), dim3(BLOCK), 0, s, m->vt_ptr.p, m->vt_list.p, V);
    HIP_CHECK(hipGetLastError());

    // neighbours: counts, then edges, incidences and the CSR pattern (one 16-lane group per vertex)
    DBuf<int32_t> n_up, row_len, n_inc;
    n_up.alloc(ctx, V);
    row_len.alloc(ctx, V);
    n_inc.alloc(ctx, V);
    hipLaunchKernelGGL(k_nbr_count, dim3(grid_for(NG * V)), dim3(BLOCK), 0, s, tq, m->vt_ptr.p, m->vt_list.p, V,
                       n_up.p, row_len.p, n_inc.p);
    HIP_CHECK(hipGetLastError());
    m->up_ptr.alloc(ctx, V + 1);
    DBuf<int64_t> row_ptr64, inc_ptr;
    row_ptr64.alloc(ctx, V + 1);
    inc_ptr.alloc(ctx, V + 1);
    const int32_t* scan_in[3] = {n_up.p, row_len.p, n_inc.p};
    int64_t* scan_out[3] = {m->up_ptr.p, row_ptr64.p, inc_ptr.p};
    int64_t tot[3];
    scan_exclusive_multi(ctx, 3, scan_in, scan_out, V, tot);
    const int64_t E = tot[0], nnz = tot[1], ninc = tot[2];
    DEC_REQUIRE(nnz == V + 2 * E, DEC_ETOPO, "internal: pattern size mismatch");
    DEC_REQUIRE(ninc == 6 * T, DEC_ETOPO, "internal: incidence count mismatch");
    DEC_REQUIRE(nnz < (int64_t(1) << 31) && 6 * T < (int64_t(1) << 31), DEC_EINVAL,
                "mesh too large for int32 CSR indices");
    m->E = E;
    m->nnz = nnz;

    m->edges.alloc(ctx, 2 * E);
    m->et_ptr.alloc(ctx, E + 1);
    m->et_inc.alloc(ctx, 6 * T);
    DBuf<int32_t> tet_edge;
    tet_edge.alloc(ctx, 6 * T);
    m->col.alloc(ctx, nnz);
    m->nz_edge.alloc(ctx, nnz);
    m->diag_pos.alloc(ctx, V);
    hipLaunchKernelGGL(k_nbr_fill, dim3(grid_for(NG * V)), dim3(BLOCK), 0, s, tq, m->vt_ptr.p, m->vt_list.p, V,
                       m->up_ptr.p, row_ptr64.p, inc_ptr.p, m->edges.p, m->et_ptr.p, m->et_inc.p, tet_edge.p,
                       m->col.p, m->nz_edge.p, m->diag_pos.p);
    // [0] owned faces, [1] boundary faces, [2] error bits (low word): one read-back for all three
    DBuf<unsigned long long> fc;
    fc.alloc(ctx, 3);
    fc.zero();
    unsigned* err2 = reinterpret_cast<unsigned*>(fc.p + 2);
    hipLaunchKernelGGL(k_lower_edge_ids, dim3(grid_xcd(V)), dim3(BLOCK), 0, s, V, row_ptr64.p, m->col.p,
                       m->up_ptr.p, m->edges.p, m->nz_edge.p, err2);
    HIP_CHECK(hipGetLastError());
    m->row_ptr.alloc(ctx, V + 1);
    copy_i64_to_i32(ctx, row_ptr64.p, m->row_ptr.p, V + 1);

    // faces
    m->tet_bface.alloc(ctx, T);
    hipLaunchKernelGGL(k_faces, dim3(grid_xcd(4 * T)), dim3(BLOCK), 0, s, T, tet_edge.p, m->et_ptr.p,
                       m->et_inc.p, m->tet_bface.p, fc.p, err2);
    HIP_CHECK(hipGetLastError());
    unsigned long long hc[3];
    std::memcpy(hc, ctx->readback(fc.p, sizeof(hc)), sizeof(hc));
    m->F = (int64_t)hc[0];
    m->Fb = (int64_t)hc[1];
    const unsigned e1 = static_cast<unsigned>(hc[2] & 0xffffffffu);
    if (e1) dec_fail(DEC_ETOPO, topo_message(e1));
}


// The topology of src copied into the empty mesh m (same device, m's stream),
// with src's geometry (the dual areas over edge lengths) when src has it and
// its sliced-ELL pattern when src built one for the same pruning: what
// build_topology_device, the geometry and the pattern build would compute for
// src's xyz and tets, without their kernels and read-backs.
void clone_topology_device(dec_mesh* m, const dec_mesh* src) {
    DEC_REQUIRE(!src->dual && src->tets.p && src->vt_list.p && src->et_inc.p, DEC_EINVAL,
                "a request's mesh must be a mesh of vertex unknowns from dec_build_topology");
    dec_ctx* ctx = m->ctx;
    hipStream_t s = ctx->stream;
    m->V = src->V;
    m->T = src->T;
    m->E = src->E;
    m->F = src->F;
    m->Fb = src->Fb;
    m->nnz = src->nnz;
    auto dup = [&](auto& dst, const auto& from, int64_t count) {
        dst.alloc(ctx, count);
        if (count) HIP_CHECK(hipMemcpyAsync(dst.p, from.p, count * sizeof(*from.p), hipMemcpyDeviceToDevice, s));
    };
    const int64_t V = m->V, T = m->T, E = m->E, nnz = m->nnz;
    dup(m->xyz, src->xyz, 3 * V);
    dup(m->tets, src->tets, 4 * T);
    dup(m->vt_ptr, src->vt_ptr, V + 1);
    dup(m->vt_list, src->vt_list, 4 * T);
    dup(m->edges, src->edges, 2 * E);
    dup(m->up_ptr, src->up_ptr, V + 1);
    dup(m->et_ptr, src->et_ptr, E + 1);
    dup(m->et_inc, src->et_inc, 6 * T);
    dup(m->tet_bface, src->tet_bface, T);
    dup(m->row_ptr, src->row_ptr, V + 1);
    dup(m->col, src->col, nnz);
    dup(m->nz_edge, src->nz_edge, nnz);
    dup(m->diag_pos, src->diag_pos, V);
    if (src->geo_ready) {
        dup(m->geo, src->geo, E);
        std::memcpy(m->extent, src->extent, sizeof(m->extent));
        m->geo_ready = true;
    }
    const SellMatrix& S = src->sell;
    if (S.nslices && S.src.p && src->prune_geometric_zeros == m->prune_geometric_zeros) {
        SellMatrix& D = m->sell;
        D.nslices = S.nslices;
        D.entries = S.entries;
        D.kept = S.kept;
        D.ntab = S.ntab;
        dup(D.ptr, S.ptr, S.nslices + 1);
        dup(D.col, S.col, S.entries);
        dup(D.src, S.src, S.entries);
        if (S.dcol.p) dup(D.dcol, S.dcol, S.entries);
        if (S.tcol.p) dup(D.tcol, S.tcol, S.entries);
        if (S.otab.p) dup(D.otab, S.otab, S.ntab);
        D.val64.alloc(ctx, S.entries);
        D.val32.alloc(ctx, S.entries);
    }
}

extern "C" {

int dec_build_topology(dec_ctx* ctx, int64_t V, const double* xyz, int64_t T, const int32_t* tets, dec_mesh** out) {
    if (!ctx || !out) return DEC_EINVAL;
    *out = nullptr;
    dec_mesh* m = new dec_mesh();
    m->ctx = ctx;
    m->owner = ctx;
    ctx->live_children += 1;
    try {
        DEC_REQUIRE(V > 0 && T > 0 && xyz && tets, DEC_EINVAL, "empty mesh or NULL array");
        DEC_REQUIRE(V < (int64_t(1) << 31), DEC_EINVAL, "too many vertices for int32 indices");
        ctx->set_device();
        m->V = V;
        m->T = T;
        build_topology_device(m, xyz, tets);
    } catch (const DecError& e) {
        ctx->last_error = e.msg;
        delete m;
        return e.code;
    }
    *out = m;
    return DEC_OK;
}

int dec_mesh_info(const dec_mesh* m, int64_t* V, int64_t* T, int64_t* E, int64_t* F, int64_t* Fb, int64_t* nnz) {
    if (!m) return DEC_EINVAL;
    if (V) *V = m->V;
    if (T) *T = m->T;
    if (E) *E = m->E;
    if (F) *F = m->F;
    if (Fb) *Fb = m->Fb;
    if (nnz) *nnz = m->nnz;
    return DEC_OK;
}

int dec_get_edges(const dec_mesh* m, int32_t* edges) {
    if (!m) return DEC_EINVAL;
    if (!edges) return null_argument(m->ctx, "dec_get_edges");
    try {
        HIP_CHECK(hipMemcpyAsync(edges, m->edges.p, 2 * m->E * sizeof(int32_t), hipMemcpyDeviceToDevice,
                                 m->ctx->stream));
    } catch (const DecError& e) {
        m->ctx->last_error = e.msg;
        return e.code;
    }
    return DEC_OK;
}

int dec_mesh_destroy(dec_mesh* m) {
    if (!m) return DEC_EINVAL;
    try {
        m->ctx->sync();
    } catch (const DecError&) {
    }
    delete m;
    return DEC_OK;
}

}  // extern "C"
