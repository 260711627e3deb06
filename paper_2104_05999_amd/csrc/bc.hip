// Boundary data (eqs. 3-4 and 12-13 restated for vertex unknowns).
//
// * Parts of the mesh that cracks cut off from every Dirichlet vertex
//   (connected components of the graph of edges with *1 != 0) have no unique
//   solution; they are found with a union-find over those edges and pinned
//   to T = 0.
// * Neumann faces load b_v -= f0_v A*_{v,f}, A*_{v,f} the circumcentric
//   part of boundary face f belonging to vertex v.
// * Dirichlet and pinned rows/columns are eliminated symmetrically: for a
//   free row, b_i -= sum_j L_ij T_j over Dirichlet j; fixed rows and columns
//   become identity rows with b = T0 (or 0 when pinned).  The pattern stays.
//
// Compiled without floating-point contraction (fixed operation order).
#include "common.h"
#include "row_scan.h"
#include "uf.h"

void refresh_sell_values(dec_mesh* m);
void assemble_values(dec_mesh* m);

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

__device__ d3 tri_circumcentre(d3 p0, d3 p1, d3 p2) {
    const d3 a = sub(p1, p0), b = sub(p2, p0);
    const d3 axb = cross(a, b);
    const double sa = dot(a, a), sb = dot(b, b);
    const d3 num = cross(sub(scale(sa, b), scale(sb, a)), axb);
    const double den = 2.0 * dot(axb, axb);
    return {p0.x + num.x / den, p0.y + num.y / den, p0.z + num.z / den};
}

__device__ double edge_to_face(d3 pi, d3 pj, d3 pk, d3 cf) {
    const d3 m = {0.5 * (pi.x + pj.x), 0.5 * (pi.y + pj.y), 0.5 * (pi.z + pj.z)};
    const d3 e = sub(pj, pi), w = sub(pk, pi);
    const double f = dot(w, e) / dot(e, e);
    d3 u = sub(w, scale(f, e));
    const double nu = sqrt(dot(u, u));
    u = {u.x / nu, u.y / nu, u.z / nu};
    return dot(sub(cf, m), u);
}

__device__ __forceinline__ int vget(const int4& q, int k) {
    return k == 0 ? q.x : (k == 1 ? q.y : (k == 2 ? q.z : q.w));
}

__global__ void k_bc_init(int64_t V, const int8_t* __restrict__ bc_type, const double* __restrict__ bc_value,
                          double* __restrict__ dval, unsigned* __restrict__ err) {
    GRID_STRIDE_LOOP(v, V) {
        const int8_t t = bc_type[v];
        if (t < 0 || t > 2) atomicOr(err, 1u);
        dval[v] = (t == 1) ? bc_value[v] : 0.0;
    }
}

// Components of the graph of edges with *1 != 0, in two passes over the rows.
// k_uf_tiles: each workgroup joins, in LDS, the edges between vertices of its
// own tile of UF_TILE consecutive vertices, then stores as every vertex's
// parent the root of its part of the tile (that part's smallest vertex).
// k_uf_cross: the edges between tiles, each from its lower end, through the
// global union-find.  The forest that results has the same components and
// the same roots (each component's smallest vertex) as one global pass over
// all edges, but only the edges whose ends lie in different tiles meet the
// device-scope atomics: on a lattice numbered plane by plane, with planes
// larger than a tile, the edges between planes and a few more.
// NT threads per tile: a mesh of few tiles takes 1024 (two rows per thread, as
// the rows' dependent loads are the latency), one of many takes 256 (more
// tiles resident per CU).
constexpr int UF_TILE = 2048;

template <int NT>
__global__ __launch_bounds__(NT) void k_uf_tiles(int64_t V, const int32_t* __restrict__ row_ptr,
                                                    const int32_t* __restrict__ col,
                                                    const int32_t* __restrict__ nz_edge,
                                                    const double* __restrict__ star1, int32_t* __restrict__ parent) {
    __shared__ int32_t lp[UF_TILE];
    const int64_t v0 = (int64_t)blockIdx.x * UF_TILE;
    const int n = (int)(V - v0 < UF_TILE ? V - v0 : UF_TILE);
    for (int i = threadIdx.x; i < n; i += NT) lp[i] = i;
    __syncthreads();
    for (int i = threadIdx.x; i < n; i += NT) {
        const int64_t v = v0 + i;
        const int32_t k1 = row_ptr[v + 1];
        for (int32_t k = row_ptr[v]; k < k1; k += 8) {  // eight entries' loads at a time
            int32_t c[8], e[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) c[u] = k + u < k1 ? col[k + u] : -1;
#pragma unroll
            for (int u = 0; u < 8; ++u) e[u] = (c[u] > v && c[u] < v0 + n) ? nz_edge[k + u] : -1;
#pragma unroll
            for (int u = 0; u < 8; ++u)
                if (e[u] >= 0 && star1[e[u]] != 0.0)
                    uf_union<__HIP_MEMORY_SCOPE_WORKGROUP>(lp, i, (int32_t)(c[u] - v0));
        }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < n; i += NT)
        parent[v0 + i] = (int32_t)(v0 + uf_find<__HIP_MEMORY_SCOPE_WORKGROUP>(lp, i));
}

// A wavefront takes 64 consecutive rows, one per lane.  A lane's first edge
// between tiles joins the sets holding parent[v] and parent[c]; when the lane
// before it names the same two values, the two edges join the same two sets
// (values of parent[] are always ancestors within a set), so only the first
// lane of such a run makes the device-scope union.  On a lattice that leaves
// about one union per wavefront for the edges between planes.
__global__ __launch_bounds__(BLOCK) void k_uf_cross(int64_t V, const int32_t* __restrict__ row_ptr,
                                                   const int32_t* __restrict__ col, const int32_t* __restrict__ nz_edge,
                                                   const double* __restrict__ star1, int32_t* parent) {
    const int lane = threadIdx.x & 63;
    const int64_t stride = (int64_t)gridDim.x * BLOCK;
    for (int64_t base = (int64_t)blockIdx.x * BLOCK + (threadIdx.x & ~63); base < V; base += stride) {
        const int64_t v = base + lane;
        int32_t c1 = -1;
        if (v < V) {
            const int64_t tile_end = (v / UF_TILE + 1) * UF_TILE;
            const int32_t k1 = row_ptr[v + 1];
            for (int32_t k = row_ptr[v]; k < k1; k += 8) {  // eight entries' loads at a time
                int32_t c[8];
#pragma unroll
                for (int u = 0; u < 8; ++u) c[u] = k + u < k1 ? col[k + u] : -1;
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    if (c[u] < tile_end) continue;  // a lower neighbour, or one in v's own tile
                    const int32_t e = nz_edge[k + u];
                    if (e < 0 || star1[e] == 0.0) continue;
                    if (c1 < 0)
                        c1 = c[u];
                    else
                        uf_union(parent, (int32_t)v, c[u]);
                }
            }
        }
        const int32_t a = c1 >= 0 ? __hip_atomic_load(parent + v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : -1;
        const int32_t b = c1 >= 0 ? __hip_atomic_load(parent + c1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : -1;
        const int32_t pa = __shfl_up(a, 1), pb = __shfl_up(b, 1);
        if (c1 >= 0 && !(lane > 0 && pa == a && pb == b)) uf_union(parent, (int32_t)v, c1);
    }
}

__global__ void k_uf_anchor(int64_t V, const int8_t* __restrict__ bc_type, int32_t* parent,
                            uint32_t* __restrict__ anchored) {
    GRID_STRIDE_LOOP(v, V) {
        if (bc_type[v] == 1) anchored[uf_find(parent, (int32_t)v)] = 1u;
    }
}

__global__ void k_mark_fixed(int64_t V, const int8_t* __restrict__ bc_type, int32_t* parent,
                             const uint32_t* __restrict__ anchored, uint8_t* __restrict__ fixed,
                             unsigned long long* __restrict__ n_pinned) {
    unsigned long long local = 0;
    GRID_STRIDE_LOOP(v, V) {
        uint8_t f = 0;
        if (bc_type[v] == 1)
            f = 1;
        else if (!anchored[uf_find(parent, (int32_t)v)]) {
            f = 2;
            ++local;
        }
        fixed[v] = f;
    }
    if (local) atomicAdd(n_pinned, local);
}

// Neumann load g_v = sum over Neumann faces at v (ascending tet, then local
// face) of f0_v * (v's circumcentric part of the face).
__constant__ int kFaceV[4][3] = {{1, 2, 3}, {0, 2, 3}, {0, 1, 3}, {0, 1, 2}};

__global__ void k_neumann_load(int64_t V, const int8_t* __restrict__ bc_type, const double* __restrict__ f0,
                               const int4* __restrict__ tets, const uint8_t* __restrict__ bface,
                               const int64_t* __restrict__ vt_ptr, const int32_t* __restrict__ vt_list,
                               const double* __restrict__ xyz, double* __restrict__ g) {
    GRID_STRIDE_LOOP(v, V) {
        double acc = 0.0;
        if (bc_type[v] == 2) {
            for (int64_t j = vt_ptr[v]; j < vt_ptr[v + 1]; ++j) {
                const int t = vt_list[j];
                const uint8_t mask = bface[t];
                if (!mask) continue;
                const int4 q = tets[t];
                for (int k = 0; k < 4; ++k) {
                    if (!(mask & (1u << k))) continue;
                    int verts[3];
                    int a = -1;
                    bool ok = true;
                    for (int r = 0; r < 3; ++r) {
                        verts[r] = vget(q, kFaceV[k][r]);
                        const int8_t ty = bc_type[verts[r]];
                        ok &= (ty == 1 || ty == 2);
                        if (verts[r] == v) a = r;
                    }
                    if (a < 0 || !ok) continue;
                    const d3 p[3] = {load3(xyz + 3 * (int64_t)verts[0]), load3(xyz + 3 * (int64_t)verts[1]),
                                     load3(xyz + 3 * (int64_t)verts[2])};
                    const d3 cf = tri_circumcentre(p[0], p[1], p[2]);
                    const int b = a == 0 ? 1 : 0;
                    const int c = a == 2 ? 1 : 2;
                    const d3 dab = sub(p[b], p[a]), dac = sub(p[c], p[a]);
                    const double lab = sqrt(dot(dab, dab));
                    const double lac = sqrt(dot(dac, dac));
                    const double hab = edge_to_face(p[a], p[b], p[c], cf);
                    const double hac = edge_to_face(p[a], p[c], p[b], cf);
                    const double part = 0.5 * (0.5 * lab) * hab + 0.5 * (0.5 * lac) * hac;
                    acc = acc + f0[v] * part;
                }
            }
        }
        g[v] = acc;
    }
}

// b for free rows: (-g_v) - sum_k L_vk xd_k (all stored entries, ascending);
// fixed rows: T0 (Dirichlet) or 0 (pinned).  One ROWG-lane group per row
// loads runs of ROWG entries (coalesced); the products are added in entry
// order (row_seq_sum), the same sequential sum as a one-thread loop.
constexpr int ROWG = 16;

__global__ void k_rhs(int64_t V, const int32_t* __restrict__ row_ptr, const int32_t* __restrict__ col,
                      const double* __restrict__ val, const uint8_t* __restrict__ fixed,
                      const double* __restrict__ dval, const double* __restrict__ g, double* __restrict__ b) {
    const int gl = threadIdx.x & (ROWG - 1);
    int64_t v0, v1;
    block_range(V, &v0, &v1);
    for (int64_t v = v0 + threadIdx.x / ROWG; v < v1; v += blockDim.x / ROWG) {
        const uint8_t f = fixed[v];
        if (f) {
            if (gl == 0) b[v] = (f == 1) ? dval[v] : 0.0;
            continue;
        }
        const int32_t r0 = row_ptr[v], n = row_ptr[v + 1] - r0;
        double acc = 0.0;  // lane 0's
        for (int32_t k0 = 0; k0 < n; k0 += ROWG) {
            const int32_t k = k0 + gl;
            const double t = k < n ? val[r0 + k] * dval[col[r0 + k]] : 0.0;
            acc = row_seq_sum(acc, t, k < n, gl);
        }
        if (gl == 0) {
            const double base = g ? (0.0 - g[v]) : 0.0;
            b[v] = base - acc;
        }
    }
}

__global__ void k_eliminate(int64_t V, const int32_t* __restrict__ row_ptr, const int32_t* __restrict__ col,
                            const uint8_t* __restrict__ fixed, double* __restrict__ val64, float* __restrict__ val32,
                            const int32_t* __restrict__ diag_pos, double* __restrict__ inv64,
                            float* __restrict__ inv32, unsigned long long* __restrict__ nonpos) {
    unsigned long long bad = 0;
    RANGE_LOOP(v, V) {
        const bool fv = fixed[v] != 0;
        const int32_t k1 = row_ptr[v + 1];
        for (int32_t k = row_ptr[v]; k < k1; k += 8) {  // eight entries' loads at a time
            int32_t c[8];
            bool fc[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) c[u] = k + u < k1 ? col[k + u] : -1;
#pragma unroll
            for (int u = 0; u < 8; ++u) fc[u] = c[u] >= 0 && (fv || fixed[c[u]]);
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                if (!fc[u]) continue;
                const double nv = (c[u] == v && fv) ? 1.0 : 0.0;
                val64[k + u] = nv;
                val32[k + u] = static_cast<float>(nv);
            }
        }
        const int32_t d = diag_pos[v];
        inv64[v] = 1.0 / val64[d];
        inv32[v] = 1.0f / val32[d];
        bad += !(val64[d] > 0.0) || !isfinite(val64[d]);
    }
    if (bad) atomicAdd(nonpos, bad);  // rows whose diagonal is not positive and finite
}

void apply_bc_device(dec_mesh* m, const int8_t* bc_type, const double* bc_value, const double* f0) {
    dec_ctx* ctx = m->ctx;
    hipStream_t s = ctx->stream;
    const int64_t V = m->V;
    DEC_REQUIRE(m->assembled, DEC_ESTATE, "dec_apply_bc needs dec_assemble first");
    // boundary data applied before to this assembly overwrote the rows and columns it
    // fixed: start again from L (and until this call completes, there is no system to solve)
    if (m->bc_ready) assemble_values(m);
    m->bc_ready = false;
    DBuf<unsigned> flags;
    flags.alloc(ctx, 16);
    flags.zero();
    DBuf<int32_t> parent;
    parent.alloc(ctx, V);
    m->bc_value.alloc(ctx, V);
    hipLaunchKernelGGL(k_bc_init, dim3(grid_for(V)), dim3(BLOCK), 0, s, V, bc_type, bc_value, m->bc_value.p,
                       flags.p);
    HIP_CHECK(hipGetLastError());
    unsigned e0 = *static_cast<unsigned*>(ctx->readback(flags.p, sizeof(unsigned)));
    DEC_REQUIRE(e0 == 0, DEC_EINVAL, "bc_type must be 0, 1 or 2");

    // parts of the graph of edges with *1 != 0 holding no Dirichlet vertex are pinned
    const unsigned tiles = (unsigned)((V + UF_TILE - 1) / UF_TILE);
    if (tiles < 512)
        hipLaunchKernelGGL(k_uf_tiles<1024>, dim3(tiles), dim3(1024), 0, s, V, m->row_ptr.p, m->col.p, m->nz_edge.p,
                           m->star1.p, parent.p);
    else
        hipLaunchKernelGGL(k_uf_tiles<256>, dim3(tiles), dim3(256), 0, s, V, m->row_ptr.p, m->col.p, m->nz_edge.p,
                           m->star1.p, parent.p);
    hipLaunchKernelGGL(k_uf_cross, dim3(grid_for(V)), dim3(BLOCK), 0, s, V, m->row_ptr.p, m->col.p, m->nz_edge.p,
                       m->star1.p, parent.p);
    DBuf<uint32_t> anchored;
    anchored.alloc(ctx, V);
    anchored.zero();
    hipLaunchKernelGGL(k_uf_anchor, dim3(grid_for(V)), dim3(BLOCK), 0, s, V, bc_type, parent.p, anchored.p);
    m->fixed.alloc(ctx, V);
    DBuf<unsigned long long> npin;  // pinned vertices, rows with a diagonal that is not positive
    npin.alloc(ctx, 2);
    npin.zero();
    hipLaunchKernelGGL(k_mark_fixed, dim3(grid_for(V)), dim3(BLOCK), 0, s, V, bc_type, parent.p, anchored.p,
                       m->fixed.p, npin.p);
    HIP_CHECK(hipGetLastError());
    DBuf<double> gload;
    if (f0) {
        gload.alloc(ctx, V);
        hipLaunchKernelGGL(k_neumann_load, dim3(grid_for(V)), dim3(BLOCK), 0, s, V, bc_type, f0,
                           reinterpret_cast<const int4*>(m->tets.p), m->tet_bface.p, m->vt_ptr.p, m->vt_list.p,
                           m->xyz.p, gload.p);
    }
    m->rhs.alloc(ctx, V);
    hipLaunchKernelGGL(k_rhs, dim3(grid_xcd(V, BLOCK / ROWG)), dim3(BLOCK), 0, s, V, m->row_ptr.p, m->col.p, m->val64.p,
                       m->fixed.p, m->bc_value.p, f0 ? gload.p : nullptr, m->rhs.p);
    m->invdiag64.alloc(ctx, V);
    m->invdiag32.alloc(ctx, V);
    hipLaunchKernelGGL(k_eliminate, dim3(grid_xcd(V)), dim3(BLOCK), 0, s, V, m->row_ptr.p, m->col.p, m->fixed.p,
                       m->val64.p, m->val32.p, m->diag_pos.p, m->invdiag64.p, m->invdiag32.p, npin.p + 1);
    HIP_CHECK(hipGetLastError());
    refresh_sell_values(m);
    unsigned long long h[2];
    std::memcpy(h, ctx->readback(npin.p, sizeof(h)), sizeof(h));
    m->n_pinned = (int64_t)h[0];
    m->neumann = f0 != nullptr;
    m->diag_positive = h[1] == 0;
    m->bc_ready = true;
    m->fsai.ready = false;
    m->jsplit.ready = false;
}

}  // namespace

void apply_bc_internal(dec_mesh* m, const int8_t* bc_type, const double* bc_value, const double* f0) {
    apply_bc_device(m, bc_type, bc_value, f0);
}

extern "C" int dec_apply_bc(dec_mesh* m, const int8_t* bc_type, const double* bc_value, const double* neumann_f0,
                            int64_t* n_pinned_out, double* b_out) {
    if (!m) return DEC_EINVAL;
    try {
        DEC_REQUIRE(!m->dual, DEC_ESTATE, "dec_apply_bc is for meshes of vertex unknowns");
        DEC_REQUIRE(bc_type && bc_value, DEC_EINVAL, "NULL bc_type or bc_value");
        m->ctx->set_device();
        apply_bc_device(m, bc_type, bc_value, neumann_f0);
        if (n_pinned_out) *n_pinned_out = m->n_pinned;
        if (b_out)
            HIP_CHECK(hipMemcpyAsync(b_out, m->rhs.p, m->V * sizeof(double), hipMemcpyDeviceToDevice, m->ctx->stream));
    } catch (const DecError& e) {
        m->ctx->last_error = e.msg;
        return e.code;
    }
    return DEC_OK;
}
