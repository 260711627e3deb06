// Heat flux and effective conductivity (Section 2.5): with T fixed on two
// opposite faces, the effective conductivity equals the flux density through
// either Dirichlet face.  (L T)_v over the operator before boundary
// elimination is the heat leaving v's dual cell, so
//     Q_in = sum over inflow-face vertices of (L T)_v,
//     Q_out = -sum over outflow-face vertices of (L T)_v,
// and, without a Neumann load, the dissipated energy
// E = sum_e *1_e (T_hi - T_lo)^2 equals Q_in dT at the exact solution, so
// k_eff = E length / (area dT^2), which is second order in the solution's
// error; with a Neumann load the energy also holds the work of the
// prescribed fluxes, and k_eff = Q length / (area dT), the flux density
// itself through a Dirichlet side: Q = Q_in when inflow vertices are marked,
// else Q_out.  Deterministic block partials.
#include <climits>
#include <cmath>

#include "solver.h"

namespace {

// Sums of k_flux: Q_in, Q_out, energy, inflow vertices, outflow vertices.
constexpr int FLUX_SUMS = 5;

// Q_in / Q_out from the rows of the two Dirichlet faces only (side != 0);
// the energy edge by edge (coalesced over the edge arrays).  Partials per
// block, folded in a fixed order by the last block.
__global__ __launch_bounds__(BLOCK) void k_flux(int64_t V, int64_t E, const int32_t* __restrict__ row_ptr,
                                                const int32_t* __restrict__ col, const int32_t* __restrict__ nz_edge,
                                                const int32_t* __restrict__ edges, const double* __restrict__ star1,
                                                const double* __restrict__ T, const int8_t* __restrict__ side,
                                                double* __restrict__ edge_flux, double* __restrict__ partials,
                                                double* __restrict__ out, unsigned* __restrict__ counter) {
    __shared__ double lds[BLOCK / 64];
    double qin = 0.0, qout = 0.0, en = 0.0, nin = 0.0, nout = 0.0;
    if (side) {
        int64_t i0, i1;
        block_range(V, &i0, &i1);
        for (int64_t v = i0 + threadIdx.x; v < i1; v += BLOCK) {
            const int8_t sd = side[v];
            if (sd != 1 && sd != 2) continue;
            nin += sd == 1;
            nout += sd == 2;
            const double tv = T[v];
            double o = 0.0;
            for (int32_t k = row_ptr[v]; k < row_ptr[v + 1]; ++k) {
                const int32_t e = nz_edge[k];
                if (e < 0) continue;
                o += star1[e] * (tv - T[col[k]]);
            }
            if (sd == 1) qin += o;
            if (sd == 2) qout -= o;
        }
    }
    {
        int64_t e0, e1;
        block_range(E, &e0, &e1);
        const int2* ed = reinterpret_cast<const int2*>(edges);
        for (int64_t e = e0 + threadIdx.x; e < e1; e += BLOCK) {
            const int2 lh = ed[e];
            const double s = star1[e];
            const double tl = T[lh.x], th = T[lh.y];
            const double d = th - tl;
            en += s * d * d;
            if (edge_flux) edge_flux[e] = s * (tl - th);
        }
    }
    const int G = gridDim.x;
    const double in[FLUX_SUMS] = {qin, qout, en, nin, nout};
    for (int k = 0; k < FLUX_SUMS; ++k) {
        const double t = block_sum(in[k], lds);
        if (threadIdx.x == 0) partials[k * G + blockIdx.x] = t;
    }
    if (last_block_arrived(counter)) {
        for (int k = 0; k < FLUX_SUMS; ++k) {
            const double t = reduce_partials(partials + k * G, G, lds);
            if (threadIdx.x == 0) out[k] = t;
        }
        if (threadIdx.x == 0) *counter = 0;
    }
}

// Largest heat-flux density over the eligible faces (Section 3, deterministic
// cracking): density_e = |*1_e (T_hi - T_lo)| / |*e| with |*e| = geo_e |e|
// the dual area.  Pairs (density, edge) are ordered by density, then by the
// smaller edge id; that order is total, so the block partials and their fold
// give the same pair whatever the schedule.
__device__ __forceinline__ bool flux_better(double v, int64_t e, double bv, int64_t be) {
    return v > bv || (v == bv && e < be);
}

__global__ __launch_bounds__(BLOCK) void k_max_flux_partial(int64_t E, const int32_t* __restrict__ edges,
                                                            const double* __restrict__ xyz,
                                                            const double* __restrict__ geo,
                                                            const double* __restrict__ star1,
                                                            const double* __restrict__ T,
                                                            const uint8_t* __restrict__ eligible,
                                                            double* __restrict__ pv, int64_t* __restrict__ pe) {
    __shared__ double sv[BLOCK];
    __shared__ int64_t se[BLOCK];
    double bv = -1.0;
    int64_t be = INT64_MAX;
    RANGE_LOOP(e, E) {
        const double g = geo[e], s1 = star1[e];
        if (eligible ? eligible[e] == 0 : (g == 0.0 || s1 == 0.0)) continue;
        const int32_t lo = edges[2 * e], hi = edges[2 * e + 1];
        const double dx = xyz[3 * (int64_t)hi] - xyz[3 * (int64_t)lo];
        const double dy = xyz[3 * (int64_t)hi + 1] - xyz[3 * (int64_t)lo + 1];
        const double dz = xyz[3 * (int64_t)hi + 2] - xyz[3 * (int64_t)lo + 2];
        const double area = fabs(g * sqrt((dx * dx + dy * dy) + dz * dz));
        const double v = fabs(s1 * (T[hi] - T[lo])) / area;
        if (!(v >= 0.0) || isinf(v)) continue;  // no face (zero area) or a non-finite solution
        if (flux_better(v, e, bv, be)) {
            bv = v;
            be = e;
        }
    }
    sv[threadIdx.x] = bv;
    se[threadIdx.x] = be;
    __syncthreads();
    for (int w = BLOCK / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w && flux_better(sv[threadIdx.x + w], se[threadIdx.x + w], sv[threadIdx.x], se[threadIdx.x])) {
            sv[threadIdx.x] = sv[threadIdx.x + w];
            se[threadIdx.x] = se[threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        pv[blockIdx.x] = sv[0];
        pe[blockIdx.x] = se[0];
    }
}

__global__ __launch_bounds__(BLOCK) void k_max_flux_final(int nb, const double* __restrict__ pv,
                                                          const int64_t* __restrict__ pe, double* __restrict__ out_v,
                                                          int64_t* __restrict__ out_e) {
    __shared__ double sv[BLOCK];
    __shared__ int64_t se[BLOCK];
    double bv = -1.0;
    int64_t be = INT64_MAX;
    for (int b = threadIdx.x; b < nb; b += BLOCK)
        if (flux_better(pv[b], pe[b], bv, be)) {
            bv = pv[b];
            be = pe[b];
        }
    sv[threadIdx.x] = bv;
    se[threadIdx.x] = be;
    __syncthreads();
    for (int w = BLOCK / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w && flux_better(sv[threadIdx.x + w], se[threadIdx.x + w], sv[threadIdx.x], se[threadIdx.x])) {
            sv[threadIdx.x] = sv[threadIdx.x + w];
            se[threadIdx.x] = se[threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        out_v[0] = sv[0];
        out_e[0] = se[0] == INT64_MAX ? -1 : se[0];
    }
}

}  // namespace

extern "C" int dec_max_flux_edge(dec_mesh* m, const double* T, const uint8_t* eligible, int64_t* edge_out,
                                 double* density_out) {
    if (!m) return DEC_EINVAL;
    if (!T || !edge_out) return null_argument(m->ctx, "dec_max_flux_edge");
    dec_ctx* ctx = m->ctx;
    try {
        DEC_REQUIRE(!m->dual, DEC_ESTATE, "dec_max_flux_edge is for meshes of vertex unknowns");
        DEC_REQUIRE(m->star_ready && m->geo_ready && m->xyz.p, DEC_ESTATE, "max flux edge needs dec_hodge1 first");
        ctx->set_device();
        const unsigned G = grid_xcd(m->E);
        DBuf<double> pv, ov;
        DBuf<int64_t> pe, oe;
        pv.alloc(ctx, G);
        pe.alloc(ctx, G);
        ov.alloc(ctx, 1);
        oe.alloc(ctx, 1);
        hipLaunchKernelGGL(k_max_flux_partial, dim3(G), dim3(BLOCK), 0, ctx->stream, m->E, m->edges.p, m->xyz.p,
                           m->geo.p, m->star1.p, T, eligible, pv.p, pe.p);
        hipLaunchKernelGGL(k_max_flux_final, dim3(1), dim3(BLOCK), 0, ctx->stream, (int)G, pv.p, pe.p, ov.p, oe.p);
        HIP_CHECK(hipGetLastError());
        int64_t e = 0;
        std::memcpy(&e, ctx->readback(oe.p, sizeof(int64_t)), sizeof(int64_t));
        double v = 0.0;
        std::memcpy(&v, ctx->readback(ov.p, sizeof(double)), sizeof(double));
        *edge_out = e;
        if (density_out) *density_out = e >= 0 ? v : NAN;
    } catch (const DecError& e) {
        ctx->last_error = e.msg;
        return e.code;
    }
    return DEC_OK;
}

extern "C" int dec_flux_effective_conductivity(dec_mesh* m, const double* T, const int8_t* side, double length,
                                               double area, double dT, double* k_eff, double* q_in, double* q_out,
                                               double* energy, double* edge_flux_out) {
    if (!m) return DEC_EINVAL;
    if (!T) return null_argument(m->ctx, "dec_flux_effective_conductivity");
    dec_ctx* ctx = m->ctx;
    try {
        DEC_REQUIRE(!m->dual, DEC_ESTATE, "dec_flux_effective_conductivity is for meshes of vertex unknowns");
        DEC_REQUIRE(m->star_ready, DEC_ESTATE, "flux needs dec_hodge1 first");
        DEC_REQUIRE(area > 0.0 && length > 0.0 && dT != 0.0, DEC_EINVAL, "bad length/area/dT");
        ctx->set_device();
        int64_t G = 8 * (int64_t)ctx->num_cus;
        const int64_t want = ((m->V + BLOCK - 1) / BLOCK + 7) / 8 * 8;
        if (want < G) G = want;
        DBuf<double> part, out;
        part.alloc(ctx, FLUX_SUMS * G);
        out.alloc(ctx, FLUX_SUMS);
        DBuf<unsigned> counter;
        counter.alloc(ctx, 1);
        counter.zero();
        hipLaunchKernelGGL(k_flux, dim3(G), dim3(BLOCK), 0, ctx->stream, m->V, m->E, m->row_ptr.p, m->col.p,
                           m->nz_edge.p, m->edges.p, m->star1.p, T, side, edge_flux_out, part.p, out.p, counter.p);
        HIP_CHECK(hipGetLastError());
        double h[FLUX_SUMS];
        std::memcpy(h, ctx->readback(out.p, sizeof(h)), sizeof(h));
        if (q_in) *q_in = h[0];
        if (q_out) *q_out = h[1];
        if (energy) *energy = h[2];
        if (k_eff) {
            if (!m->neumann)
                *k_eff = h[2] * length / (area * dT * dT);
            else  // the flux density through a Dirichlet side given in `side`
                *k_eff = (h[3] > 0 ? h[0] : h[4] > 0 ? h[1] : NAN) * length / (area * dT);
        }
    } catch (const DecError& e) {
        ctx->last_error = e.msg;
        return e.code;
    }
    return DEC_OK;
}
