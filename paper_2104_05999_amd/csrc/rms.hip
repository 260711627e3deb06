// The volume-integrated RMS error of eq. 15 against a linear field
// T_exact(p) = a + g.p (the pristine-cube verification of Section 3.1):
//     RMS = sqrt(sum over unknowns of w_i (T_i - T_exact(p_i))^2).
// Tet unknowns (as in the paper): p_i the tet's circumcentre, w_i its volume.
// Vertex unknowns: p_i the vertex, w_i = sum over its tets of vol / 4, summed
// here tet by tet (each tet adds vol / 4 times its four vertices' squares).
// Deterministic block partials folded in a fixed order.
#include <cmath>
#include <cstring>

#include "geom.h"

namespace {

__global__ __launch_bounds__(BLOCK) void k_rms_partial(int64_t T, const int4* __restrict__ tets,
                                                       const double* __restrict__ xyz, const double* __restrict__ u,
                                                       int on_tets, double a, double gx, double gy, double gz,
                                                       double* __restrict__ partials) {
    __shared__ double lds[BLOCK / 64];
    double acc = 0.0;
    RANGE_LOOP(t, T) {
        const int4 q = tets[t];
        const d3 p0 = load3(xyz + 3 * (int64_t)q.x), p1 = load3(xyz + 3 * (int64_t)q.y);
        const d3 p2 = load3(xyz + 3 * (int64_t)q.z), p3 = load3(xyz + 3 * (int64_t)q.w);
        const double vol = fabs(dot(cross(sub(p1, p0), sub(p2, p0)), sub(p3, p0))) / 6.0;
        if (on_tets) {
            const d3 c = tet_circumcentre(p0, p1, p2, p3);
            const double d = u[t] - (a + ((gx * c.x + gy * c.y) + gz * c.z));
            acc += vol * (d * d);
        } else {
            const d3 p[4] = {p0, p1, p2, p3};
            double s = 0.0;
            for (int k = 0; k < 4; ++k) {
                const double d = u[vget(q, k)] - (a + ((gx * p[k].x + gy * p[k].y) + gz * p[k].z));
                s += d * d;
            }
            acc += 0.25 * vol * s;
        }
    }
    const double b = block_sum(acc, lds);
    if (threadIdx.x == 0) partials[blockIdx.x] = b;
}

__global__ void k_rms_fold(int n, const double* __restrict__ partials, double* __restrict__ out) {
    __shared__ double lds[BLOCK / 64 + 1];
    const double s = reduce_bcast(partials, n, lds);
    if (threadIdx.x == 0) out[0] = s;
}

}  // namespace

extern "C" int dec_rms_error(dec_mesh* m, int32_t on_tets, const double* T, const double* field, double* rms) {
    if (!m) return DEC_EINVAL;
    if (!T || !field || !rms) return null_argument(m->ctx, "dec_rms_error");
    dec_ctx* ctx = m->ctx;
    try {
        DEC_REQUIRE(!m->dual && m->tets.p && m->xyz.p, DEC_ESTATE,
                    "dec_rms_error takes the mesh (vertices and tets) the unknowns live on");
        DEC_REQUIRE(on_tets == 0 || on_tets == 1, DEC_EINVAL, "on_tets is 0 or 1");
        ctx->set_device();
        const unsigned G = grid_xcd(m->T, BLOCK, 1024);
        DBuf<double> part, out;
        part.alloc(ctx, G);
        out.alloc(ctx, 1);
        hipLaunchKernelGGL(k_rms_partial, dim3(G), dim3(BLOCK), 0, ctx->stream, m->T,
                           reinterpret_cast<const int4*>(m->tets.p), m->xyz.p, T, on_tets, field[0], field[1],
                           field[2], field[3], part.p);
        hipLaunchKernelGGL(k_rms_fold, dim3(1), dim3(BLOCK), 0, ctx->stream, (int)G, part.p, out.p);
        HIP_CHECK(hipGetLastError());
        double s;
        std::memcpy(&s, ctx->readback(out.p, sizeof(double)), sizeof(double));
        *rms = std::sqrt(s);
    } catch (const DecError& e) {
        ctx->last_error = e.msg;
        return e.code;
    }
    return DEC_OK;
}
