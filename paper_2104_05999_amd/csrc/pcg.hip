// Preconditioned conjugate gradients on the DEC system, FP64 and FP32, and
// FP64 iterative refinement around FP32 inner solves.
//
// The paper solves its system with PETSc (Section 2.3); the vertex system
// A T = b here is symmetric positive definite, so the recurrence is the
// textbook PCG (Hestenes-Stiefel; Saad, Algorithm 9.1):
//     q = A p; alpha = rho / p.q; x += alpha p; r -= alpha q;
//     z = M^-1 r; rho' = r.z; beta = rho'/rho; p = z + beta p.
// One iteration is three fused kernels with Jacobi (SpMV + p.q; updates +
// z + r.z + r.r; p update) or five with FSAI (two more for z = G^T (G r)).
// Every reduction is a fixed-shape block tree followed by a fixed-order sum
// of per-block partials in the block that arrives last, so results do not
// depend on scheduling.  Scalars stay on the device; the host launches
// batches of iterations (optionally a captured hipGraph) and reads the
// state once per batch.
#include <chrono>
#include <cmath>
#include <cstdlib>
#include <mutex>

#include <hip/hip_ext.h>

#include "solver.h"

namespace {

// Rows per thread whose loads the update and closing kernels issue together:
// the first group before the opening fold (so the fold's latency overlaps
// their transfer), every later group before any of its rows is used, so that
// each wavefront keeps ROWS x 3 loads in flight instead of 3.  Measured on the
// box: the update kernel is fastest with groups of 4 while a thread has about
// 8 rows (128^3 on 1024 workgroups: 12.3 against 12.7 us for 4 rows before
// the fold and then one at a time, 13.2 with groups of 8) and with groups of
// 8 when it has about 32 (256^3 on 2048 workgroups: 94.8 against 101.5 us);
// the closing kernel with 6 to 8 at both sizes; issuing the fold's loads
// before the rows' gained nothing.
constexpr int CLOSE_ROWS = 8;
constexpr int64_t VEC_WIDE_ROWS = int64_t(1) << 22;  // from here the vector kernels take 8 blocks per CU
constexpr int UPDATE_ROWS_FEW = 4, UPDATE_ROWS_MANY = 8;
// regions of the partials array, G doubles each
enum { R_PQ = 0, R_RR = 1, R_RZ = 2 };
enum { FIN_NORM2 = 0, FIN_RR = 1, FIN_START = 2 };

// ---------------------------------------------------------------- SpMV kernels
// k_sell (sliced ELL) is in sell.h.
template <class VT>
__global__ void k_csr_plain(CsrView<VT> A, const VT* __restrict__ x, VT* __restrict__ y) {
    GRID_STRIDE_LOOP(row, A.V) y[row] = csr_row(A, row, x);
}

// ---------------------------------------------------------------- start-up kernels
__global__ void k_norm2(int64_t V, const double* __restrict__ b, double* __restrict__ partials) {
    __shared__ double lds[BLOCK / 64 + 1];
    int64_t i0, i1;
    block_range(V, &i0, &i1);
    double s = 0.0;
    for (int64_t i = i0 + threadIdx.x; i < i1; i += BLOCK) s += b[i] * b[i];
    const double bs = block_sum(s, lds);
    if (threadIdx.x == 0) partials[blockIdx.x] = bs;
}

// partials of x.(b + r): the A-norm squared of x when r = b - A x
__global__ void k_xbr(int64_t V, const double* __restrict__ x, const double* __restrict__ b,
                      const double* __restrict__ r, double* __restrict__ partials) {
    __shared__ double lds[BLOCK / 64 + 1];
    int64_t i0, i1;
    block_range(V, &i0, &i1);
    double s = 0.0;
    for (int64_t i = i0 + threadIdx.x; i < i1; i += BLOCK) s += x[i] * (b[i] + r[i]);
    const double bs = block_sum(s, lds);
    if (threadIdx.x == 0) partials[blockIdx.x] = bs;
}

// energy-norm state: cum = sum of the partials, window cleared, rr_stop = tol^2
__global__ void k_energy_start(const double* __restrict__ partials, int n, double tol2, PcgScalars* __restrict__ st) {
    __shared__ double lds[BLOCK / 64 + 1];
    const double s = reduce_bcast(partials, n, lds);
    if (threadIdx.x == 0) {
        st->cum = s;
        st->rr_stop = tol2;
        for (int j = 0; j < ENERGY_DELAY; ++j) st->hist[j] = 0.0;
    }
}

__global__ void k_reset(PcgScalars* st, int64_t max_iter, int32_t use_energy) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        st->iter = 0;
        st->max_iter = max_iter;
        st->use_energy = use_energy;
        st->done = PCG_RUNNING;
        st->rho = st->pq = st->alpha = st->beta = 0.0;
    }
}

// One block: fold the partials of the previous kernel(s) into the state.
//   FIN_NORM2: aux = sum(R_RR), rr_stop = factor * aux
//   FIN_RR:    rr = aux = sum(R_RR)
//   FIN_START: rr = sum(R_RR), rho = sum(R_RZ), iteration 0; rr_stop =
//              factor * rr when `relative`, else kept; done when rr <= rr_stop
//              (energy-norm state: done only when rho is 0, x is the solution)
__global__ void k_finalize(const double* __restrict__ partials, int P, int n_rr, int n_rz, int what, double factor,
                           int relative, PcgScalars* __restrict__ st) {
    __shared__ double lds[BLOCK / 64 + 1];
    const double rr = reduce_bcast(partials + R_RR * P, n_rr, lds);
    const double rz = what == FIN_START ? reduce_bcast(partials + R_RZ * P, n_rz, lds) : 0.0;
    if (threadIdx.x != 0) return;
    if (what == FIN_NORM2) {
        st->aux = rr;
        st->rr_stop = factor * rr;
    } else if (what == FIN_RR) {
        st->rr = rr;
        st->aux = rr;
    } else {
        st->rr = rr;
        st->rho = rz;
        if (relative) st->rr_stop = factor * rr;
        st->iter = 0;
        const bool conv = st->use_energy ? rz == 0.0 : rr <= st->rr_stop;
        st->done = conv ? PCG_CONVERGED : (isfinite(rz) ? PCG_RUNNING : PCG_BREAKDOWN);
    }
}

// x0: Dirichlet values on Dirichlet rows, 0 on pinned rows, the warm start
// (or 0) elsewhere
__global__ void k_init_x(int64_t V, const uint8_t* __restrict__ fixed, const double* __restrict__ dval,
                         const double* __restrict__ warm, double* __restrict__ x) {
    GRID_STRIDE_LOOP(i, V) {
        const uint8_t f = fixed[i];
        x[i] = f == 1 ? dval[i] : (f == 2 ? 0.0 : (warm ? warm[i] : 0.0));
    }
}

// Jacobi start: z = D^-1 r, p = z, partials of r.z
template <class VT>
__global__ void k_init_jacobi(int64_t V, const VT* __restrict__ r, const VT* __restrict__ invd, VT* __restrict__ p,
                              double* __restrict__ partials) {
    __shared__ double lds[BLOCK / 64 + 1];
    int64_t i0, i1;
    block_range(V, &i0, &i1);
    VT rz = 0;
    for (int64_t i = i0 + threadIdx.x; i < i1; i += BLOCK) {
        const VT ri = r[i];
        const VT z = invd[i] * ri;
        p[i] = z;
        rz += ri * z;
    }
    const double bs = block_sum(static_cast<double>(rz), lds);
    if (threadIdx.x == 0) partials[blockIdx.x] = bs;
}

// Split-Jacobi start (CG on D^-1/2 A D^-1/2): p = r^, partials of r^.r^ (= r.D^-1 r)
// and of r^.D r^ (= r.r, for the stopping test on the residual of A); dg = diag(A).
template <class VT>
__global__ void k_init_split(int64_t V, const VT* __restrict__ r, const VT* __restrict__ dg, VT* __restrict__ p,
                             double* __restrict__ rz_part, double* __restrict__ rr_part) {
    __shared__ double lds[BLOCK / 64 + 1];
    int64_t i0, i1;
    block_range(V, &i0, &i1);
    VT rz = 0, rr = 0;
    for (int64_t i = i0 + threadIdx.x; i < i1; i += BLOCK) {
        const VT ri = r[i];
        p[i] = ri;
        rz += ri * ri;
        rr += (ri * ri) * dg[i];
    }
    const double a = block_sum(static_cast<double>(rz), lds);
    if (threadIdx.x == 0) rz_part[blockIdx.x] = a;
    const double b = block_sum(static_cast<double>(rr), lds);
    if (threadIdx.x == 0) rr_part[blockIdx.x] = b;
}

// Split-Jacobi values: a_ij (s_i s_j) in every stored slot (the product s_i s_j
// is the same for (i, j) and (j, i), so the scaled matrix stays exactly
// symmetric; padding stays 0), s = sqrt(1 / a_ii), s b and a_ii = 1 / invd_i.
// Every diagonal entry is positive (checked with the boundary data).
__global__ void k_jacobi_split(int64_t V, int64_t nslices, const int64_t* __restrict__ sptr,
                               const int32_t* __restrict__ scol, const double* __restrict__ sval,
                               const double* __restrict__ invd, const double* __restrict__ rhs, double* __restrict__ v64,
                               float* __restrict__ v32, double* __restrict__ s64, double* __restrict__ b64,
                               double* __restrict__ d64, float* __restrict__ d32) {
    RANGE_LOOP(i, nslices * SELL_C) {
        const int64_t sl = i / SELL_C;
        const int lane = static_cast<int>(i % SELL_C);
        const int width = static_cast<int>((sptr[sl + 1] - sptr[sl]) / SELL_C);
        const double si = i < V ? sqrt(invd[i]) : 0.0;
        if (i < V) {
            s64[i] = si;
            b64[i] = si * rhs[i];
            d64[i] = 1.0 / invd[i];
            d32[i] = static_cast<float>(1.0 / invd[i]);
        }
        for (int j = 0; j < width; ++j) {
            const int64_t idx = sell_index(sptr[sl], width, j, lane);
            const double v = sval[idx] * (si * sqrt(invd[scol[idx]]));
            v64[idx] = v;
            v32[idx] = static_cast<float>(v);
        }
    }
}

// x *= s (to_hat = 0) or x /= s (to_hat = 1): between x and x^ = D^1/2 x
__global__ void k_split_x(int64_t V, double* __restrict__ x, const double* __restrict__ s, int to_hat) {
    GRID_STRIDE_LOOP(i, V) x[i] = to_hat ? x[i] / s[i] : x[i] * s[i];
}

// ---------------------------------------------------------------- iteration kernels
// Every block folds the p.q partials of the SpMV in the same order, so all
// blocks see the same alpha.  The update kernel moves r only (r -= alpha q);
// the closing kernel moves x (x += alpha p) together with p, so p is read
// once per iteration.  A non-positive p.q leaves x and r untouched; the
// closing kernel reports the breakdown.
// PJ: the preconditioner's part in these kernels.  PJ_NONE: z comes from
// another kernel (FSAI, block Jacobi); PJ_JACOBI: z = D^-1 r (`invd` is
// D^-1); PJ_SPLIT: the system is D^-1/2 A D^-1/2 and z = r (the vectors are
// the hatted ones), with r.r of the unscaled residual taken as sum d_i r_i^2
// (`invd` is then D itself).
enum { PJ_NONE = 0, PJ_JACOBI = 1, PJ_SPLIT = 2 };

// The vector kernels take W consecutive rows per element: FP32 vectors are
// read and written as float2, so each load of a wavefront moves as many bytes
// as in FP64 (one float per lane left the FP32 kernels at two thirds of the
// FP64 kernels' rate).  The last row of an odd V is taken by block 0's first
// thread after its elements.
template <class VT, int W>
struct Rows;
template <class VT>
struct Rows<VT, 1> {
    typedef VT T;
    static __device__ __forceinline__ VT get(const T& v, int) { return v; }
    static __device__ __forceinline__ void set(T& v, int, VT x) { v = x; }
};
template <>
struct Rows<float, 2> {
    typedef float2 T;
    static __device__ __forceinline__ float get(const float2& v, int c) { return c ? v.y : v.x; }
    static __device__ __forceinline__ void set(float2& v, int c, float x) {
        if (c)
            v.y = x;
        else
            v.x = x;
    }
};

template <class VT, int PJ, int ROWS, int W>
__global__ __launch_bounds__(BLOCK) void k_update(int64_t V, VT* __restrict__ r, const VT* __restrict__ q,
                                                  const VT* __restrict__ invd, double* __restrict__ partials,
                                                  int P, int n_pq, PcgScalars* __restrict__ S) {
    typedef Rows<VT, W> RW;
    typedef typename RW::T E;
    __shared__ double lds[BLOCK / 64 + 1];
    if (S->done) return;
    E* re = reinterpret_cast<E*>(r);
    const E* qe = reinterpret_cast<const E*>(q);
    const E* de = reinterpret_cast<const E*>(invd);
    const FrontRange32 R = front_range32(V / W);
    E fr[ROWS], fq[ROWS], fd[ROWS];
#pragma unroll
    for (int k = 0; k < ROWS; ++k) {
        const uint32_t i = R.first + k * R.step;
        if (i < R.end) {
            fr[k] = re[i];
            fq[k] = qe[i];
            fd[k] = PJ != PJ_NONE ? de[i] : E{};
        }
    }
    const double pq = reduce_bcast(partials + R_PQ * P, n_pq, lds);
    if (blockIdx.x == 0 && threadIdx.x == 0) S->pq_now = pq;  // for the closing kernel (no other reader here)
    if (!(pq > 0.0) || !isfinite(pq)) return;
    const VT a = static_cast<VT>(S->rho / pq);
    VT rz = 0, rr = 0;
    auto row = [&](VT fri, VT fqi, VT fdi) {  // r_i - a q_i and its terms of r.z and r.r
        const VT ri = fri - a * fqi;
        if (PJ == PJ_JACOBI) rz += ri * (fdi * ri);
        if (PJ == PJ_SPLIT) rz += ri * ri;
        rr += PJ == PJ_SPLIT ? (ri * ri) * fdi : ri * ri;
        return ri;
    };
    for (uint32_t first = R.first; first < R.end; first += ROWS * R.step) {
        if (first != R.first) {
#pragma unroll
            for (int k = 0; k < ROWS; ++k) {
                const uint32_t i = first + k * R.step;
                if (i < R.end) {
                    fr[k] = re[i];
                    fq[k] = qe[i];
                    fd[k] = PJ != PJ_NONE ? de[i] : E{};
                }
            }
        }
#pragma unroll
        for (int k = 0; k < ROWS; ++k) {
            const uint32_t i = first + k * R.step;
            if (i < R.end) {
                E o;
#pragma unroll
                for (int c = 0; c < W; ++c) RW::set(o, c, row(RW::get(fr[k], c), RW::get(fq[k], c), RW::get(fd[k], c)));
                re[i] = o;
            }
        }
    }
    if (W > 1 && blockIdx.x == 0 && threadIdx.x == 0)
        for (int64_t t = V / W * W; t < V; ++t) r[t] = row(r[t], q[t], PJ != PJ_NONE ? invd[t] : VT(0));
    const double b2 = block_sum(static_cast<double>(rr), lds);
    if (threadIdx.x == 0) partials[R_RR * P + blockIdx.x] = b2;
    if (PJ != PJ_NONE) {
        const double b1 = block_sum(static_cast<double>(rz), lds);
        if (threadIdx.x == 0) partials[R_RZ * P + blockIdx.x] = b1;
    }
}

// Energy-norm test of the iteration being closed (k = S->iter): the window of
// the last ENERGY_DELAY terms alpha_j rho_j, this one included, against
// tol^2 times cum (summed in slot order, as on the host).
__device__ __forceinline__ bool energy_converged(const PcgScalars* S, double pq) {
    const int64_t k = S->iter;
    if (k + 1 < ENERGY_DELAY) return false;
    const double term = S->rho * (S->rho / pq);
    const int slot = static_cast<int>(k % ENERGY_DELAY);
    double win = 0.0;
#pragma unroll 1
    for (int j = 0; j < ENERGY_DELAY; ++j) win += j == slot ? term : S->hist[j];
    return win <= S->rr_stop * (S->cum + term);
}

// Close the iteration: p.q as the update kernel folded it, fold r.r and r.z;
// decide breakdown / convergence / iteration cap; x += alpha p (unless p.q
// broke down), then p = z + beta p while running (z = D^-1 r for Jacobi);
// block 0 writes the next state N.  A finished state is carried forward
// unchanged.
template <class VT, int PJ, int W>
__global__ __launch_bounds__(BLOCK) void k_close(int64_t V, VT* __restrict__ x, const VT* __restrict__ r,
                                                 const VT* __restrict__ invd, const VT* __restrict__ z,
                                                 VT* __restrict__ p, const double* __restrict__ partials, int P,
                                                 int n_rz, const PcgScalars* __restrict__ S,
                                                 PcgScalars* __restrict__ N) {
    typedef Rows<VT, W> RW;
    typedef typename RW::T E;
    __shared__ double lds[2 * (BLOCK / 64 + 1)];
    const bool lead = blockIdx.x == 0 && threadIdx.x == 0;
    if (S->done) {
        if (lead) copy_state(N, S);
        return;
    }
    const int G = gridDim.x;
    E* xe = reinterpret_cast<E*>(x);
    E* pe = reinterpret_cast<E*>(p);
    const E* re = reinterpret_cast<const E*>(r);
    const E* de = reinterpret_cast<const E*>(invd);
    const E* ze = reinterpret_cast<const E*>(z);
    const FrontRange32 R = front_range32(V / W);
    constexpr int ROWS = CLOSE_ROWS;
    // z (or D^-1 r), p and x of the first elements, loaded before the fold
    auto zof = [&](uint32_t i) {
        if (PJ == PJ_SPLIT) return re[i];
        if (PJ == PJ_NONE) return ze[i];
        const E rv = re[i], dv = de[i];
        E o;
#pragma unroll
        for (int c = 0; c < W; ++c) RW::set(o, c, RW::get(dv, c) * RW::get(rv, c));
        return o;
    };
    E fz[ROWS], fp[ROWS], fx[ROWS];
#pragma unroll
    for (int k = 0; k < ROWS; ++k) {
        const uint32_t i = R.first + k * R.step;
        if (i < R.end) {
            fz[k] = zof(i);
            fp[k] = pe[i];
            fx[k] = xe[i];
        }
    }
    const double pq = S->pq_now;
    double rr, rz;
    reduce_bcast2(partials + R_RR * P, G, partials + R_RZ * P, n_rz, lds, &rr, &rz);
    const bool pq_ok = pq > 0.0 && isfinite(pq);
    int done = PCG_RUNNING;
    if (!pq_ok || !isfinite(rr) || !isfinite(rz))
        done = PCG_BREAKDOWN;
    else if (S->use_energy ? energy_converged(S, pq) : rr <= S->rr_stop)
        done = PCG_CONVERGED;
    else if (S->iter + 1 >= S->max_iter)
        done = PCG_MAXITER;
    const double beta = rz / S->rho;
    if (pq_ok) {
        const VT a = static_cast<VT>(S->rho / pq);
        const VT bt = static_cast<VT>(beta);
        const bool run = done == PCG_RUNNING;
        for (uint32_t first = R.first; first < R.end; first += ROWS * R.step) {
            if (first != R.first) {
#pragma unroll
                for (int k = 0; k < ROWS; ++k) {
                    const uint32_t i = first + k * R.step;
                    if (i < R.end) {
                        if (run) fz[k] = zof(i);
                        fp[k] = pe[i];
                        fx[k] = xe[i];
                    }
                }
            }
#pragma unroll
            for (int k = 0; k < ROWS; ++k) {
                const uint32_t i = first + k * R.step;
                if (i < R.end) {
                    E ox, op;
#pragma unroll
                    for (int c = 0; c < W; ++c) {
                        RW::set(ox, c, RW::get(fx[k], c) + a * RW::get(fp[k], c));
                        RW::set(op, c, RW::get(fz[k], c) + bt * RW::get(fp[k], c));
                    }
                    xe[i] = ox;
                    if (run) pe[i] = op;
                }
            }
        }
        if (W > 1 && lead)
            for (int64_t t = V / W * W; t < V; ++t) {
                const VT zt = PJ == PJ_JACOBI ? invd[t] * r[t] : (PJ == PJ_SPLIT ? r[t] : z[t]);
                const VT pt = p[t];
                x[t] = x[t] + a * pt;
                if (run) p[t] = zt + bt * pt;
            }
    }
    if (lead) {
        N->rho = rz;
        N->rr = rr;
        N->rr_stop = S->rr_stop;
        N->aux = S->aux;
        N->alpha = S->rho / pq;
        N->beta = beta;
        N->pq = pq;
        N->iter = S->iter + (done == PCG_BREAKDOWN ? 0 : 1);
        N->max_iter = S->max_iter;
        N->use_energy = S->use_energy;
        N->done = done;
        if (S->use_energy) {
            const double term = S->rho * (S->rho / pq);
            N->cum = S->cum + term;
#pragma unroll 1
            for (int j = 0; j < ENERGY_DELAY; ++j) N->hist[j] = S->hist[j];
            N->hist[S->iter % ENERGY_DELAY] = term;
        }
    }
}

// ---------------------------------------------------------------- refinement kernels
// r32 = r64 / ||r64|| (||r64||^2 in src->rr), x32 = 0, partials of r32.r32;
// with split Jacobi (sc set) r32 = sc * r64 / ||r64||, the hatted residual
__global__ void k_to_f32(int64_t V, const double* __restrict__ r64, const PcgScalars* __restrict__ src,
                         const double* __restrict__ sc, float* __restrict__ r32, float* __restrict__ x32,
                         double* __restrict__ partials) {
    __shared__ double lds[BLOCK / 64 + 1];
    const double inv = 1.0 / sqrt(src->rr);
    int64_t i0, i1;
    block_range(V, &i0, &i1);
    float s = 0.0f;
    for (int64_t i = i0 + threadIdx.x; i < i1; i += BLOCK) {
        const float ri = static_cast<float>(sc ? sc[i] * (r64[i] * inv) : r64[i] * inv);
        r32[i] = ri;
        x32[i] = 0.0f;
        s += ri * ri;
    }
    const double bs = block_sum(static_cast<double>(s), lds);
    if (threadIdx.x == 0) partials[blockIdx.x] = bs;
}

// x64 += scale * x32 (scale = ||r64|| of the refinement step, or its negative to undo it);
// with split Jacobi (sc set) x32 is hatted: x64 += scale * sc * x32
__global__ void k_correct(int64_t V, double* __restrict__ x64, const float* __restrict__ x32, const double* __restrict__ sc,
                          double scale) {
    GRID_STRIDE_LOOP(i, V) {
        const double c = static_cast<double>(x32[i]);
        x64[i] = x64[i] + scale * (sc ? sc[i] * c : c);
    }
}

// ---------------------------------------------------------------- host driver
template <class VT>
struct Run {
    SellView<VT> A;
    SellView<VT> G, GT;  // FSAI factor and its transpose (sliced ELL)
    SellView<VT> M;      // block-Jacobi inverse (tet systems)
    VT *x, *r, *p, *q, *z, *w;
    const VT* invd;  // D^-1 (Jacobi), D (split Jacobi)
    PcgScalars* st;  // two parities
    int precond;
    bool split;          // Jacobi in split form: A is D^-1/2 A D^-1/2, the vectors are hatted
    const double* b;     // right-hand side of the system A is (s b with split Jacobi)
    const double* sc;    // split Jacobi: s = D^-1/2 (null otherwise)
};

template <class VT>
constexpr int prec_index() {
    return sizeof(VT) == 8 ? 0 : 1;
}

// With events, the launch carries them (hipExtLaunchKernelGGL): the
// timestamps are those of the dispatch itself, not of separate markers.
// Blocks of the iteration's product (MODE_DOT) for precision VT: Gd, else Gs.
template <class VT>
int dot_grid(const SolveCache* c) {
    const int g = c->Gd[prec_index<VT>()];
    return g > 0 ? g : c->Gs;
}

template <class VT, int MODE, int U, bool NT, bool DIFF, int CF, int ORD>
void launch_sell_o(SolveCache* c, const SellView<VT>& A, const VT* x, VT* y, const VT* b, double* part,
                   const int32_t* done, hipEvent_t ev_a, hipEvent_t ev_b) {
    const dim3 g(MODE == MODE_DOT ? dot_grid<VT>(c) : c->Gs), blk(BLOCK);
    if (ev_a)
        hipExtLaunchKernelGGL((k_sell<VT, MODE, U, NT, DIFF, CF, ORD>), g, blk, 0, c->stream, ev_a, ev_b, 0, A, x,
                              y, b, part, done);
    else
        hipLaunchKernelGGL((k_sell<VT, MODE, U, NT, DIFF, CF, ORD>), g, blk, 0, c->stream, A, x, y, b, part, done);
}

// the load order is the tuner's for the iteration's product (MODE_DOT); the
// other modes keep the interleaved order
template <class VT, int MODE, int U, bool NT, bool DIFF, int CF>
void launch_sell_k(SolveCache* c, const SellView<VT>& A, const VT* x, VT* y, const VT* b, double* part,
                   const int32_t* done, hipEvent_t ev_a, hipEvent_t ev_b) {
    if constexpr (MODE == MODE_DOT)
        if (c->order[prec_index<VT>()] == 1)
            return launch_sell_o<VT, MODE, U, NT, DIFF, CF, 1>(c, A, x, y, b, part, done, ev_a, ev_b);
    launch_sell_o<VT, MODE, U, NT, DIFF, CF, 0>(c, A, x, y, b, part, done, ev_a, ev_b);
}

template <class VT, int MODE, int U, bool NT, bool DIFF>
void launch_sell_d(SolveCache* c, const SellView<VT>& A, const VT* x, VT* y, const VT* b, double* part,
                   const int32_t* done, hipEvent_t ev_a, hipEvent_t ev_b) {
    if (A.tcol)
        launch_sell_k<VT, MODE, U, NT, DIFF, CF_U8>(c, A, x, y, b, part, done, ev_a, ev_b);
    else if (A.dcol)
        launch_sell_k<VT, MODE, U, NT, DIFF, CF_I16>(c, A, x, y, b, part, done, ev_a, ev_b);
    else
        launch_sell_k<VT, MODE, U, NT, DIFF, CF_I32>(c, A, x, y, b, part, done, ev_a, ev_b);
}

// the column format is the one the view carries (A.tcol, A.dcol, or neither)
template <class VT, int MODE, int U, bool NT>
void launch_sell_u(SolveCache* c, const SellView<VT>& A, const VT* x, VT* y, const VT* b, double* part,
                   const PcgScalars* st, hipEvent_t ev_a, hipEvent_t ev_b) {
    const int32_t* done = st ? &st->done : nullptr;
    if (A.excess)
        launch_sell_d<VT, MODE, U, NT, true>(c, A, x, y, b, part, done, ev_a, ev_b);
    else
        launch_sell_d<VT, MODE, U, NT, false>(c, A, x, y, b, part, done, ev_a, ev_b);
}

template <class VT, int MODE, bool NT>
void launch_sell_nt(SolveCache* c, int unroll, const SellView<VT>& A, const VT* x, VT* y, const VT* b, double* part,
                    const PcgScalars* st, hipEvent_t ev_a, hipEvent_t ev_b) {
    // unroll = pairs of entries in flight per lane
    switch (unroll) {
        case 2:
            launch_sell_u<VT, MODE, 2, NT>(c, A, x, y, b, part, st, ev_a, ev_b);
            break;
        case 3:
            launch_sell_u<VT, MODE, 3, NT>(c, A, x, y, b, part, st, ev_a, ev_b);
            break;
        default:
            launch_sell_u<VT, MODE, 4, NT>(c, A, x, y, b, part, st, ev_a, ev_b);
            break;
    }
}

// SpMV launch on Gs blocks; MODE_DOT / MODE_RESID leave Gs partials in `part`
template <class VT, int MODE>
void launch_sell(SolveCache* c, const SellView<VT>& A, const VT* x, VT* y, const VT* b, double* part,
                 const PcgScalars* st, hipEvent_t ev_a = nullptr, hipEvent_t ev_b = nullptr) {
    const int pi = prec_index<VT>();
    if (c->nt[pi])
        launch_sell_nt<VT, MODE, true>(c, c->unroll[pi], A, x, y, b, part, st, ev_a, ev_b);
    else
        launch_sell_nt<VT, MODE, false>(c, c->unroll[pi], A, x, y, b, part, st, ev_a, ev_b);
}

int stride(const SolveCache* c) { return c->G > c->Gs ? c->G : c->Gs; }
double* region(SolveCache* c, int r) { return c->partials.p + (int64_t)r * stride(c); }

template <class VT>
const VT* values(const SellMatrix& S);
template <>
const double* values<double>(const SellMatrix& S) {
    return S.val64.p;
}
template <>
const float* values<float>(const SellMatrix& S) {
    return S.val32.p;
}
template <class VT>
const VT* excess(const SellMatrix& S);
template <>
const double* excess<double>(const SellMatrix& S) {
    return S.excess64.p;
}
template <>
const float* excess<float>(const SellMatrix& S) {
    return S.excess32.p;
}

// A view of the sliced-ELL matrix S (V rows) whose product reads its columns in
// format `cf`, or in the most compact format S has below it (every matrix has
// its int32 columns); its row excess if any.
template <class VT>
SellView<VT> view_cf(const SellMatrix& S, int64_t V, int cf) {
    SellView<VT> v{S.ptr.p, S.col.p, values<VT>(S), S.nslices, V, excess<VT>(S)};
    v.band_plane = S.band_plane;
    v.band = S.band;
    if (cf >= CF_U8 && S.tcol.p) {
        v.tcol = S.tcol.p;
        v.otab = S.otab.p;
        v.ntab = S.ntab;
    } else if (cf >= CF_I16 && S.dcol.p) {
        v.dcol = S.dcol.p;
    }
    return v;
}

// The solver's view: the column format chosen for this precision.
template <class VT>
SellView<VT> view(const SolveCache* c, const SellMatrix& S, int64_t V) {
    return view_cf<VT>(S, V, c->cf[prec_index<VT>()]);
}

// Bytes one stored column costs the product of a view.
template <class VT>
double column_bytes(const SellView<VT>& v) {
    return v.tcol ? 1.0 : v.dcol ? 2.0 : 4.0;
}

// Pick the sliced-ELL variant by timing the iteration's product (y = A x with
// the partials of x.y) on this matrix: the column format (one-byte table
// indices, 16-bit offsets or int32 columns, as far as S has them), 2, 3 or 4
// entry pairs in flight, non-temporal loads on or off, and the order of a
// row's loads (interleaved, or columns first).  Every variant sums each row
// in the same order over the same columns, so the choice never changes a
// result.
template <class VT>
void autotune_spmv(SolveCache* c, const SellMatrix& S, int64_t V, const VT* x, VT* y) {
    const int pi = prec_index<VT>();
    if (c->tuned[pi]) return;
    std::vector<int> formats;
    if (c->force_cols) {  // that format, or the most compact one S has below it
        const int want = c->force_cols == 8 ? CF_U8 : c->force_cols == 16 ? CF_I16 : CF_I32;
        const double cb = column_bytes(view_cf<VT>(S, V, want));
        formats.push_back(cb == 1.0 ? CF_U8 : cb == 2.0 ? CF_I16 : CF_I32);
    } else {
        for (int cf : {CF_U8, CF_I16, CF_I32})
            if ((cf != CF_U8 || S.tcol.p) && (cf != CF_I16 || S.dcol.p)) formats.push_back(cf);
    }
    std::vector<std::array<int, 4>> cand;  // unroll, non-temporal, column format, load order
    for (int cf : formats) {
        if (c->pinned_variant) {
            cand.push_back({c->unroll[pi], c->nt[pi], cf, c->order[pi]});
            continue;
        }
        for (int u : {4, 3, 2})
            for (int nt : {1, 0})
                for (int ord : {0, 1}) cand.push_back({u, nt, cf, ord});
    }
    const bool free_choice = !c->pinned_variant && c->force_cols == 0;
    const std::array<int64_t, 4> shape{pi + (S.excess64.p ? 2 : 0) + (S.dcol.p ? 4 : 0) + (S.tcol.p ? 8 : 0), V,
                                       S.nslices, S.entries};
    auto pick_as = [&](const std::array<int, 4>& v) {
        c->unroll[pi] = v[0];
        c->nt[pi] = v[1];
        c->cf[pi] = v[2];
        c->order[pi] = v[3];
        c->tuned[pi] = true;
    };
    if (cand.size() == 1) return pick_as(cand[0]);
    if (free_choice) {
        auto known = c->ctx->spmv_tune.find(shape);
        if (known != c->ctx->spmv_tune.end()) return pick_as(known->second);  // timed before on this context
    }
    // three rounds over the variants, each timing three launches; a variant's
    // figure is its best round, so that one slow round (clock or
    // neighbouring-work noise) does not decide the pick
    const int nc = (int)cand.size();
    std::vector<float> best(nc, 1e30f);
    for (int round = 0; round < 3; ++round) {
        for (int k = 0; k < nc; ++k) {
            c->unroll[pi] = cand[k][0];
            c->nt[pi] = cand[k][1];
            c->order[pi] = cand[k][3];
            const SellView<VT> A = view_cf<VT>(S, V, cand[k][2]);
            // the iteration's own mode (y = A x with the partials of x.y)
            launch_sell<VT, MODE_DOT>(c, A, x, y, nullptr, region(c, R_PQ), nullptr);
            HIP_CHECK(hipEventRecord(c->t0, c->stream));
            for (int r = 0; r < 3; ++r) launch_sell<VT, MODE_DOT>(c, A, x, y, nullptr, region(c, R_PQ), nullptr);
            HIP_CHECK(hipEventRecord(c->t1, c->stream));
            HIP_CHECK(hipEventSynchronize(c->t1));
            float ms = 0.0f;
            HIP_CHECK(hipEventElapsedTime(&ms, c->t0, c->t1));
            if (ms < best[k]) best[k] = ms;
        }
    }
    int pick = 0;
    for (int k = 1; k < nc; ++k)
        if (best[k] < best[pick]) pick = k;
    pick_as(cand[pick]);
    if (free_choice) c->ctx->spmv_tune[shape] = cand[pick];
}


// n_rr: blocks of the kernel that left the r.r partials; r.z partials always come from a G-block kernel
void finalize(SolveCache* c, int what, int n_rr, double factor, int relative, PcgScalars* st, int n_rz = 0) {
    hipLaunchKernelGGL(k_finalize, dim3(1), dim3(BLOCK), 0, c->stream, c->partials.p, stride(c), n_rr,
                       n_rz ? n_rz : c->G, what, factor, relative, st);
}

// blocks that leave the r.z partials: the Jacobi kernels run on G blocks, the
// FSAI product G^T w and the block-Jacobi product on the SpMV's Gs blocks
int rz_parts(const SolveCache* c, int precond) { return precond == DEC_PRECOND_JACOBI ? c->G : c->Gs; }

// The update kernel on G blocks, its row groups sized by the rows each thread has.
// Rows per element of the vector kernels: 2 for FP32 vectors that all sit on
// 8-byte boundaries (every buffer this library allocates does), else 1.
template <class VT>
int vec_lanes(std::initializer_list<const void*> ptrs) {
    uintptr_t o = 0;
    for (const void* q : ptrs) o |= reinterpret_cast<uintptr_t>(q);
    return (o & 7) == 0 ? 2 : 1;
}

// The update kernel on G blocks, its element groups sized by the elements each thread has.
template <class VT, int PJ, int W>
void launch_update_w(hipStream_t s, int G, int64_t V, VT* r, const VT* q, const VT* invd, double* part, int P,
                     int n_pq, PcgScalars* S) {
    const int64_t per_thread = (V / W + (int64_t)G * BLOCK - 1) / ((int64_t)G * BLOCK);
    if (per_thread > 12)
        hipLaunchKernelGGL((k_update<VT, PJ, UPDATE_ROWS_MANY, W>), dim3(G), dim3(BLOCK), 0, s, V, r, q, invd, part,
                           P, n_pq, S);
    else
        hipLaunchKernelGGL((k_update<VT, PJ, UPDATE_ROWS_FEW, W>), dim3(G), dim3(BLOCK), 0, s, V, r, q, invd, part,
                           P, n_pq, S);
}

// pairs = false keeps one row per element (DEC_VEC_PAIRS=0, for tests)
template <class VT, int PJ>
void launch_update(hipStream_t s, int G, int64_t V, VT* r, const VT* q, const VT* invd, double* part, int P, int n_pq,
                   PcgScalars* S, bool pairs = true) {
    if constexpr (sizeof(VT) == 4)
        if (pairs && vec_lanes<VT>({r, q, invd}) == 2)
            return launch_update_w<VT, PJ, 2>(s, G, V, r, q, invd, part, P, n_pq, S);
    launch_update_w<VT, PJ, 1>(s, G, V, r, q, invd, part, P, n_pq, S);
}

template <class VT, int PJ>
void launch_close(hipStream_t s, int G, int64_t V, VT* x, const VT* r, const VT* invd, const VT* z, VT* p,
                  const double* part, int P, int n_rz, const PcgScalars* S, PcgScalars* N, bool pairs = true) {
    if constexpr (sizeof(VT) == 4)
        if (pairs && vec_lanes<VT>({x, r, invd, z, p}) == 2) {
            hipLaunchKernelGGL((k_close<VT, PJ, 2>), dim3(G), dim3(BLOCK), 0, s, V, x, r, invd, z, p, part, P, n_rz,
                               S, N);
            return;
        }
    hipLaunchKernelGGL((k_close<VT, PJ, 1>), dim3(G), dim3(BLOCK), 0, s, V, x, r, invd, z, p, part, P, n_rz, S, N);
}

template <class VT>
void enqueue_iteration(SolveCache* c, const Run<VT>& R, int par, hipEvent_t ev_a = nullptr,
                       hipEvent_t ev_b = nullptr) {
    const int64_t V = R.A.V;
    const int G = c->G, P = stride(c), n_pq = dot_grid<VT>(c);
    double* part = c->partials.p;
    PcgScalars* S = R.st + par;
    PcgScalars* N = R.st + (par ^ 1);
    launch_sell<VT, MODE_DOT>(c, R.A, R.p, R.q, nullptr, region(c, R_PQ), S, ev_a, ev_b);
    const bool pp = c->vec_pairs;
    if (R.precond == DEC_PRECOND_JACOBI && R.split) {
        launch_update<VT, PJ_SPLIT>(c->stream, G, V, R.r, R.q, R.invd, part, P, n_pq, S, pp);
        launch_close<VT, PJ_SPLIT>(c->stream, G, V, R.x, R.r, nullptr, nullptr, R.p, part, P, G, S, N, pp);
    } else if (R.precond == DEC_PRECOND_JACOBI) {
        launch_update<VT, PJ_JACOBI>(c->stream, G, V, R.r, R.q, R.invd, part, P, n_pq, S, pp);
        launch_close<VT, PJ_JACOBI>(c->stream, G, V, R.x, R.r, R.invd, nullptr, R.p, part, P, G, S, N, pp);
    } else if (R.precond == DEC_PRECOND_BLOCK) {
        launch_update<VT, PJ_NONE>(c->stream, G, V, R.r, R.q, nullptr, part, P, n_pq, S, pp);
        launch_sell<VT, MODE_DOTB>(c, R.M, R.r, R.z, R.r, region(c, R_RZ), S);       // z = M r, r.z partials
        launch_close<VT, PJ_NONE>(c->stream, G, V, R.x, R.r, nullptr, R.z, R.p, part, P, c->Gs, S, N, pp);
    } else {
        launch_update<VT, PJ_NONE>(c->stream, G, V, R.r, R.q, nullptr, part, P, n_pq, S, pp);
        launch_sell<VT, MODE_PLAIN>(c, R.G, R.r, R.w, nullptr, nullptr, S);          // w = G r
        launch_sell<VT, MODE_DOTB>(c, R.GT, R.w, R.z, R.r, region(c, R_RZ), S);      // z = G^T w, r.z partials
        launch_close<VT, PJ_NONE>(c->stream, G, V, R.x, R.r, nullptr, R.z, R.p, part, P, c->Gs, S, N, pp);
    }
    HIP_CHECK(hipGetLastError());
}

// preconditioner start from r (r.r partials already in R_RR): p = M^-1 r, partials of r.z;
// split Jacobi also rewrites the R_RR partials (G blocks) with r.r of the unscaled residual
template <class VT>
void enqueue_precond_start(SolveCache* c, const Run<VT>& R) {
    const int64_t V = R.A.V;
    if (R.precond == DEC_PRECOND_JACOBI && R.split) {
        hipLaunchKernelGGL(k_init_split<VT>, dim3(c->G), dim3(BLOCK), 0, c->stream, V, R.r, R.invd, R.p,
                           region(c, R_RZ), region(c, R_RR));
    } else if (R.precond == DEC_PRECOND_JACOBI) {
        hipLaunchKernelGGL(k_init_jacobi<VT>, dim3(c->G), dim3(BLOCK), 0, c->stream, V, R.r, R.invd, R.p,
                           region(c, R_RZ));
    } else if (R.precond == DEC_PRECOND_BLOCK) {
        launch_sell<VT, MODE_DOTB>(c, R.M, R.r, R.p, R.r, region(c, R_RZ), nullptr);    // p = M r, r.z partials
    } else {
        launch_sell<VT, MODE_PLAIN>(c, R.G, R.r, R.w, nullptr, nullptr, nullptr);       // w = G r
        launch_sell<VT, MODE_DOTB>(c, R.GT, R.w, R.p, R.r, region(c, R_RZ), nullptr);   // p = G^T w, r.z partials
    }
    HIP_CHECK(hipGetLastError());
}

PcgScalars read_state(SolveCache* c, const PcgScalars* st) {
    PcgScalars h;
    HIP_CHECK(hipMemcpyAsync(c->ctx->pinned, st, sizeof(PcgScalars), hipMemcpyDeviceToHost, c->stream));
    HIP_CHECK(hipStreamSynchronize(c->stream));
    std::memcpy(&h, c->ctx->pinned, sizeof(h));
    return h;
}

int even_chunk(const dec_solve_opts& o) {
    int chunk = o.chunk > 0 ? o.chunk : 32;
    return chunk < 2 ? 2 : (chunk + 1) / 2 * 2;
}

// Run batches of iterations (an even number each, so that the current state
// is copy 0 after every batch) until the state says done.
template <class VT>
PcgScalars iterate(SolveCache* c, const Run<VT>& R, const dec_solve_opts& o, dec_solve_stats* stats) {
    const int chunk = even_chunk(o);
    const int prec = sizeof(VT) == 8 ? 0 : 1;
    int64_t last_iter = -1;
    for (int64_t batch = 0;; ++batch) {
        // every batch must advance the iteration count until the state says done
        DEC_REQUIRE(batch <= o.max_iters / chunk + 4, DEC_EHIP, "PCG batches exceed the iteration cap");
        if (o.profile) {
            // SpMV k of the batch carries events when k % every == every - 1: mid-batch launches,
            // queued behind other work like the untimed ones (the first launch of a batch follows
            // the host's read of the state and starts on an idle device)
            const int every = o.profile;
            // timing-only events: no system-scope fence (its cache writeback and invalidation
            // would lengthen the timed launch and slow the work after it); the elapsed times
            // are read after the batch's stream synchronisation
            while ((int)c->events.size() < 2 * chunk) {
                hipEvent_t e;
                HIP_CHECK(hipEventCreateWithFlags(&e, hipEventDisableSystemFence));
                c->events.push_back(e);
            }
            if (batch == 0) last_iter = read_state(c, R.st).iter;
            for (int k = 0; k < chunk; ++k) {
                const bool timed = k % every == every - 1;
                enqueue_iteration(c, R, k & 1, timed ? c->events[2 * k] : nullptr,
                                  timed ? c->events[2 * k + 1] : nullptr);
            }
            const PcgScalars after = read_state(c, R.st);
            const int64_t ran = after.iter - last_iter;  // SpMVs 0 .. ran-1 did work; later ones returned at once
            for (int64_t k = every - 1; k < ran && k < chunk; k += every) {
                float ms = 0.0f;
                HIP_CHECK(hipEventElapsedTime(&ms, c->events[2 * k], c->events[2 * k + 1]));
                if (stats) {
                    stats->spmv_ms += ms;
                    stats->spmv_launches += 1;
                }
            }
            if (after.done) return after;
            DEC_REQUIRE(ran > 0, DEC_EHIP, "PCG made no progress in a batch");
            last_iter = after.iter;
            continue;
        }
        if (o.use_graph) {
            GraphKey key{prec,         R.precond + (R.split ? 8 : 0), chunk, c->unroll[prec], c->nt[prec],
                         c->cf[prec], c->order[prec]};
            auto it = c->graphs.find(key);
            hipGraphExec_t exec = nullptr;
            if (it == c->graphs.end()) {
                hipGraph_t g;
                HIP_CHECK(hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
                for (int k = 0; k < chunk; ++k) enqueue_iteration(c, R, k & 1);
                HIP_CHECK(hipStreamEndCapture(c->stream, &g));
                HIP_CHECK(hipGraphInstantiate(&exec, g, nullptr, nullptr, 0));
                HIP_CHECK(hipGraphDestroy(g));
                c->graphs[key] = exec;
            } else {
                exec = it->second;
            }
            HIP_CHECK(hipGraphLaunch(exec, c->stream));
        } else {
            for (int k = 0; k < chunk; ++k) enqueue_iteration(c, R, k & 1);
        }
        const PcgScalars s = read_state(c, R.st);
        if (s.done) return s;
        DEC_REQUIRE(s.iter > last_iter, DEC_EHIP, "PCG made no progress in a batch");
        last_iter = s.iter;
    }
}


template <class VT>
Run<VT> make_run(dec_mesh* m, SolveCache* c, int precond);

// Rows from which the split form pays: it saves one vector per iteration but
// adds three small kernels per solve, which on systems this small (short,
// launch-bound iterations, often warm-started) cost more than they save.
constexpr int64_t SPLIT_MIN_ROWS = int64_t(1) << 16;

// Split Jacobi for a Jacobi solve of a plain (not difference-form) system
// whose diagonal is positive (checked with the boundary data), from
// SPLIT_MIN_ROWS rows (DEC_JACOBI_SPLIT=1: always, 0: never): builds the
// scaled values once per assembly and boundary data.  Returns whether the
// solve takes it.
bool use_split(dec_mesh* m, SolveCache* c, int precond) {
    if (precond != DEC_PRECOND_JACOBI || m->sell.excess64.p || !m->diag_positive) return false;
    if (c->split == 0 || (c->split < 0 && m->V < SPLIT_MIN_ROWS)) return false;
    JacobiSplit& J = m->jsplit;
    if (J.ready) return true;
    dec_ctx* ctx = m->ctx;
    const SellMatrix& S = m->sell;
    const void* before[4] = {J.v64.p, J.v32.p, J.d64.p, J.d32.p};
    J.v64.alloc(ctx, S.entries);  // kept when large enough, so graphs stay valid
    J.v32.alloc(ctx, S.entries);
    J.s64.alloc(ctx, m->V);
    J.b64.alloc(ctx, m->V);
    J.d64.alloc(ctx, m->V);
    J.d32.alloc(ctx, m->V);
    // on the solve's stream, so the iterations that read the values follow it (its inputs are
    // complete: the solve waited for the caller's stream)
    hipLaunchKernelGGL(k_jacobi_split, dim3(grid_xcd(S.nslices * SELL_C)), dim3(BLOCK), 0, c->stream, m->V,
                       S.nslices, S.ptr.p, S.col.p, S.val64.p, m->invdiag64.p, m->rhs.p, J.v64.p, J.v32.p, J.s64.p,
                       J.b64.p, J.d64.p, J.d32.p);
    HIP_CHECK(hipGetLastError());
    J.ready = true;
    // graphs hold the scaled values' and the diagonal's pointers
    if (before[0] != J.v64.p || before[1] != J.v32.p || before[2] != J.d64.p || before[3] != J.d32.p)
        clear_graphs(c);
    return true;
}

template <>
Run<double> make_run<double>(dec_mesh* m, SolveCache* c, int precond) {
    Run<double> R{};
    R.A = view<double>(c, m->sell, m->V);
    R.split = use_split(m, c, precond);
    R.b = m->rhs.p;
    if (R.split) {
        R.A.val = m->jsplit.v64.p;
        R.b = m->jsplit.b64.p;
        R.sc = m->jsplit.s64.p;
    }
    R.G = view<double>(c, m->fsai.g_sell, m->V);
    R.GT = view<double>(c, m->fsai.gt_sell, m->V);
    R.M = view<double>(c, m->blockinv, m->V);
    R.x = c->x64.p;
    R.r = c->r64.p;
    R.p = c->p64.p;
    R.q = c->q64.p;
    R.z = c->z64.p;
    R.w = c->w64.p;
    R.invd = R.split ? m->jsplit.d64.p : m->invdiag64.p;  // split Jacobi: the diagonal itself
    R.st = c->st.p;
    R.precond = precond;
    return R;
}

template <>
Run<float> make_run<float>(dec_mesh* m, SolveCache* c, int precond) {
    Run<float> R{};
    R.A = view<float>(c, m->sell, m->V);
    R.split = use_split(m, c, precond);
    if (R.split) {
        R.A.val = m->jsplit.v32.p;
        R.sc = m->jsplit.s64.p;
    }
    R.G = view<float>(c, m->fsai.g_sell, m->V);
    R.GT = view<float>(c, m->fsai.gt_sell, m->V);
    R.M = view<float>(c, m->blockinv, m->V);
    R.x = c->x32.p;
    R.r = c->r32.p;
    R.p = c->p32.p;
    R.q = c->q32.p;
    R.z = c->z32.p;
    R.w = c->w32.p;
    R.invd = R.split ? m->jsplit.d32.p : m->invdiag32.p;
    R.st = c->st.p + 2;
    R.precond = precond;
    return R;
}

Run<double> run64(dec_mesh* m, SolveCache* c, int precond) { return make_run<double>(m, c, precond); }
Run<float> run32(dec_mesh* m, SolveCache* c, int precond) { return make_run<float>(m, c, precond); }

SellView<double> sell64(dec_mesh* m, const SolveCache* c) { return view<double>(c, m->sell, m->V); }

// ||b - A x64||^2 in FP64 (through t64), via the scratch state
double true_rr(dec_mesh* m, SolveCache* c) {
    PcgScalars* s4 = c->st.p + 4;
    launch_sell<double, MODE_RESID>(c, sell64(m, c), c->x64.p, c->t64.p, m->rhs.p, region(c, R_RR), nullptr);
    finalize(c, FIN_RR, c->Gs, 0.0, 0, s4);
    HIP_CHECK(hipGetLastError());
    return read_state(c, s4).rr;
}

// The energy-norm estimate of a finished state: sqrt(window / cum).
double energy_estimate(const PcgScalars& s) {
    double win = 0.0;
    for (int j = 0; j < ENERGY_DELAY; ++j) win += s.hist[j];
    return s.cum > 0.0 ? sqrt(win / s.cum) : 0.0;
}

// FP64 PCG from the current x64.  Returns a DEC status.  With the energy
// norm, the state's estimate is the test and no true residual is taken (the
// plain residual of such systems can sit far above tol at full accuracy).
int pcg_fp64(dec_mesh* m, SolveCache* c, const dec_solve_opts& o, double bb, int64_t* iters_out,
             dec_solve_stats* stats) {
    Run<double> R = run64(m, c, o.precond);
    const double tol2 = o.tol * o.tol;
    const bool en = o.norm == DEC_NORM_ENERGY;
    int64_t total = 0;
    // split Jacobi iterates on x^ = D^1/2 x, in x64 between these two calls
    auto hat = [&](int to_hat) {
        if (R.split)
            hipLaunchKernelGGL(k_split_x, dim3(grid_for(m->V)), dim3(BLOCK), 0, c->stream, m->V, R.x, R.sc, to_hat);
    };
    for (int restart = 0;; ++restart) {
        const int64_t left = o.max_iters - total;
        hipLaunchKernelGGL(k_reset, dim3(1), dim3(64), 0, c->stream, R.st, left > 0 ? left : (int64_t)1, (int32_t)en);
        // rr_stop = tol^2 b.b (the relative test in absolute form)
        hipLaunchKernelGGL(k_norm2, dim3(c->G), dim3(BLOCK), 0, c->stream, m->V, m->rhs.p, region(c, R_RR));
        finalize(c, FIN_NORM2, c->G, tol2, 0, R.st);
        hat(1);
        launch_sell<double, MODE_RESID>(c, R.A, R.x, R.r, R.b, region(c, R_RR), nullptr);
        if (en) {
            // ||x0||_A^2 = x0.(b + r0) seeds cum (the same on the split system); rr_stop = tol^2
            hipLaunchKernelGGL(k_xbr, dim3(c->G), dim3(BLOCK), 0, c->stream, m->V, R.x, R.b, R.r, region(c, R_PQ));
            hipLaunchKernelGGL(k_energy_start, dim3(1), dim3(BLOCK), 0, c->stream, region(c, R_PQ), c->G, tol2,
                               R.st);
        }
        enqueue_precond_start<double>(c, R);
        finalize(c, FIN_START, R.split ? c->G : c->Gs, 0.0, 0, R.st, rz_parts(c, R.precond));
        HIP_CHECK(hipGetLastError());
        PcgScalars s = read_state(c, R.st);
        if (!s.done) {
            if (left <= 0) {
                hat(0);
                *iters_out = total;
                return DEC_ENOTCONV;
            }
            s = iterate(c, R, o, stats);
        }
        hat(0);
        total += s.iter;
        *iters_out = total;
        if (s.done == PCG_BREAKDOWN) return DEC_EBREAKDOWN;
        if (s.done == PCG_MAXITER) return DEC_ENOTCONV;
        if (en) {
            if (stats) stats->rel_residual = energy_estimate(s);
            return DEC_OK;
        }
        // converged on the recursive residual: confirm with the true one
        const double rr = true_rr(m, c);
        if (rr <= tol2 * bb) return DEC_OK;
        if (stats) stats->restarts += 1;
        if (restart >= 20) return DEC_ENOTCONV;
    }
}

int ir_mixed(dec_mesh* m, SolveCache* c, const dec_solve_opts& o, double bb, dec_solve_stats* stats) {
    Run<float> R = run32(m, c, o.precond);
    PcgScalars* s4 = c->st.p + 4;
    const double bn = sqrt(bb);
    double rn_prev = INFINITY;
    int64_t inner_total = 0;
    // FP64 PCG from the current x64 with the iterations left
    auto finish_fp64 = [&]() {
        if (stats) stats->fp64_fallback = 1;
        int64_t it64 = 0;
        dec_solve_opts o64 = o;
        o64.max_iters = o.max_iters > inner_total ? o.max_iters - inner_total : 1;
        const int st = pcg_fp64(m, c, o64, bb, &it64, stats);
        if (stats) stats->iterations = inner_total + it64;
        return st;
    };
    // one inner solve gets at most an eighth of the budget, so that a stalled FP32
    // solve leaves FP64 the rest
    const int64_t inner_cap = o.max_iters / 8 > 64 ? o.max_iters / 8 : 64;
    for (int outer = 0; outer < 100; ++outer) {
        // r64 = b - A x64 (FP64), ||r64||^2 into s4->rr
        launch_sell<double, MODE_RESID>(c, sell64(m, c), c->x64.p, c->r64.p, m->rhs.p, region(c, R_RR), nullptr);
        finalize(c, FIN_RR, c->Gs, 0.0, 0, s4);
        const double rn = sqrt(read_state(c, s4).rr);
        if (stats) stats->outer_iterations = outer;
        if (rn <= o.tol * bn) return DEC_OK;
        if (outer > 0 && rn > 0.5 * rn_prev) {
            // refinement stagnates (FP32 cannot reduce the residual further): finish in FP64,
            // from the previous iterate when the last correction made the residual larger
            // (an FP32 solve below its own rounding floor can return nonsense)
            if (rn > rn_prev) {
                hipLaunchKernelGGL(k_correct, dim3(grid_for(m->V)), dim3(BLOCK), 0, c->stream, m->V, c->x64.p,
                                   c->x32.p, R.sc, -rn_prev);
                HIP_CHECK(hipGetLastError());
            }
            return finish_fp64();
        }
        double itol = o.inner_tol;
        if (o.adaptive_final_inner) itol = fmax(o.inner_tol, 0.5 * o.tol * bn / rn);
        if (itol >= 1.0) itol = 0.5;
        const int64_t left = o.max_iters - inner_total;
        if (left <= 0) return DEC_ENOTCONV;
        hipLaunchKernelGGL(k_reset, dim3(1), dim3(64), 0, c->stream, R.st, left < inner_cap ? left : inner_cap, 0);
        hipLaunchKernelGGL(k_to_f32, dim3(c->G), dim3(BLOCK), 0, c->stream, m->V, c->r64.p, s4, R.sc, c->r32.p,
                           c->x32.p, region(c, R_RR));
        enqueue_precond_start<float>(c, R);
        finalize(c, FIN_START, c->G, itol * itol, 1, R.st, rz_parts(c, R.precond));
        HIP_CHECK(hipGetLastError());
        PcgScalars s = read_state(c, R.st);
        if (!s.done) s = iterate(c, R, o, stats);
        inner_total += s.iter;
        if (stats) stats->iterations = inner_total;
        // an FP32 solve that broke down or ran out of iterations is not applied
        if (s.done != PCG_CONVERGED) return finish_fp64();
        hipLaunchKernelGGL(k_correct, dim3(grid_for(m->V)), dim3(BLOCK), 0, c->stream, m->V, c->x64.p, c->x32.p, R.sc,
                           rn);
        HIP_CHECK(hipGetLastError());
        rn_prev = rn;
    }
    return DEC_ENOTCONV;
}

void ensure_vectors(dec_mesh* m, SolveCache* c, int precision) {
    const int64_t V = m->V;
    for (DBuf<double>* b : {&c->x64, &c->r64, &c->p64, &c->q64, &c->z64, &c->w64, &c->t64}) b->alloc(c->ctx, V);
    if (precision == DEC_PREC_MIXED)
        for (DBuf<float>* b : {&c->x32, &c->r32, &c->p32, &c->q32, &c->z32, &c->w32}) b->alloc(c->ctx, V);
}

}  // namespace

// ---------------------------------------------------------------- solve without allocation
// dec_solve_noalloc keeps its vectors, partial sums and scalar state in one
// static device array per GPU (each device holds its own copy of the code
// object's variables), laid out in doubles as
//     [0, NA_STATE)                 PcgScalars: two parity copies and a scratch copy
//     [NA_STATE, NA_HEAD)           partial sums: regions R_PQ, R_RR, R_RZ of NA_PARTS each
//     [NA_HEAD, + 3 DEC_NOALLOC_MAX_ROWS)  r, p, q
// The solution vector is the caller's T.  In host code the array's name is
// only a host-side stand-in: the kernels get the device address that
// hipGetSymbolAddress gave for the device (noalloc_setup, called by
// dec_create with the device current), never `scratch` itself.
namespace {
constexpr int64_t NA_STATE = 128;       // doubles: room for 4 PcgScalars
constexpr int64_t NA_PARTS = 2048;      // partials per region: more than any launch's blocks
constexpr int64_t NA_HEAD = 8192;       // doubles before the vectors (64 KiB)
constexpr int64_t NA_ROWS = DEC_NOALLOC_MAX_ROWS;
constexpr int NA_MAX_DEVICES = 64;
static_assert(4 * sizeof(PcgScalars) <= NA_STATE * sizeof(double), "scalar states fit their region");
static_assert(NA_STATE + 3 * NA_PARTS <= NA_HEAD, "partials fit before the vectors");
}  // namespace

static __device__ __align__(256) double scratch[NA_HEAD + 3 * NA_ROWS];

namespace {
std::mutex na_mutex;                           // set-up of the table below
std::mutex na_solve_mutex[NA_MAX_DEVICES];     // one solve at a time per device in this process
double* na_ptr[NA_MAX_DEVICES] = {};           // device address of `scratch`, per device
std::string na_error[NA_MAX_DEVICES];          // why set-up failed, per device

// x = Dirichlet values on Dirichlet rows, 0 on pinned rows, and on the others
// x itself (warm start) or 0
__global__ void k_init_x_inplace(int64_t V, const uint8_t* __restrict__ fixed, const double* __restrict__ dval,
                                 int warm, double* x) {
    GRID_STRIDE_LOOP(i, V) {
        const uint8_t f = fixed[i];
        x[i] = f == 1 ? dval[i] : (f == 2 ? 0.0 : (warm ? x[i] : 0.0));
    }
}

__global__ void k_zero(int64_t V, double* __restrict__ x) { GRID_STRIDE_LOOP(i, V) x[i] = 0.0; }

// FP64 Jacobi PCG on A (the recurrence and kernels of dec_solve's FP64 path)
// with every buffer beyond m's system and T in the scratch at `base`.
int solve_noalloc(dec_mesh* m, const dec_solve_opts& o, double* T, double* base, dec_solve_stats* stats) {
    dec_ctx* ctx = m->ctx;
    const int64_t V = m->V;
    PcgScalars* st = reinterpret_cast<PcgScalars*>(base);  // [0], [1] parities, [2] scratch
    PcgScalars* s2 = st + 2;
    double* part = base + NA_STATE;
    const int P = static_cast<int>(NA_PARTS);
    double* r = base + NA_HEAD;
    double* p = r + NA_ROWS;
    double* q = p + NA_ROWS;
    // launch settings only: this cache owns no buffer, stream or graph
    SolveCache c;
    c.ctx = ctx;
    c.stream = ctx->stream;
    auto blocks = [&](int64_t rows_per_block, int per_cu) {
        const int64_t want = (V + rows_per_block - 1) / rows_per_block;
        int64_t cap = (int64_t)per_cu * ctx->num_cus;
        if (cap > NA_PARTS) cap = NA_PARTS;
        const int64_t g = want < cap ? want : cap;
        return (int)(((g + 7) / 8) * 8);
    };
    c.G = blocks(BLOCK, V >= VEC_WIDE_ROWS ? 8 : 4);
    c.Gs = blocks(SELL_C * (BLOCK / 64), 8);
    c.Gd[0] = blocks(SELL_C * (BLOCK / 64), m->sell.excess64.p ? 8 : 4);  // as dec_solve's FP64 iteration
    c.Gd[1] = c.Gs;
    const SellMatrix& S = m->sell;
    const std::array<int64_t, 4> shape{0 + (S.excess64.p ? 2 : 0) + (S.dcol.p ? 4 : 0) + (S.tcol.p ? 8 : 0), V,
                                       S.nslices, S.entries};
    auto known = ctx->spmv_tune.find(shape);  // a variant timed earlier for this shape, else the default
    if (known != ctx->spmv_tune.end()) {
        c.unroll[0] = known->second[0];
        c.nt[0] = known->second[1];
        c.cf[0] = known->second[2];
        c.order[0] = known->second[3];
    }
    const SellView<double> A = view<double>(&c, m->sell, V);
    if (stats) {
        stats->spmv_unroll = c.unroll[0];
        stats->spmv_nontemporal = c.nt[0];
        stats->spmv_col_bytes = (int32_t)column_bytes(A);
        stats->spmv_band = (int32_t)S.band;
        stats->spmv_order = c.order[0];
    }
    const int G = c.G, Gs = c.Gs;
    const dim3 blk(BLOCK);
    auto fin = [&](int what, int n_rr, int n_rz, double factor, PcgScalars* s) {
        hipLaunchKernelGGL(k_finalize, dim3(1), blk, 0, c.stream, part, P, n_rr, n_rz, what, factor, 0, s);
    };
    auto state = [&](const PcgScalars* s) {  // the pinned staging area exists from dec_create on
        DEC_REQUIRE(ctx->pinned && ctx->pinned_bytes >= sizeof(PcgScalars), DEC_ESTATE, "no staging area");
        return read_state(&c, s);
    };
    hipLaunchKernelGGL(k_init_x_inplace, dim3(grid_for(V)), blk, 0, c.stream, V, m->fixed.p, m->bc_value.p,
                       (int)o.warm_start, T);
    hipLaunchKernelGGL(k_norm2, dim3(G), blk, 0, c.stream, V, m->rhs.p, part + R_RR * P);
    fin(FIN_NORM2, G, G, 0.0, s2);
    HIP_CHECK(hipGetLastError());
    const double bb = state(s2).aux;
    if (stats) stats->spmv_nnz = m->sell.kept;
    if (bb == 0.0) {
        hipLaunchKernelGGL(k_zero, dim3(grid_for(V)), blk, 0, c.stream, V, T);
        HIP_CHECK(hipGetLastError());
        HIP_CHECK(hipStreamSynchronize(c.stream));
        return DEC_OK;
    }
    const double tol2 = o.tol * o.tol;
    const int chunk = even_chunk(o);
    int64_t total = 0;
    double rr = 0.0;
    int status = DEC_ENOTCONV;
    for (int restart = 0; restart <= 20; ++restart) {
        const int64_t left = o.max_iters - total;
        if (left <= 0) break;
        hipLaunchKernelGGL(k_reset, dim3(1), dim3(64), 0, c.stream, st, left, (int32_t)0);
        hipLaunchKernelGGL(k_norm2, dim3(G), blk, 0, c.stream, V, m->rhs.p, part + R_RR * P);
        fin(FIN_NORM2, G, G, tol2, st);
        launch_sell<double, MODE_RESID>(&c, A, T, r, m->rhs.p, part + R_RR * P, nullptr);
        hipLaunchKernelGGL(k_init_jacobi<double>, dim3(G), blk, 0, c.stream, V, r, m->invdiag64.p, p,
                           part + R_RZ * P);
        fin(FIN_START, Gs, G, 0.0, st);
        HIP_CHECK(hipGetLastError());
        PcgScalars s = state(st);
        for (int64_t batch = 0; !s.done; ++batch) {
            DEC_REQUIRE(batch <= o.max_iters / chunk + 4, DEC_EHIP, "PCG batches exceed the iteration cap");
            const int64_t before = s.iter;
            for (int k = 0; k < chunk; ++k) {
                PcgScalars* S = st + (k & 1);
                PcgScalars* N = st + ((k & 1) ^ 1);
                launch_sell<double, MODE_DOT>(&c, A, p, q, nullptr, part + R_PQ * P, S);
                launch_update<double, PJ_JACOBI>(c.stream, G, V, r, q, m->invdiag64.p, part, P, dot_grid<double>(&c),
                                                 S);
                launch_close<double, PJ_JACOBI>(c.stream, G, V, T, r, m->invdiag64.p, nullptr, p, part, P, G, S, N);
            }
            HIP_CHECK(hipGetLastError());
            s = state(st);
            DEC_REQUIRE(s.done || s.iter > before, DEC_EHIP, "PCG made no progress in a batch");
        }
        total += s.iter;
        if (s.done == PCG_BREAKDOWN) {
            status = DEC_EBREAKDOWN;
            break;
        }
        if (s.done == PCG_MAXITER) break;
        // converged on the recursive residual: confirm with the true one (q is free now)
        launch_sell<double, MODE_RESID>(&c, A, T, q, m->rhs.p, part + R_RR * P, nullptr);
        fin(FIN_RR, Gs, G, 0.0, s2);
        HIP_CHECK(hipGetLastError());
        rr = state(s2).rr;
        if (rr <= tol2 * bb) {
            status = DEC_OK;
            break;
        }
        if (stats) stats->restarts += 1;
    }
    if (status != DEC_OK) {
        launch_sell<double, MODE_RESID>(&c, A, T, q, m->rhs.p, part + R_RR * P, nullptr);
        fin(FIN_RR, Gs, G, 0.0, s2);
        HIP_CHECK(hipGetLastError());
        rr = state(s2).rr;
    }
    if (stats) {
        stats->iterations = total;
        stats->rel_residual = stats->plain_residual = sqrt(rr / bb);
    }
    return status;
}
}  // namespace

void noalloc_setup(int device) {
    std::lock_guard<std::mutex> lock(na_mutex);
    if (device < 0 || device >= NA_MAX_DEVICES || na_ptr[device]) return;
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || p == nullptr) {
        (void)hipGetLastError();
        na_error[device] = std::string("hipGetSymbolAddress(scratch) failed: ") + hipGetErrorString(e);
        return;
    }
    na_ptr[device] = static_cast<double*>(p);
}

void clear_graphs(SolveCache* c) {
    for (auto& kv : c->graphs) (void)hipGraphExecDestroy(kv.second);
    c->graphs.clear();
}

void destroy_solve_cache(SolveCache* c) {
    if (!c) return;
    if (c->stream) (void)hipStreamSynchronize(c->stream);
    clear_graphs(c);
    for (hipEvent_t e : c->events) (void)hipEventDestroy(e);
    if (c->t0) (void)hipEventDestroy(c->t0);
    if (c->t1) (void)hipEventDestroy(c->t1);
    if (c->stream) (void)hipStreamDestroy(c->stream);
    delete c;
}

SolveCache* get_solve_cache(dec_mesh* m) {
    if (m->solve) return m->solve;
    SolveCache* c = new SolveCache();
    c->ctx = m->ctx;
    try {
        HIP_CHECK(hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking));
        HIP_CHECK(hipEventCreate(&c->t0));
        HIP_CHECK(hipEventCreate(&c->t1));
        // one block per 256 rows (64 rows for the SpMV) up to a fixed number of
        // blocks per CU, rounded to a multiple of 8 (one share per XCD): the
        // vector kernels take 8 per CU from 2^22 rows (256^3: 848 against 880 ms
        // per solve), 4 below (128^3: 48.8 against 54.3 ms)
        int per_cu = m->V >= VEC_WIDE_ROWS ? 8 : 4, per_cu_s = 8;
        if (const char* env = getenv("DEC_BLOCKS_PER_CU")) per_cu = atoi(env) > 0 ? atoi(env) : per_cu;
        bool env_cu_s = false;
        if (const char* env = getenv("DEC_SPMV_BLOCKS_PER_CU")) {
            per_cu_s = atoi(env) > 0 ? atoi(env) : per_cu_s;
            env_cu_s = atoi(env) > 0;
        }
        if (const char* env = getenv("DEC_SELL_UNROLL")) {
            c->unroll[0] = c->unroll[1] = atoi(env);
            c->pinned_variant = true;
        }
        if (const char* env = getenv("DEC_SELL_NT")) {
            c->nt[0] = c->nt[1] = atoi(env);
            c->pinned_variant = true;
        }
        if (const char* env = getenv("DEC_SELL_ORDER")) {
            c->order[0] = c->order[1] = atoi(env) == 1 ? 1 : 0;
            c->pinned_variant = true;
        }
        if (const char* env = getenv("DEC_SELL_COLS")) c->force_cols = atoi(env);
        if (const char* env = getenv("DEC_JACOBI_SPLIT")) c->split = atoi(env) != 0;
        if (const char* env = getenv("DEC_VEC_PAIRS")) c->vec_pairs = atoi(env) != 0;
        auto blocks = [&](int64_t rows_per_block, int pc) {
            const int64_t want = (m->V + rows_per_block - 1) / rows_per_block;
            const int64_t cap = (int64_t)pc * m->ctx->num_cus;
            const int64_t g = want < cap ? want : cap;
            return (int)(((g + 7) / 8) * 8);
        };
        c->G = blocks(BLOCK, per_cu);
        c->Gs = blocks(SELL_C * (BLOCK / 64), per_cu_s);
        // the iteration's product: 4 blocks per CU for FP64 on a plain matrix (its
        // faster load orders keep enough loads in flight with fewer waves; 128^3:
        // 25.5 against 26.3 us, 256^3: 275 against 284 us), 8 for FP32 and the
        // difference form (128^3 FP32: 15.4 against 18.3 us, tet system: 160
        // against 177 us).  A rule, not a timing, because the block count sets how
        // the p.q partials group the rows, and so the rounding of the solve.
        const int dot_cu64 = env_cu_s ? per_cu_s : (m->sell.excess64.p ? 8 : 4);
        c->Gd[0] = blocks(SELL_C * (BLOCK / 64), dot_cu64);
        c->Gd[1] = c->Gs;
        c->partials.alloc(m->ctx, 3 * (int64_t)stride(c));
        c->st.alloc(m->ctx, 6);
        HIP_CHECK(hipMemsetAsync(c->st.p, 0, 6 * sizeof(PcgScalars), c->stream));
        (void)m->ctx->readback(c->st.p, 8);  // make sure the pinned staging area exists
    } catch (...) {
        destroy_solve_cache(c);
        throw;
    }
    m->solve = c;
    return c;
}

extern "C" {

int dec_solve_opts_default(dec_solve_opts* o) {
    if (!o) return DEC_EINVAL;
    std::memset(o, 0, sizeof(*o));
    o->precision = DEC_PREC_FP64;
    o->precond = DEC_PRECOND_JACOBI;
    o->tol = 1e-10;
    o->inner_tol = 1e-5;
    o->adaptive_final_inner = 1;
    o->warm_start = 0;
    o->max_iters = 100000;
    o->format = DEC_FMT_AUTO;
    o->chunk = 32;
    o->use_graph = 1;
    o->profile = 0;
    o->norm = DEC_NORM_RESIDUAL;
    return DEC_OK;
}

int dec_solve(dec_mesh* m, const dec_solve_opts* opts, double* T, dec_solve_stats* stats) {
    if (!m) return DEC_EINVAL;
    if (!opts || !T) return null_argument(m->ctx, "dec_solve");
    dec_ctx* ctx = m->ctx;
    try {
        const dec_solve_opts& o = *opts;
        DEC_REQUIRE(m->bc_ready, DEC_ESTATE, "dec_solve needs dec_apply_bc first");
        DEC_REQUIRE(o.precision == DEC_PREC_FP64 || o.precision == DEC_PREC_MIXED, DEC_EINVAL, "bad precision");
        DEC_REQUIRE(o.precond == DEC_PRECOND_JACOBI || o.precond == DEC_PRECOND_FSAI || o.precond == DEC_PRECOND_BLOCK,
                    DEC_EINVAL, "bad precond");
        DEC_REQUIRE(o.precond != DEC_PRECOND_BLOCK || m->blockinv.nslices > 0, DEC_EINVAL,
                    "the block preconditioner is built for tet systems (dec_dual_build)");
        DEC_REQUIRE(o.tol > 0.0 && o.inner_tol > 0.0 && o.inner_tol < 1.0, DEC_EINVAL, "bad tolerance");
        DEC_REQUIRE(o.max_iters > 0 && o.chunk >= 0 && o.chunk <= 4096, DEC_EINVAL, "bad iteration limits");
        DEC_REQUIRE(o.profile >= 0, DEC_EINVAL, "profile is a sampling stride, 0 for off");
        DEC_REQUIRE(o.norm == DEC_NORM_RESIDUAL || o.norm == DEC_NORM_ENERGY, DEC_EINVAL, "bad stopping norm");
        DEC_REQUIRE(o.norm == DEC_NORM_RESIDUAL || o.precision == DEC_PREC_FP64, DEC_EINVAL,
                    "the energy-norm test is for FP64 solves");
        ctx->set_device();
        SolveCache* c = get_solve_cache(m);
        if (o.precond == DEC_PRECOND_FSAI) fsai_setup(m);
        ensure_vectors(m, c, o.precision);
        ctx->sync();  // inputs written on the caller's stream are complete
        autotune_spmv<double>(c, m->sell, m->V, c->p64.p, c->q64.p);
        if (o.precision == DEC_PREC_MIXED) autotune_spmv<float>(c, m->sell, m->V, c->p32.p, c->q32.p);
        if (stats) {
            std::memset(stats, 0, sizeof(*stats));
            const bool mixed = o.precision == DEC_PREC_MIXED;
            const double s = mixed ? 4.0 : 8.0, nz = (double)m->sell.kept;
            // bytes per column of the format the iteration's product reads
            const double cb = mixed ? column_bytes(view<float>(c, m->sell, m->V))
                                    : column_bytes(view<double>(c, m->sell, m->V));
            stats->spmv_nnz = m->sell.kept;
            stats->spmv_bytes = nz * (s + cb) + 4.0 * (double)(m->V + 1) + 2.0 * s * (double)m->V;
            if (m->sell.excess64.p) stats->spmv_bytes += s * (double)m->V;  // difference form: the row excess
            const int pi = mixed ? 1 : 0;
            stats->spmv_unroll = c->unroll[pi];
            stats->spmv_nontemporal = c->nt[pi];
            stats->spmv_col_bytes = (int32_t)cb;
            stats->spmv_band = (int32_t)m->sell.band;
            stats->spmv_order = c->order[pi];
        }
        HIP_CHECK(hipEventRecord(c->t0, c->stream));
        hipLaunchKernelGGL(k_init_x, dim3(grid_for(m->V)), dim3(BLOCK), 0, c->stream, m->V, m->fixed.p,
                           m->bc_value.p, o.warm_start ? T : nullptr, c->x64.p);
        // b.b
        PcgScalars* s4 = c->st.p + 4;
        hipLaunchKernelGGL(k_norm2, dim3(c->G), dim3(BLOCK), 0, c->stream, m->V, m->rhs.p, region(c, R_RR));
        finalize(c, FIN_NORM2, c->G, 0.0, 0, s4);
        HIP_CHECK(hipGetLastError());
        const double bb = read_state(c, s4).aux;
        int status = DEC_OK;
        if (bb == 0.0) {
            HIP_CHECK(hipMemsetAsync(c->x64.p, 0, m->V * sizeof(double), c->stream));
        } else if (o.precision == DEC_PREC_FP64) {
            int64_t it = 0;
            status = pcg_fp64(m, c, o, bb, &it, stats);
            if (stats) stats->iterations = it;
        } else {
            status = ir_mixed(m, c, o, bb, stats);
        }
        HIP_CHECK(hipEventRecord(c->t1, c->stream));
        HIP_CHECK(hipMemcpyAsync(T, c->x64.p, m->V * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
        const double rr = bb == 0.0 ? 0.0 : true_rr(m, c);
        HIP_CHECK(hipStreamSynchronize(c->stream));
        if (stats) {
            float ms = 0.0f;
            HIP_CHECK(hipEventElapsedTime(&ms, c->t0, c->t1));
            stats->solve_ms = ms;
            // the energy-norm test leaves its own estimate (when it converged)
            const bool keep = o.norm == DEC_NORM_ENERGY && status == DEC_OK && bb != 0.0;
            if (!keep) stats->rel_residual = bb == 0.0 ? 0.0 : sqrt(rr / bb);
            stats->plain_residual = bb == 0.0 ? 0.0 : sqrt(rr / bb);
            stats->status = status;
        }
        if (status != DEC_OK) ctx->last_error = dec_status_string(status);
        return status;
    } catch (const DecError& e) {
        ctx->last_error = e.msg;
        return e.code;
    }
}

int dec_solve_noalloc(dec_mesh* m, const dec_solve_opts* opts, double* T, dec_solve_stats* stats) {
    if (!m) return DEC_EINVAL;
    if (!opts || !T) return null_argument(m->ctx, "dec_solve_noalloc");
    dec_ctx* ctx = m->ctx;
    try {
        const dec_solve_opts& o = *opts;
        DEC_REQUIRE(m->V <= DEC_NOALLOC_MAX_ROWS, DEC_EINVAL,
                    "dec_solve_noalloc: " + std::to_string(m->V) + " rows exceed the scratch's maximum of " +
                        std::to_string((long long)DEC_NOALLOC_MAX_ROWS));
        DEC_REQUIRE(m->bc_ready, DEC_ESTATE, "dec_solve_noalloc needs dec_apply_bc first");
        DEC_REQUIRE(o.precision == DEC_PREC_FP64 && o.precond == DEC_PRECOND_JACOBI && o.norm == DEC_NORM_RESIDUAL,
                    DEC_EINVAL, "dec_solve_noalloc runs FP64 Jacobi PCG with the residual test only");
        DEC_REQUIRE(o.profile == 0, DEC_EINVAL, "dec_solve_noalloc does not profile");
        DEC_REQUIRE(o.tol > 0.0 && o.max_iters > 0 && o.chunk >= 0 && o.chunk <= 4096, DEC_EINVAL,
                    "bad tolerance or iteration limits");
        DEC_REQUIRE(ctx->device >= 0 && ctx->device < NA_MAX_DEVICES, DEC_EINVAL, "device index beyond the table");
        double* base = nullptr;
        {
            std::lock_guard<std::mutex> lock(na_mutex);
            base = na_ptr[ctx->device];
            DEC_REQUIRE(base != nullptr, DEC_EHIP,
                        na_error[ctx->device].empty() ? "scratch not set up" : na_error[ctx->device]);
        }
        ctx->set_device();
        std::lock_guard<std::mutex> solve_lock(na_solve_mutex[ctx->device]);
        if (stats) {
            std::memset(stats, 0, sizeof(*stats));
            SolveCache probe;  // the format this call reads: a variant timed earlier for the shape, else the default
            const std::array<int64_t, 4> shape{(m->sell.excess64.p ? 2 : 0) + (m->sell.dcol.p ? 4 : 0) +
                                                   (m->sell.tcol.p ? 8 : 0), m->V, m->sell.nslices, m->sell.entries};
            auto known = ctx->spmv_tune.find(shape);
            if (known != ctx->spmv_tune.end()) probe.cf[0] = known->second[2];
            const double cb = column_bytes(view<double>(&probe, m->sell, m->V)), nz = (double)m->sell.kept;
            stats->spmv_bytes = nz * (8.0 + cb) + 4.0 * (double)(m->V + 1) + 16.0 * (double)m->V;
            if (m->sell.excess64.p) stats->spmv_bytes += 8.0 * (double)m->V;
        }
        const auto t0 = std::chrono::steady_clock::now();
        const int status = solve_noalloc(m, o, T, base, stats);
        if (stats) {
            stats->solve_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
            stats->status = status;
        }
        if (status != DEC_OK) ctx->last_error = dec_status_string(status);
        return status;
    } catch (const DecError& e) {
        ctx->last_error = e.msg;
        return e.code;
    }
}

int dec_spmv(dec_mesh* m, int32_t precision, int32_t format, const void* x, void* y) {
    if (!m) return DEC_EINVAL;
    if (!x || !y) return null_argument(m->ctx, "dec_spmv");
    dec_ctx* ctx = m->ctx;
    try {
        DEC_REQUIRE(m->assembled, DEC_ESTATE, "dec_spmv needs dec_assemble first");
        DEC_REQUIRE(precision == DEC_PREC_FP64 || precision == DEC_PREC_MIXED, DEC_EINVAL, "bad precision");
        ctx->set_device();
        SolveCache* c = get_solve_cache(m);
        if (format == DEC_FMT_CSR) {
            if (precision == DEC_PREC_FP64)
                hipLaunchKernelGGL(k_csr_plain<double>, dim3(grid_for(m->V)), dim3(BLOCK), 0, ctx->stream,
                                   CsrView<double>{m->row_ptr.p, m->col.p, m->val64.p, m->V},
                                   static_cast<const double*>(x), static_cast<double*>(y));
            else
                hipLaunchKernelGGL(k_csr_plain<float>, dim3(grid_for(m->V)), dim3(BLOCK), 0, ctx->stream,
                                   CsrView<float>{m->row_ptr.p, m->col.p, m->val32.p, m->V},
                                   static_cast<const float*>(x), static_cast<float*>(y));
        } else {
            hipStream_t keep = c->stream;
            c->stream = ctx->stream;
            if (precision == DEC_PREC_FP64)
                launch_sell<double, MODE_PLAIN>(c, view<double>(c, m->sell, m->V), static_cast<const double*>(x),
                                                static_cast<double*>(y), nullptr, nullptr, nullptr);
            else
                launch_sell<float, MODE_PLAIN>(c, view<float>(c, m->sell, m->V), static_cast<const float*>(x),
                                               static_cast<float*>(y), nullptr, nullptr, nullptr);
            c->stream = keep;
        }
        HIP_CHECK(hipGetLastError());
    } catch (const DecError& e) {
        ctx->last_error = e.msg;
        return e.code;
    }
    return DEC_OK;
}

}  // extern "C"
