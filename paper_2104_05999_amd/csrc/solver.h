// Device building blocks of the PCG solver: the scalar state shared by the
// fused kernels, the CSR view and the host-side solve cache.  The sliced-ELL
// product lives in sell.h.
#pragma once

#include <map>

#include "common.h"
#include "sell.h"

// Scalar state of one PCG run, kept in device memory so that a batch of
// iterations can be launched (or replayed from a graph) without the host.
// Each run owns two copies: iteration k reads copy k&1 and the last kernel
// of the iteration (block 0 only) writes copy (k+1)&1, so no kernel reads a
// field that the same kernel writes.
struct PcgScalars {
    double rho;      // r.z of the current iterate
    double rr;       // r.r of the current iterate
    double rr_stop;  // converged when rr <= rr_stop
    double aux;      // b.b (FP64 solves) or the last reduction result
    double alpha, beta, pq;
    double pq_now;   // p.q of the iteration in progress, folded by the update kernel
    int64_t iter;
    int64_t max_iter;
    int32_t done;    // PCG_RUNNING / PCG_CONVERGED / PCG_MAXITER / PCG_BREAKDOWN
    int32_t use_energy;  // stop on the estimate of the A-norm error instead of r.r
    int32_t pad1[2];
    // Energy-norm stopping test (Hestenes-Stiefel): iteration j adds
    // alpha_j rho_j = ||x* - x_j||_A^2 - ||x* - x_{j+1}||_A^2, so the sum of the
    // last ENERGY_DELAY terms is a lower bound of the A-norm error squared of
    // the iterate ENERGY_DELAY - 1 steps back; `cum` is x0^T (b + r0) plus all
    // terms so far (tending to ||x*||_A^2).  Converged when the window sum is
    // <= rr_stop * cum (rr_stop = tol^2).
    double cum;
    double hist[16];  // the last ENERGY_DELAY terms, term j in slot j % ENERGY_DELAY
};

constexpr int ENERGY_DELAY = 16;
static_assert(sizeof(PcgScalars) % 8 == 0, "PcgScalars is copied in 8-byte words");

// Copy a state word by word: a plain struct copy stages all of its bytes in
// registers at once, which in the closing kernels cost half the resident waves.
__device__ __forceinline__ void copy_state(PcgScalars* __restrict__ dst, const PcgScalars* __restrict__ src) {
    const uint64_t* s = reinterpret_cast<const uint64_t*>(src);
    uint64_t* d = reinterpret_cast<uint64_t*>(dst);
#pragma unroll 1
    for (int w = 0; w < static_cast<int>(sizeof(PcgScalars) / 8); ++w) d[w] = s[w];
}

enum { PCG_RUNNING = 0, PCG_CONVERGED = 1, PCG_MAXITER = 2, PCG_BREAKDOWN = 3 };

template <class VT>
struct CsrView {
    const int32_t* ptr;
    const int32_t* col;
    const VT* val;
    int64_t V;
};

template <class VT>
__device__ __forceinline__ VT csr_row(const CsrView<VT>& A, int64_t row, const VT* __restrict__ x) {
    VT acc = 0;
    for (int32_t k = A.ptr[row]; k < A.ptr[row + 1]; ++k) acc += A.val[k] * x[A.col[k]];
    return acc;
}

// ---------------------------------------------------------------- host side
struct GraphKey {
    int prec, precond, chunk, unroll, nt, cf, order;
    bool operator<(const GraphKey& o) const {
        if (prec != o.prec) return prec < o.prec;
        if (precond != o.precond) return precond < o.precond;
        if (chunk != o.chunk) return chunk < o.chunk;
        if (unroll != o.unroll) return unroll < o.unroll;
        if (nt != o.nt) return nt < o.nt;
        if (cf != o.cf) return cf < o.cf;
        return order < o.order;
    }
};

struct SolveCache {
    dec_ctx* ctx = nullptr;
    hipStream_t stream = nullptr;  // internal stream (graph capture needs a non-null stream)
    int G = 0;                     // blocks of the vector kernels (multiple of 8)
    int Gs = 0;                    // blocks of the SpMV kernels (multiple of 8)
    int Gd[2] = {0, 0};            // blocks of the iteration's product (y = A p, p.q partials) per precision, <= Gs
    // sliced-ELL variant per precision ([0] FP64, [1] FP32), chosen by the
    // tuner among variants whose products are bit-for-bit identical
    int unroll[2] = {4, 4};
    int nt[2] = {1, 0};            // non-temporal matrix loads
    int cf[2] = {CF_U8, CF_U8};    // column format, the most compact a matrix has up to this
    int order[2] = {0, 0};         // load order of the iteration's product: 0 interleaved, 1 columns first
    bool tuned[2] = {false, false};
    bool pinned_variant = false;  // unroll / non-temporal loads / load order set through the environment
    int force_cols = 0;           // 32, 16 or 8: this column format where a matrix has it (environment)
    int split = -1;               // Jacobi in split form: 1 always, 0 never, -1 by size (environment)
    bool vec_pairs = true;        // FP32 vector kernels on float2 elements where the vectors allow (environment)
    DBuf<double> x64, r64, p64, q64, z64, w64, t64;
    DBuf<float> x32, r32, p32, q32, z32, w32;
    DBuf<double> partials;  // [3G]: per-block partial sums of p.q, r.r, r.z
    DBuf<PcgScalars> st;    // [6]: FP64 PCG (2 parities), FP32 inner PCG (2), scratch (2)
    std::map<GraphKey, hipGraphExec_t> graphs;
    std::vector<hipEvent_t> events;
    hipEvent_t t0 = nullptr, t1 = nullptr;
};

SolveCache* get_solve_cache(dec_mesh* m);
void clear_graphs(SolveCache* c);
void fsai_setup(dec_mesh* m);
