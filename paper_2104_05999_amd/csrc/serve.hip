// Serving: many uneven systems solved together.
//
// Requests (mesh, conductivity, cracks, boundary data) are admitted while
// the HBM budget allows; their setup (topology, *1, assembly, boundary
// data) runs on a side stream while the batch already on the device keeps
// iterating.  Every admitted system keeps its sliced-ELL matrix and Krylov
// state resident.  One batch step replays a captured graph of `chunk`
// iterations of three batched PCG kernels over a work table of
// (system, 2048-row chunk) items; between replays the host retires
// converged systems, runs the FP64 refinement steps of systems whose inner
// solve ended, admits new systems and rewrites the tables.
//
// Each system's reductions are partitioned by its own chunks only and
// folded in a fixed order, so its iterates do not depend on which other
// systems share the batch: a result is bit-for-bit the same alone and in
// any mix.
#include <hip/hip_ext.h>

#include <chrono>
#include <cmath>
#include <deque>
#include <memory>

#include "solver.h"

void build_topology_device(dec_mesh* m, const double* xyz, const int32_t* tets);
void clone_topology_device(dec_mesh* m, const dec_mesh* src);
void hodge1_device(dec_mesh* m, const double* kappa, int32_t n_cracks, const double* cracks);
void assemble_device(dec_mesh* m);
void apply_bc_internal(dec_mesh* m, const int8_t* bc_type, const double* bc_value, const double* f0);

namespace {

constexpr int CHUNK_ROWS = 2048;
constexpr int CHUNK_SLICES = CHUNK_ROWS / SELL_C;
enum { Q_PQ = 0, Q_RR = 1, Q_RZ = 2, Q_OUT = 3 };  // partial regions, nchunks doubles each

// Device descriptor of one admitted system.
struct BSlot {
    const int64_t* sptr;
    const int32_t* scol;   // int32 columns, null when a more compact format is kept instead
    const int16_t* sdcol;  // 16-bit column offsets, or null
    const uint8_t* stcol;  // one-byte indices into sotab, or null
    const int32_t* sotab;  // [sntab] the column offsets stcol indexes
    int32_t sntab;
    int32_t pad3;
    const double* sval64;
    const float* sval32;
    const double* invd64;
    const float* invd32;
    const double* b;
    const uint8_t* fixed;
    const double* dval;
    const double* x0;      // warm start of the request, or null
    double *x64, *r64, *p64, *q64;
    float *x32, *r32, *p32, *q32;
    double* part;       // [4 * nchunks]
    PcgScalars* st;     // [2] inner state (parity copies)
    PcgScalars* outer;  // rr = ||r64||^2 of the last refinement residual, aux = b.b
    int64_t V, nslices;
    int32_t nchunks;
    int32_t pad;
    double stop_factor;  // inner rr_stop = stop_factor * (relative ? r.r : b.b)
    int32_t relative;
    int32_t pad2;
    int64_t max_iter;    // iterations of the next inner solve
    double undo_scale;   // bk_undo: x64 -= undo_scale * x32
};

struct BItem {
    int32_t slot, chunk;
};

template <class VT>
struct SlotVec;
template <>
struct SlotVec<double> {
    __device__ static const double* val(const BSlot& s) { return s.sval64; }
    __device__ static const double* invd(const BSlot& s) { return s.invd64; }
    __device__ static double* x(const BSlot& s) { return s.x64; }
    __device__ static double* r(const BSlot& s) { return s.r64; }
    __device__ static double* p(const BSlot& s) { return s.p64; }
    __device__ static double* q(const BSlot& s) { return s.q64; }
};
template <>
struct SlotVec<float> {
    __device__ static const float* val(const BSlot& s) { return s.sval32; }
    __device__ static const float* invd(const BSlot& s) { return s.invd32; }
    __device__ static float* x(const BSlot& s) { return s.x32; }
    __device__ static float* r(const BSlot& s) { return s.r32; }
    __device__ static float* p(const BSlot& s) { return s.p32; }
    __device__ static float* q(const BSlot& s) { return s.q32; }
};

// Work items in XCD order: XCD x (blockIdx.x & 7) takes the contiguous x-th
// eighth of the n items, its blocks in turn, so that the neighbouring chunks
// of one system, which gather the same parts of its vectors, share an L2.
// Each item's work and partial sums do not depend on which block takes it.
// gridDim.x must be a multiple of 8.
#define ITEM_LOOP(it, n)                                                          \
    const int it##_step = static_cast<int>(gridDim.x >> 3);                       \
    const int it##_end = static_cast<int>((int64_t)(n) * ((blockIdx.x & 7) + 1) / 8); \
    for (int it = static_cast<int>((int64_t)(n) * (blockIdx.x & 7) / 8) + static_cast<int>(blockIdx.x >> 3); \
         it < it##_end; it += it##_step)

__device__ __forceinline__ void chunk_rows(const BSlot& S, int c, int64_t* r0, int64_t* r1) {
    *r0 = (int64_t)c * CHUNK_ROWS;
    *r1 = *r0 + CHUNK_ROWS < S.V ? *r0 + CHUNK_ROWS : S.V;
}

// ---------------------------------------------------------------- batched inner PCG
// A system's matrix as the product reads it: in the most compact column format
// the system keeps (one-byte table indices, 16-bit offsets, int32 columns).
template <class VT>
__device__ __forceinline__ SellView<VT> slot_view(const BSlot& S, const VT* val) {
    SellView<VT> A{S.sptr, S.scol, val, S.nslices, S.V, nullptr, S.sdcol};
    A.tcol = S.stcol;
    A.otab = S.sotab;
    A.ntab = S.sntab;
    return A;
}

// y = A x over the rows of one work item (the slices [s0, s1)), in column
// format CF; the sum of w[row] * y[row] (w = x for DOT, b for RESID's r.r).
template <class VT, int U, bool NT, int CF, bool RESID, int ORD = 0>
__device__ __forceinline__ VT item_product(const SellView<VT>& A, int64_t s0, int64_t s1, const VT* __restrict__ x,
                                           VT* __restrict__ y, const VT* __restrict__ b, const int32_t* tab) {
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    VT d = 0;
    for (int64_t s = s0 + w; s < s1; s += BLOCK / 64) {
        const int64_t base = A.ptr[s];
        const int width = static_cast<int>((A.ptr[s + 1] - base) / SELL_C);
        const int64_t row = s * SELL_C + lane;
        const int32_t rowc = static_cast<int32_t>(CF == CF_U8 && row >= A.V ? A.V - 1 : row);
        const VT acc = ORD == 1 ? sell_row_cfirst<VT, U, NT, false, CF>(A, base, width, lane, x, VT(0), rowc, tab)
                                : sell_row<VT, U, NT, false, CF>(A, base, width, lane, x, VT(0), rowc, tab);
        if (row < A.V) {
            if (RESID) {
                const VT ri = b[row] - acc;
                y[row] = ri;
                d += ri * ri;
            } else {
                if (NT)  // the non-temporal variant stores y non-temporally too
                    __builtin_nontemporal_store(acc, y + row);
                else
                    y[row] = acc;
                d += x[row] * acc;
            }
        }
    }
    return d;
}

// item_product in the format the system keeps; a one-byte table is first
// staged in LDS (the block's threads all take this item; the barrier of the
// previous item's block sum has ended that item's reads of the table).
template <class VT, int U, bool NT, bool RESID, int ORD = 0>
__device__ __forceinline__ VT item_product_any(const BSlot& S, const SellView<VT>& A, int64_t s0, int64_t s1,
                                               const VT* __restrict__ x, VT* __restrict__ y, const VT* __restrict__ b,
                                               int32_t* tab) {
    if (A.tcol) {
        stage_offsets(A.otab, A.ntab, tab);
        return item_product<VT, U, NT, CF_U8, RESID, ORD>(A, s0, s1, x, y, b, tab);
    }
    if (A.dcol) return item_product<VT, U, NT, CF_I16, RESID, ORD>(A, s0, s1, x, y, b, tab);
    return item_product<VT, U, NT, CF_I32, RESID, ORD>(A, s0, s1, x, y, b, tab);
}

template <class VT, int U, bool NT, int ORD>
__global__ __launch_bounds__(BLOCK) void bk_spmv_dot(const BSlot* __restrict__ slots, const BItem* __restrict__ items,
                                                     const int32_t* __restrict__ n_items, int par) {
    __shared__ double lds[BLOCK / 64 + 1];
    __shared__ int32_t tab[OTAB_MAX];
    const int n = *n_items;
    ITEM_LOOP(it, n) {
        const BItem item = items[it];
        const BSlot& S = slots[item.slot];
        if (S.st[par].done) continue;
        const SellView<VT> A = slot_view<VT>(S, SlotVec<VT>::val(S));
        const int64_t s0 = (int64_t)item.chunk * CHUNK_SLICES;
        const int64_t s1 = s0 + CHUNK_SLICES < S.nslices ? s0 + CHUNK_SLICES : S.nslices;
        const VT d =
            item_product_any<VT, U, NT, false, ORD>(S, A, s0, s1, SlotVec<VT>::p(S), SlotVec<VT>::q(S), nullptr, tab);
        const double bs = block_sum(static_cast<double>(d), lds);
        if (threadIdx.x == 0) S.part[Q_PQ * S.nchunks + item.chunk] = bs;
    }
}

// The update and closing kernels split the vector work as the single-system
// solver does: the update moves r only (r -= alpha q, partials of r.z and
// r.r), the closing kernel moves x together with p (x += alpha p, p = D^-1 r
// + beta p), so p is read once per iteration.  The update's first item
// stores its fold of p.q in the system's scalars, where the closing kernel
// reads it instead of folding the partials again.  A thread takes eight rows
// of the chunk in groups of four: the first group's loads are issued before
// the fold of the system's partials, so the fold's latency overlaps with their
// transfer, and holding one group at a time leaves registers for more
// resident waves.  The rows are taken in the same order either way.
constexpr int ROWS_PER_THREAD = CHUNK_ROWS / BLOCK;
static_assert(ROWS_PER_THREAD * BLOCK == CHUNK_ROWS, "a chunk is a whole number of rows per thread");
constexpr int ROW_GROUP = 4;
static_assert(ROWS_PER_THREAD % ROW_GROUP == 0, "whole groups of rows per thread");

template <class VT>
__global__ __launch_bounds__(BLOCK) void bk_update(const BSlot* __restrict__ slots, const BItem* __restrict__ items,
                                                   const int32_t* __restrict__ n_items, int par) {
    __shared__ double lds[BLOCK / 64 + 1];
    const int n = *n_items;
    ITEM_LOOP(it, n) {
        const BItem item = items[it];
        const BSlot& S = slots[item.slot];
        PcgScalars* st = S.st + par;
        if (st->done) continue;
        VT* r = SlotVec<VT>::r(S);
        const VT *q = SlotVec<VT>::q(S), *invd = SlotVec<VT>::invd(S);
        int64_t r0, r1;
        chunk_rows(S, item.chunk, &r0, &r1);
        VT fr[ROW_GROUP], fq[ROW_GROUP], fd[ROW_GROUP];
        auto load = [&](int g) {
#pragma unroll
            for (int k = 0; k < ROW_GROUP; ++k) {
                const int64_t i = r0 + threadIdx.x + (g * ROW_GROUP + k) * BLOCK;
                if (i < r1) {
                    fr[k] = r[i];
                    fq[k] = q[i];
                    fd[k] = invd[i];
                }
            }
        };
        load(0);
        const double pq = reduce_bcast(S.part + Q_PQ * S.nchunks, S.nchunks, lds);
        if (item.chunk == 0 && threadIdx.x == 0) st->pq_now = pq;
        if (!(pq > 0.0) || !isfinite(pq)) continue;
        const VT a = static_cast<VT>(st->rho / pq);
        VT rz = 0, rr = 0;
        for (int g = 0; g < ROWS_PER_THREAD / ROW_GROUP; ++g) {
            if (g > 0) load(g);
#pragma unroll
            for (int k = 0; k < ROW_GROUP; ++k) {
                const int64_t i = r0 + threadIdx.x + (g * ROW_GROUP + k) * BLOCK;
                if (i < r1) {
                    const VT ri = fr[k] - a * fq[k];
                    r[i] = ri;
                    rz += ri * (fd[k] * ri);
                    rr += ri * ri;
                }
            }
        }
        const double b1 = block_sum(static_cast<double>(rz), lds);
        const double b2 = block_sum(static_cast<double>(rr), lds);
        if (threadIdx.x == 0) {
            S.part[Q_RZ * S.nchunks + item.chunk] = b1;
            S.part[Q_RR * S.nchunks + item.chunk] = b2;
        }
    }
}

template <class VT>
__global__ __launch_bounds__(BLOCK) void bk_close(const BSlot* __restrict__ slots, const BItem* __restrict__ items,
                                                  const int32_t* __restrict__ n_items, int par) {
    __shared__ double lds[2 * (BLOCK / 64 + 1)];
    const int n = *n_items;
    ITEM_LOOP(it, n) {
        const BItem item = items[it];
        const BSlot& S = slots[item.slot];
        const PcgScalars* Sp = S.st + par;
        PcgScalars* N = S.st + (par ^ 1);
        const bool lead = item.chunk == 0 && threadIdx.x == 0;
        if (Sp->done) {
            if (lead) copy_state(N, Sp);
            continue;
        }
        VT *x = SlotVec<VT>::x(S), *p = SlotVec<VT>::p(S);
        const VT *r = SlotVec<VT>::r(S), *invd = SlotVec<VT>::invd(S);
        int64_t r0, r1;
        chunk_rows(S, item.chunk, &r0, &r1);
        VT fz[ROW_GROUP], fp[ROW_GROUP], fx[ROW_GROUP];
        auto load = [&](int g) {
#pragma unroll
            for (int k = 0; k < ROW_GROUP; ++k) {
                const int64_t i = r0 + threadIdx.x + (g * ROW_GROUP + k) * BLOCK;
                if (i < r1) {
                    fz[k] = invd[i] * r[i];
                    fp[k] = p[i];
                    fx[k] = x[i];
                }
            }
        };
        load(0);
        const int nc = S.nchunks;
        const double pq = Sp->pq_now;
        double rr, rz;
        reduce_bcast2(S.part + Q_RR * nc, nc, S.part + Q_RZ * nc, nc, lds, &rr, &rz);
        const bool pq_ok = pq > 0.0 && isfinite(pq);
        int done = PCG_RUNNING;
        if (!pq_ok || !isfinite(rr) || !isfinite(rz))
            done = PCG_BREAKDOWN;
        else if (rr <= Sp->rr_stop)
            done = PCG_CONVERGED;
        else if (Sp->iter + 1 >= Sp->max_iter)
            done = PCG_MAXITER;
        const double beta = rz / Sp->rho;
        if (pq_ok) {
            const VT a = static_cast<VT>(Sp->rho / pq);
            const VT bt = static_cast<VT>(beta);
            const bool run = done == PCG_RUNNING;
            for (int g = 0; g < ROWS_PER_THREAD / ROW_GROUP; ++g) {
                if (g > 0) load(g);
#pragma unroll
                for (int k = 0; k < ROW_GROUP; ++k) {
                    const int64_t i = r0 + threadIdx.x + (g * ROW_GROUP + k) * BLOCK;
                    if (i < r1) {
                        x[i] = fx[k] + a * fp[k];
                        if (run) p[i] = fz[k] + bt * fp[k];
                    }
                }
            }
        }
        if (lead) {
            N->rho = rz;
            N->rr = rr;
            N->rr_stop = Sp->rr_stop;
            N->aux = Sp->aux;
            N->alpha = Sp->rho / pq;
            N->beta = beta;
            N->pq = pq;
            N->iter = Sp->iter + (done == PCG_BREAKDOWN ? 0 : 1);
            N->max_iter = Sp->max_iter;
            N->done = done;
        }
    }
}

// ---------------------------------------------------------------- refinement steps (FP64)
// x0 on admission: Dirichlet values on Dirichlet rows, 0 on pinned rows, the
// request's warm start (or 0) elsewhere; FP32 correction zero
__global__ void bk_admit_init(const BSlot* __restrict__ slots, const BItem* __restrict__ items, int n) {
    __shared__ double lds[BLOCK / 64 + 1];
    ITEM_LOOP(it, n) {
        const BItem item = items[it];
        const BSlot& S = slots[item.slot];
        int64_t r0, r1;
        chunk_rows(S, item.chunk, &r0, &r1);
        double bb = 0.0;
        for (int64_t i = r0 + threadIdx.x; i < r1; i += BLOCK) {
            const uint8_t f = S.fixed[i];
            S.x64[i] = f == 1 ? S.dval[i] : (f == 2 || !S.x0 ? 0.0 : S.x0[i]);
            if (S.x32) S.x32[i] = 0.0f;
            bb += S.b[i] * S.b[i];
        }
        const double t = block_sum(bb, lds);
        if (threadIdx.x == 0) S.part[Q_OUT * S.nchunks + item.chunk] = t;
    }
}

// mixed: x64 += ||r_prev|| x32 (the correction of the inner solve just ended)
__global__ void bk_correct(const BSlot* __restrict__ slots, const BItem* __restrict__ items, int n) {
    ITEM_LOOP(it, n) {
        const BItem item = items[it];
        const BSlot& S = slots[item.slot];
        if (!S.x32) continue;
        const double scale = sqrt(S.outer->rr);
        int64_t r0, r1;
        chunk_rows(S, item.chunk, &r0, &r1);
        for (int64_t i = r0 + threadIdx.x; i < r1; i += BLOCK)
            S.x64[i] = S.x64[i] + scale * static_cast<double>(S.x32[i]);
    }
}

// x64 -= undo_scale * x32: takes back a refinement correction that raised the residual
__global__ void bk_undo(const BSlot* __restrict__ slots, const BItem* __restrict__ items, int n) {
    ITEM_LOOP(it, n) {
        const BItem item = items[it];
        const BSlot& S = slots[item.slot];
        if (!S.x32) continue;
        int64_t r0, r1;
        chunk_rows(S, item.chunk, &r0, &r1);
        for (int64_t i = r0 + threadIdx.x; i < r1; i += BLOCK)
            S.x64[i] = S.x64[i] - S.undo_scale * static_cast<double>(S.x32[i]);
    }
}

// r64 = b - A64 x64, partials of r.r
__global__ __launch_bounds__(BLOCK) void bk_residual(const BSlot* __restrict__ slots, const BItem* __restrict__ items,
                                                     int n) {
    __shared__ double lds[BLOCK / 64 + 1];
    __shared__ int32_t tab[OTAB_MAX];
    ITEM_LOOP(it, n) {
        const BItem item = items[it];
        const BSlot& S = slots[item.slot];
        const SellView<double> A = slot_view<double>(S, S.sval64);
        const int64_t s0 = (int64_t)item.chunk * CHUNK_SLICES;
        const int64_t s1 = s0 + CHUNK_SLICES < S.nslices ? s0 + CHUNK_SLICES : S.nslices;
        const double d = item_product_any<double, 4, true, true>(S, A, s0, s1, S.x64, S.r64, S.b, tab);
        const double bs = block_sum(d, lds);
        if (threadIdx.x == 0) S.part[Q_OUT * S.nchunks + item.chunk] = bs;
    }
}

// one block per listed system: fold the Q_OUT partials into outer->rr (what 0) or outer->aux (what 1)
__global__ void bk_fold_outer(const BSlot* __restrict__ slots, const int32_t* __restrict__ ids, int n, int what) {
    __shared__ double lds[BLOCK / 64 + 1];
    for (int k = blockIdx.x; k < n; k += gridDim.x) {
        const BSlot& S = slots[ids[k]];
        const double t = reduce_bcast(S.part + Q_OUT * S.nchunks, S.nchunks, lds);
        if (threadIdx.x == 0) {
            if (what == 0)
                S.outer->rr = t;
            else {
                S.outer->aux = t;
                S.outer->rr = 0.0;
            }
        }
    }
}

// Start an inner solve from the refinement residual r64.
// mixed: r32 = r64 / ||r64||, x32 = 0, p32 = D^-1 r32.  FP64: p64 = D^-1 r64 (x64 continues).
template <class VT>
__global__ void bk_inner_start(const BSlot* __restrict__ slots, const BItem* __restrict__ items, int n) {
    __shared__ double lds[BLOCK / 64 + 1];
    ITEM_LOOP(it, n) {
        const BItem item = items[it];
        const BSlot& S = slots[item.slot];
        const double inv = 1.0 / sqrt(S.outer->rr);
        VT *r = SlotVec<VT>::r(S), *p = SlotVec<VT>::p(S);
        const VT* invd = SlotVec<VT>::invd(S);
        int64_t r0, r1;
        chunk_rows(S, item.chunk, &r0, &r1);
        VT rr = 0, rz = 0;
        for (int64_t i = r0 + threadIdx.x; i < r1; i += BLOCK) {
            VT ri;
            if (sizeof(VT) == 4) {
                ri = static_cast<VT>(S.r64[i] * inv);
                r[i] = ri;
                S.x32[i] = 0.0f;
            } else {
                ri = r[i];
            }
            const VT z = invd[i] * ri;
            p[i] = z;
            rr += ri * ri;
            rz += ri * z;
        }
        const double b1 = block_sum(static_cast<double>(rr), lds);
        const double b2 = block_sum(static_cast<double>(rz), lds);
        if (threadIdx.x == 0) {
            S.part[Q_RR * S.nchunks + item.chunk] = b1;
            S.part[Q_RZ * S.nchunks + item.chunk] = b2;
        }
    }
}

// one block per listed system: inner state copy 0 from the start partials
__global__ void bk_inner_fold(const BSlot* __restrict__ slots, const int32_t* __restrict__ ids, int n) {
    __shared__ double lds[BLOCK / 64 + 1];
    for (int k = blockIdx.x; k < n; k += gridDim.x) {
        const BSlot& S = slots[ids[k]];
        const double rr = reduce_bcast(S.part + Q_RR * S.nchunks, S.nchunks, lds);
        const double rz = reduce_bcast(S.part + Q_RZ * S.nchunks, S.nchunks, lds);
        if (threadIdx.x == 0) {
            PcgScalars* st = S.st;
            st->rr = rr;
            st->rho = rz;
            st->rr_stop = S.stop_factor * (S.relative ? rr : S.outer->aux);
            st->aux = S.outer->aux;
            st->iter = 0;
            st->max_iter = S.max_iter;
            st->alpha = st->beta = st->pq = 0.0;
            st->done = (rr <= st->rr_stop) ? PCG_CONVERGED : (isfinite(rz) ? PCG_RUNNING : PCG_BREAKDOWN);
        }
    }
}

double now_ms(std::chrono::steady_clock::time_point t0) {
    return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
}

}  // namespace

// ---------------------------------------------------------------- host side
enum SlotPhase { PH_FREE = 0, PH_OUTER = 1, PH_INNER = 2 };

struct ServeReq {
    uint64_t ticket;
    dec_request req;
    double t_submit;
    hipEvent_t inputs;  // recorded on the caller's stream at submit; the setup waits for it
};

struct ServeSlot {
    SlotPhase phase = PH_FREE;
    int mode = DEC_PREC_MIXED;  // DEC_PREC_FP64 or DEC_PREC_MIXED (inner precision)
    uint64_t ticket = 0;
    dec_request req{};
    dec_mesh* mesh = nullptr;
    hipEvent_t inputs = nullptr;  // the request's input event, released with the slot
    int64_t budget_bytes = 0;
    int32_t nchunks = 0;
    DBuf<double> x64, r64, p64, q64, part;
    DBuf<float> x32, r32, p32, q32;
    hipEvent_t ready = nullptr;  // setup finished on the setup stream
    double t_submit = 0, t_admit = 0, t_start = 0;
    double rn_prev = 0;
    int64_t inner_total = 0, outer = 0;
    bool fresh = true;      // no inner solve yet
    bool fallback = false;  // a mixed-precision system that went on in FP64
    bool broke = false;     // its last FP64 inner solve broke down
    int64_t iter_mark = 0;  // inner iterations of the current inner solve already counted in the batch bytes
};

struct dec_server {
    dec_ctx* ctx = nullptr;
    dec_ctx setup_ctx;  // same device and allocator, setup stream
    hipStream_t solve_stream = nullptr, setup_stream = nullptr;
    dec_server_opts opts{};
    size_t budget = 0;
    int64_t committed = 0;
    std::chrono::steady_clock::time_point t0;
    uint64_t next_ticket = 1;
    std::deque<ServeReq> pending;
    std::vector<ServeSlot> slots;
    std::vector<dec_result> done;
    int G = 0;
    // device tables
    DBuf<BSlot> d_slots;
    DBuf<BItem> d_items32, d_items64, d_items_aux;
    DBuf<int32_t> d_n;  // [2]: items in the FP32 and the FP64 inner tables
    DBuf<int32_t> d_ids;
    DBuf<PcgScalars> d_st;  // [3 * max_slots]: 2 inner parity copies + outer
    BSlot* h_slots = nullptr;
    BItem* h_items = nullptr;
    int32_t* h_n = nullptr;
    int32_t* h_ids = nullptr;
    PcgScalars* h_st = nullptr;
    int max_items = 0;
    hipGraphExec_t graph[2] = {nullptr, nullptr};  // [0] FP64 inner, [1] FP32 inner
    hipEvent_t ev_chunk = nullptr;
    // batched SpMV variant per precision ([0] FP64, [1] FP32), tuned on the live batch
    int unroll[2] = {4, 4};
    int nt[2] = {1, 0};
    int order[2] = {0, 0};
    bool tuned[2] = {false, false};
    int tuned_items[2] = {0, 0};  // work items of the batch the variant was timed on
    int tunings[2] = {0, 0};
    hipEvent_t ev_b0 = nullptr, ev_b1 = nullptr;  // around a step's graph replays (timing)
    double batch_ms = 0, batch_bytes = 0;         // replay time and algorithmic bytes of the batched iterations
    int64_t batch_iterations = 0;                 // system-iterations in them
    double host_ms[4] = {0, 0, 0, 0};             // dec_server_step phases: launch, admissions, wait, refinement
    int64_t steps = 0;
};

namespace {

int64_t estimate_bytes(int64_t V, int64_t T) {
    // resident arrays plus the transient peak of the setup (elementary areas, tet-edge map)
    return 300 * V + 220 * T + (int64_t(64) << 20);
}

void free_slot(dec_server* s, ServeSlot& sl) {
    if (sl.mesh) {
        delete sl.mesh;
        sl.mesh = nullptr;
    }
    if (sl.inputs) {
        (void)hipEventDestroy(sl.inputs);
        sl.inputs = nullptr;
    }
    for (DBuf<double>* b : {&sl.x64, &sl.r64, &sl.p64, &sl.q64, &sl.part}) b->release();
    for (DBuf<float>* b : {&sl.x32, &sl.r32, &sl.p32, &sl.q32}) b->release();
    s->committed -= sl.budget_bytes;
    sl.budget_bytes = 0;
    sl.phase = PH_FREE;
}

// drop the setup-only arrays of an admitted mesh
void compact_mesh(dec_mesh* m) {
    m->tets.release();
    m->vt_ptr.release();
    m->vt_list.release();
    m->et_ptr.release();
    m->et_inc.release();
    m->tet_bface.release();
    m->xyz.release();
    m->cut.release();
    m->val64.release();
    m->val32.release();
    m->sell.src.release();
    // the products read the most compact column format the system has
    if (m->sell.tcol.p) m->sell.dcol.release();
    if (m->sell.tcol.p || m->sell.dcol.p) m->sell.col.release();
    m->geo.release();
}

BSlot describe(dec_server* s, int k) {
    ServeSlot& sl = s->slots[k];
    dec_mesh* m = sl.mesh;
    BSlot d{};
    d.sptr = m->sell.ptr.p;
    d.scol = m->sell.col.p;
    d.sdcol = m->sell.dcol.p;
    d.stcol = m->sell.tcol.p;
    d.sotab = m->sell.otab.p;
    d.sntab = m->sell.ntab;
    d.sval64 = m->sell.val64.p;
    d.sval32 = m->sell.val32.p;
    d.invd64 = m->invdiag64.p;
    d.invd32 = m->invdiag32.p;
    d.b = m->rhs.p;
    d.fixed = m->fixed.p;
    d.dval = m->bc_value.p;
    d.x0 = sl.req.T0;
    d.x64 = sl.x64.p;
    d.r64 = sl.r64.p;
    d.p64 = sl.p64.p;
    d.q64 = sl.q64.p;
    // FP32 vectors only while the system refines FP32 corrections (a system that
    // fell back to FP64 must not apply its last FP32 correction again)
    const bool mixed = sl.mode == DEC_PREC_MIXED;
    d.x32 = mixed ? sl.x32.p : nullptr;
    d.r32 = mixed ? sl.r32.p : nullptr;
    d.p32 = mixed ? sl.p32.p : nullptr;
    d.q32 = mixed ? sl.q32.p : nullptr;
    d.part = sl.part.p;
    d.st = s->d_st.p + 3 * k;
    d.outer = s->d_st.p + 3 * k + 2;
    d.V = m->V;
    d.nslices = m->sell.nslices;
    d.nchunks = sl.nchunks;
    d.max_iter = s->opts.max_iters;
    return d;
}

// Setup of one request on the setup stream.  Returns false when it failed (result recorded).
bool admit(dec_server* s, const ServeReq& q, int k) {
    ServeSlot& sl = s->slots[k];
    hipEvent_t ev = sl.ready;  // events are kept across reuse of a slot
    sl = ServeSlot();
    sl.ready = ev;
    sl.ticket = q.ticket;
    sl.req = q.req;
    sl.t_submit = q.t_submit;
    sl.t_admit = now_ms(s->t0);
    sl.mode = s->opts.precision;
    sl.inputs = q.inputs;
    sl.budget_bytes = estimate_bytes(q.req.V, q.req.T);
    s->committed += sl.budget_bytes;
    dec_mesh* m = new dec_mesh();
    m->ctx = &s->setup_ctx;
    m->V = q.req.V;
    m->T = q.req.T;
    sl.mesh = m;
    try {
        // the caller's writes to the request arrays (on its stream, before submit) come first
        HIP_CHECK(hipStreamWaitEvent(s->setup_stream, q.inputs, 0));
        if (q.req.mesh)
            clone_topology_device(m, q.req.mesh);
        else
            build_topology_device(m, q.req.xyz, q.req.tets);
        hodge1_device(m, q.req.kappa, q.req.n_cracks, q.req.cracks);
        assemble_device(m);
        apply_bc_internal(m, q.req.bc_type, q.req.bc_value, q.req.neumann_f0);
        compact_mesh(m);
        const int64_t V = m->V;
        sl.nchunks = (int32_t)((V + CHUNK_ROWS - 1) / CHUNK_ROWS);
        dec_ctx* c = &s->setup_ctx;
        sl.x64.alloc(c, V);
        sl.r64.alloc(c, V);
        sl.part.alloc(c, 4 * (int64_t)sl.nchunks);
        if (sl.mode == DEC_PREC_MIXED) {
            sl.x32.alloc(c, V);
            sl.r32.alloc(c, V);
            sl.p32.alloc(c, V);
            sl.q32.alloc(c, V);
        } else {
            sl.p64.alloc(c, V);
            sl.q64.alloc(c, V);
        }
        if (!sl.ready) HIP_CHECK(hipEventCreateWithFlags(&sl.ready, hipEventDisableTiming));
        HIP_CHECK(hipEventRecord(sl.ready, s->setup_stream));
    } catch (const DecError& e) {
        dec_result r{};
        r.ticket = q.ticket;
        r.user_tag = q.req.user_tag;
        r.status = e.code;
        r.t_submit_ms = q.t_submit;
        r.t_admit_ms = sl.t_admit;
        r.t_finish_ms = now_ms(s->t0);
        s->done.push_back(r);
        s->setup_ctx.last_error = e.msg;
        (void)hipStreamSynchronize(s->setup_stream);  // no setup kernel may still use what free_slot returns
        free_slot(s, sl);
        return false;
    }
    sl.phase = PH_OUTER;
    sl.fresh = true;
    return true;
}

// The item table of the slots in `ids` into dst (room for `cap` items), returning the item
// count; DEC_EBUDGET before anything is written when the table would not fit.
int build_items(dec_server* s, const std::vector<int>& ids, BItem* dst, int64_t cap) {
    int64_t total = 0;
    for (int k : ids) total += s->slots[k].nchunks;
    DEC_REQUIRE(total <= cap, DEC_EBUDGET, "work table full");
    int n = 0;
    for (int k : ids)
        for (int c = 0; c < s->slots[k].nchunks; ++c) dst[n++] = BItem{k, c};
    return n;
}

void upload_slots(dec_server* s) {
    const int ns = (int)s->slots.size();
    for (int k = 0; k < ns; ++k)
        if (s->slots[k].phase != PH_FREE) s->h_slots[k] = describe(s, k);
    HIP_CHECK(hipMemcpyAsync(s->d_slots.p, s->h_slots, ns * sizeof(BSlot), hipMemcpyHostToDevice, s->solve_stream));
}

template <class VT, int ORD>
void launch_batched_spmv_o(dec_server* s, int unroll, int nt, const BItem* items, const int32_t* n_items, int par) {
    const dim3 g(s->G), b(BLOCK);
    const BSlot* sl = s->d_slots.p;
#define BK_SPMV(U, NT) \
    hipLaunchKernelGGL((bk_spmv_dot<VT, U, NT, ORD>), g, b, 0, s->solve_stream, sl, items, n_items, par)
    if (nt) {
        if (unroll == 2) BK_SPMV(2, true);
        else if (unroll == 3) BK_SPMV(3, true);
        else BK_SPMV(4, true);
    } else {
        if (unroll == 2) BK_SPMV(2, false);
        else if (unroll == 3) BK_SPMV(3, false);
        else BK_SPMV(4, false);
    }
#undef BK_SPMV
}

// ord: the order of a row's loads (0 interleaved, 1 columns first)
template <class VT>
void launch_batched_spmv(dec_server* s, int unroll, int nt, int ord, const BItem* items, const int32_t* n_items,
                         int par) {
    if (ord == 1)
        launch_batched_spmv_o<VT, 1>(s, unroll, nt, items, n_items, par);
    else
        launch_batched_spmv_o<VT, 0>(s, unroll, nt, items, n_items, par);
}

template <class VT>
void enqueue_batched_iteration(dec_server* s, const BItem* items, const int32_t* n_items, int par) {
    const dim3 g(s->G), b(BLOCK);
    const int pi = sizeof(VT) == 8 ? 0 : 1;
    launch_batched_spmv<VT>(s, s->unroll[pi], s->nt[pi], s->order[pi], items, n_items, par);
    hipLaunchKernelGGL(bk_update<VT>, g, b, 0, s->solve_stream, s->d_slots.p, items, n_items, par);
    hipLaunchKernelGGL(bk_close<VT>, g, b, 0, s->solve_stream, s->d_slots.p, items, n_items, par);
}

// Pick the batched SpMV variant (2, 3 or 4 entry pairs in flight, non-temporal
// loads on or off, a row's loads interleaved or columns first) for a
// precision by timing it on the batch about to run:
// three rounds of two launches per variant, each variant's best round.  The
// extra launches recompute q = A p and the p.q partials of the same p, which
// the batch's first iteration computes again, and every variant sums each row
// in the same order, so the choice changes no result.  The first batch of a
// stream may hold a few small systems, so the variant is timed again each
// time the batch has doubled since (at most MAX_TUNINGS times per precision).
constexpr int MAX_TUNINGS = 5;

template <class VT>
void tune_batched_spmv(dec_server* s, const BItem* items, const int32_t* n_items) {
    const int pi = sizeof(VT) == 8 ? 0 : 1;
    constexpr int NC = 12;
    int cand[NC][3];
    for (int k = 0; k < NC; ++k) {
        cand[k][0] = 4 - k / 4;     // pairs in flight
        cand[k][1] = 1 - k / 2 % 2;  // non-temporal loads
        cand[k][2] = k % 2;          // load order
    }
    float best[NC];
    for (int k = 0; k < NC; ++k) best[k] = 1e30f;
    for (int round = 0; round < 3; ++round)
        for (int k = 0; k < NC; ++k) {
            launch_batched_spmv<VT>(s, cand[k][0], cand[k][1], cand[k][2], items, n_items, 0);
            HIP_CHECK(hipEventRecord(s->ev_b0, s->solve_stream));
            for (int r = 0; r < 2; ++r)
                launch_batched_spmv<VT>(s, cand[k][0], cand[k][1], cand[k][2], items, n_items, 0);
            HIP_CHECK(hipEventRecord(s->ev_b1, s->solve_stream));
            HIP_CHECK(hipEventSynchronize(s->ev_b1));
            float ms = 0.0f;
            HIP_CHECK(hipEventElapsedTime(&ms, s->ev_b0, s->ev_b1));
            if (ms < best[k]) best[k] = ms;
        }
    int pick = 0;
    for (int k = 1; k < NC; ++k)
        if (best[k] < best[pick]) pick = k;
    s->unroll[pi] = cand[pick][0];
    s->nt[pi] = cand[pick][1];
    s->order[pi] = cand[pick][2];
    s->tuned[pi] = true;
}

// Algorithmic bytes of one batched iteration of a system: the product
// (kept entries x (value + column) + row pointer + x and y, the CSR
// definition over the entries it uses) and the vector kernels (update: r, q,
// D^-1 read, r written; close: D^-1, r, p, x read, x and p written).
double batched_iteration_bytes(const dec_mesh* m, int mode) {
    const double sv = mode == DEC_PREC_MIXED ? 4.0 : 8.0;
    const double cb = m->sell.tcol.p ? 1.0 : m->sell.dcol.p ? 2.0 : 4.0;
    const double V = (double)m->V;
    return (double)m->sell.kept * (sv + cb) + 4.0 * (V + 1) + 2.0 * sv * V + 4.0 * sv * V + 6.0 * sv * V;
}

hipGraphExec_t batched_graph(dec_server* s, int prec) {
    if (s->graph[prec]) return s->graph[prec];
    // prec: 0 FP64 (graph and tuning index 0), 1 FP32 (index 1)
    if (!s->tuned[prec]) {
        if (prec == 1)
            tune_batched_spmv<float>(s, s->d_items32.p, s->d_n.p);
        else
            tune_batched_spmv<double>(s, s->d_items64.p, s->d_n.p + 1);
    }
    const int chunk = s->opts.chunk;
    hipGraph_t g;
    HIP_CHECK(hipStreamBeginCapture(s->solve_stream, hipStreamCaptureModeThreadLocal));
    for (int k = 0; k < chunk; ++k) {
        if (prec == 1)
            enqueue_batched_iteration<float>(s, s->d_items32.p, s->d_n.p, k & 1);
        else
            enqueue_batched_iteration<double>(s, s->d_items64.p, s->d_n.p + 1, k & 1);
    }
    HIP_CHECK(hipStreamEndCapture(s->solve_stream, &g));
    HIP_CHECK(hipGraphInstantiate(&s->graph[prec], g, nullptr, nullptr, 0));
    HIP_CHECK(hipGraphDestroy(g));
    return s->graph[prec];
}

void retire(dec_server* s, int k, int status, double rel) {
    ServeSlot& sl = s->slots[k];
    dec_mesh* m = sl.mesh;
    m->ctx = s->ctx;  // flux on the caller's stream, after the solve stream
    HIP_CHECK(hipStreamSynchronize(s->solve_stream));
    if (sl.req.T_out)
        HIP_CHECK(hipMemcpyAsync(sl.req.T_out, sl.x64.p, m->V * sizeof(double), hipMemcpyDeviceToDevice,
                                 s->ctx->stream));
    dec_result r{};
    r.ticket = sl.ticket;
    r.user_tag = sl.req.user_tag;
    r.status = status;
    r.rel_residual = rel;
    r.inner_iterations = sl.inner_total;
    r.outer_iterations = sl.outer;
    r.fp64_fallback = sl.fallback ? 1 : 0;
    const int rc = dec_flux_effective_conductivity(m, sl.x64.p, sl.req.side, sl.req.length > 0 ? sl.req.length : 1.0,
                                                   sl.req.area > 0 ? sl.req.area : 1.0, sl.req.dT != 0 ? sl.req.dT : 1.0,
                                                   &r.k_eff, &r.q_in, &r.q_out, &r.energy, nullptr);
    if (rc != DEC_OK && r.status == DEC_OK) r.status = rc;
    r.t_submit_ms = sl.t_submit;
    r.t_admit_ms = sl.t_admit;
    r.t_start_ms = sl.t_start;
    r.t_finish_ms = now_ms(s->t0);
    s->done.push_back(r);
    free_slot(s, sl);
}

// Items of `ids` into the auxiliary table and the ids into d_ids (host staging reused: the
// caller synchronises the stream before building the next list).  Returns the item count.
int stage_items(dec_server* s, const std::vector<int>& ids) {
    const int n = build_items(s, ids, s->h_items, s->max_items);
    HIP_CHECK(hipMemcpyAsync(s->d_items_aux.p, s->h_items, n * sizeof(BItem), hipMemcpyHostToDevice, s->solve_stream));
    for (size_t i = 0; i < ids.size(); ++i) s->h_ids[i] = ids[i];
    HIP_CHECK(hipMemcpyAsync(s->d_ids.p, s->h_ids, ids.size() * sizeof(int32_t), hipMemcpyHostToDevice,
                             s->solve_stream));
    return n;
}

void read_states(dec_server* s) {
    const int ns = (int)s->slots.size();
    HIP_CHECK(hipMemcpyAsync(s->h_st, s->d_st.p, 3 * ns * sizeof(PcgScalars), hipMemcpyDeviceToHost, s->solve_stream));
    HIP_CHECK(hipStreamSynchronize(s->solve_stream));
}

void to_fp64(dec_server* s, ServeSlot& sl) {
    sl.mode = DEC_PREC_FP64;
    sl.fallback = true;
    sl.p64.alloc(&s->setup_ctx, sl.mesh->V);
    sl.q64.alloc(&s->setup_ctx, sl.mesh->V);
}

// Refinement steps for the systems in `ids` (phase PH_OUTER), the steps of the
// single-system refinement loop: an FP32 inner solve that did not converge is
// not applied and the system goes on in FP64; otherwise its correction is
// applied, the FP64 residual taken, and the system retires when it meets the
// tolerance, fails on a non-finite residual, a broken-down FP64 solve or the
// iteration budget, or, when refinement stagnates (the residual not halved),
// goes on in FP64 after taking back a correction that raised the residual.
// Each system then starts its next inner solve: FP32 with at most
// max(max_iters / 8, 64) iterations, FP64 with what is left.
void outer_steps(dec_server* s, const std::vector<int>& ids) {
    if (ids.empty()) return;
    const dim3 g(s->G), b(BLOCK);
    for (int k : ids) HIP_CHECK(hipStreamWaitEvent(s->solve_stream, s->slots[k].ready, 0));
    std::vector<int> fresh;
    for (int k : ids) {
        ServeSlot& sl = s->slots[k];
        if (sl.fresh) {
            fresh.push_back(k);
            continue;
        }
        const PcgScalars& in = s->h_st[3 * k];
        sl.inner_total += in.iter;
        ++sl.outer;
        if (sl.mode == DEC_PREC_MIXED && in.done != PCG_CONVERGED)
            to_fp64(s, sl);  // its correction is not applied (describe() drops the FP32 vectors)
        else if (sl.mode == DEC_PREC_FP64)
            sl.broke = in.done == PCG_BREAKDOWN;
    }
    upload_slots(s);
    const int n = stage_items(s, ids);
    if (!fresh.empty()) {
        hipLaunchKernelGGL(bk_admit_init, g, b, 0, s->solve_stream, s->d_slots.p, s->d_items_aux.p, n);
        hipLaunchKernelGGL(bk_fold_outer, dim3((int)ids.size()), b, 0, s->solve_stream, s->d_slots.p, s->d_ids.p,
                           (int)ids.size(), 1);
    }
    hipLaunchKernelGGL(bk_correct, g, b, 0, s->solve_stream, s->d_slots.p, s->d_items_aux.p, n);
    hipLaunchKernelGGL(bk_residual, g, b, 0, s->solve_stream, s->d_slots.p, s->d_items_aux.p, n);
    hipLaunchKernelGGL(bk_fold_outer, dim3((int)ids.size()), b, 0, s->solve_stream, s->d_slots.p, s->d_ids.p,
                       (int)ids.size(), 0);
    HIP_CHECK(hipGetLastError());
    read_states(s);
    std::vector<int> again, undo;
    for (int k : ids) {
        ServeSlot& sl = s->slots[k];
        const PcgScalars& out = s->h_st[3 * k + 2];
        const double bn = sqrt(out.aux), rn = sqrt(out.rr);
        const double rel = bn > 0 ? rn / bn : 0.0;
        const bool was_fresh = sl.fresh;
        sl.fresh = false;
        if (!std::isfinite(rn) || !std::isfinite(bn)) {
            retire(s, k, DEC_EBREAKDOWN, rel);
            continue;
        }
        if (bn == 0.0 || rn <= s->opts.tol * bn) {
            retire(s, k, DEC_OK, rel);
            continue;
        }
        if (sl.broke) {
            retire(s, k, DEC_EBREAKDOWN, rel);
            continue;
        }
        if (sl.inner_total >= s->opts.max_iters || sl.outer >= 100) {
            retire(s, k, DEC_ENOTCONV, rel);
            continue;
        }
        if (sl.mode == DEC_PREC_MIXED && !was_fresh && rn > 0.5 * sl.rn_prev) {
            // refinement stagnates in FP32: FP64 finishes, from the previous iterate when the
            // last correction raised the residual
            if (rn > sl.rn_prev) {
                undo.push_back(k);
                continue;  // rn_prev stays the residual of the restored iterate
            }
            to_fp64(s, sl);
        }
        sl.rn_prev = rn;
        again.push_back(k);
    }
    if (!undo.empty()) {
        upload_slots(s);  // still mixed: the FP32 correction is in place
        for (int k : undo) s->h_slots[k].undo_scale = s->slots[k].rn_prev;
        HIP_CHECK(hipMemcpyAsync(s->d_slots.p, s->h_slots, s->slots.size() * sizeof(BSlot), hipMemcpyHostToDevice,
                                 s->solve_stream));
        const int m = stage_items(s, undo);
        hipLaunchKernelGGL(bk_undo, g, b, 0, s->solve_stream, s->d_slots.p, s->d_items_aux.p, m);
        hipLaunchKernelGGL(bk_residual, g, b, 0, s->solve_stream, s->d_slots.p, s->d_items_aux.p, m);
        hipLaunchKernelGGL(bk_fold_outer, dim3((int)undo.size()), b, 0, s->solve_stream, s->d_slots.p, s->d_ids.p,
                           (int)undo.size(), 0);
        HIP_CHECK(hipGetLastError());
        HIP_CHECK(hipStreamSynchronize(s->solve_stream));  // before the staging area is reused
        for (int k : undo) {
            to_fp64(s, s->slots[k]);
            again.push_back(k);
        }
    }
    if (again.empty()) return;
    // start the next inner solves
    upload_slots(s);
    std::vector<int> by_mode[2];
    for (int k : again) by_mode[s->slots[k].mode == DEC_PREC_MIXED ? 1 : 0].push_back(k);
    const int64_t cap32 = s->opts.max_iters / 8 > 64 ? s->opts.max_iters / 8 : 64;
    for (int prec = 0; prec < 2; ++prec) {
        if (by_mode[prec].empty()) continue;
        for (int k : by_mode[prec]) {
            ServeSlot& sl = s->slots[k];
            const PcgScalars& out = s->h_st[3 * k + 2];
            const double bn = sqrt(out.aux), rn = sl.rn_prev;
            const int64_t left = s->opts.max_iters - sl.inner_total;
            if (prec == 1) {
                double itol = s->opts.inner_tol;
                if (s->opts.adaptive_final_inner) itol = fmax(itol, 0.5 * s->opts.tol * bn / rn);
                if (itol >= 1.0) itol = 0.5;
                s->h_slots[k].stop_factor = itol * itol;
                s->h_slots[k].relative = 1;
                s->h_slots[k].max_iter = left < cap32 ? left : cap32;
            } else {
                s->h_slots[k].stop_factor = s->opts.tol * s->opts.tol;
                s->h_slots[k].relative = 0;
                s->h_slots[k].max_iter = left;
            }
        }
        const int ns2 = (int)s->slots.size();
        HIP_CHECK(hipMemcpyAsync(s->d_slots.p, s->h_slots, ns2 * sizeof(BSlot), hipMemcpyHostToDevice,
                                 s->solve_stream));
        const int m = stage_items(s, by_mode[prec]);
        if (prec == 1)
            hipLaunchKernelGGL(bk_inner_start<float>, g, b, 0, s->solve_stream, s->d_slots.p, s->d_items_aux.p, m);
        else
            hipLaunchKernelGGL(bk_inner_start<double>, g, b, 0, s->solve_stream, s->d_slots.p, s->d_items_aux.p, m);
        hipLaunchKernelGGL(bk_inner_fold, dim3((int)by_mode[prec].size()), b, 0, s->solve_stream, s->d_slots.p,
                           s->d_ids.p, (int)by_mode[prec].size());
        HIP_CHECK(hipGetLastError());
        // the host copies above reuse h_items / h_ids: wait before the next list overwrites them
        HIP_CHECK(hipStreamSynchronize(s->solve_stream));
        for (int k : by_mode[prec]) {
            ServeSlot& sl = s->slots[k];
            if (sl.phase != PH_INNER) sl.t_start = sl.t_start > 0 ? sl.t_start : now_ms(s->t0);
            sl.phase = PH_INNER;
            sl.iter_mark = 0;  // a new inner solve
        }
    }
}

}  // namespace

extern "C" {

int dec_server_opts_default(dec_server_opts* o) {
    if (!o) return DEC_EINVAL;
    std::memset(o, 0, sizeof(*o));
    o->precision = DEC_PREC_MIXED;
    o->tol = 1e-10;
    o->inner_tol = 1e-5;
    o->adaptive_final_inner = 1;
    o->max_iters = 100000;
    o->max_slots = 64;
    o->chunk = 16;
    return DEC_OK;
}

int dec_server_create(dec_ctx* ctx, size_t hbm_budget_bytes, const dec_server_opts* opts, dec_server** out) {
    if (!ctx || !out) return DEC_EINVAL;
    *out = nullptr;
    dec_server* s = new dec_server();
    try {
        dec_server_opts o;
        dec_server_opts_default(&o);
        if (opts) o = *opts;
        DEC_REQUIRE(o.precision == DEC_PREC_FP64 || o.precision == DEC_PREC_MIXED, DEC_EINVAL, "bad precision");
        DEC_REQUIRE(o.max_slots > 0 && o.max_slots <= 1024, DEC_EINVAL, "max_slots must be in 1..1024");
        DEC_REQUIRE(o.chunk >= 2 && o.chunk <= 1024 && o.chunk % 2 == 0, DEC_EINVAL, "chunk must be even, 2..1024");
        DEC_REQUIRE(o.tol > 0 && o.inner_tol > 0 && o.inner_tol < 1 && o.max_iters > 0, DEC_EINVAL, "bad tolerances");
        ctx->set_device();
        s->ctx = ctx;
        ctx->live_children += 1;
        s->opts = o;
        s->budget = hbm_budget_bytes;
        s->t0 = std::chrono::steady_clock::now();
        HIP_CHECK(hipStreamCreateWithFlags(&s->solve_stream, hipStreamNonBlocking));
        HIP_CHECK(hipStreamCreateWithFlags(&s->setup_stream, hipStreamNonBlocking));
        HIP_CHECK(hipEventCreateWithFlags(&s->ev_chunk, hipEventDisableTiming));
        // timing events without the system-scope fence (its cache writeback would slow the batch)
        HIP_CHECK(hipEventCreateWithFlags(&s->ev_b0, hipEventDisableSystemFence));
        HIP_CHECK(hipEventCreateWithFlags(&s->ev_b1, hipEventDisableSystemFence));
        s->setup_ctx.device = ctx->device;
        s->setup_ctx.stream = s->setup_stream;
        s->setup_ctx.alloc = ctx->alloc;
        s->setup_ctx.free_fn = ctx->free_fn;
        s->setup_ctx.user = ctx->user;
        s->setup_ctx.num_cus = ctx->num_cus;
        s->G = 8 * ctx->num_cus;
        s->slots.resize(o.max_slots);
        s->max_items = 1 << 20;  // 2^20 chunks of 2048 rows: 2^31 rows in flight at most
        s->d_slots.alloc(ctx, o.max_slots);
        s->d_items32.alloc(ctx, s->max_items);
        s->d_items64.alloc(ctx, s->max_items);
        s->d_items_aux.alloc(ctx, s->max_items);
        s->d_n.alloc(ctx, 2);
        s->d_ids.alloc(ctx, o.max_slots);
        s->d_st.alloc(ctx, 3 * (int64_t)o.max_slots);
        HIP_CHECK(hipMemsetAsync(s->d_st.p, 0, 3 * o.max_slots * sizeof(PcgScalars), s->solve_stream));
        HIP_CHECK(hipMemsetAsync(s->d_n.p, 0, 2 * sizeof(int32_t), s->solve_stream));
        HIP_CHECK(hipHostMalloc((void**)&s->h_slots, o.max_slots * sizeof(BSlot), hipHostMallocDefault));
        HIP_CHECK(hipHostMalloc((void**)&s->h_items, s->max_items * sizeof(BItem), hipHostMallocDefault));
        HIP_CHECK(hipHostMalloc((void**)&s->h_n, 2 * sizeof(int32_t), hipHostMallocDefault));
        HIP_CHECK(hipHostMalloc((void**)&s->h_ids, o.max_slots * sizeof(int32_t), hipHostMallocDefault));
        HIP_CHECK(hipHostMalloc((void**)&s->h_st, 3 * o.max_slots * sizeof(PcgScalars), hipHostMallocDefault));
        std::memset(s->h_slots, 0, o.max_slots * sizeof(BSlot));
        HIP_CHECK(hipStreamSynchronize(s->solve_stream));
    } catch (const DecError& e) {
        ctx->last_error = e.msg;
        dec_server_destroy(s);
        return e.code;
    }
    *out = s;
    return DEC_OK;
}

int dec_server_submit(dec_server* s, const dec_request* req, uint64_t* ticket) {
    if (!s || !req) return DEC_EINVAL;
    try {
        if (req->mesh)
            DEC_REQUIRE(req->V == req->mesh->V && req->T == req->mesh->T && !req->mesh->dual &&
                            req->mesh->ctx->device == s->ctx->device,
                        DEC_EINVAL, "a request's mesh must match its V and T, hold vertex unknowns and share the device");
        DEC_REQUIRE(req->V > 0 && req->T > 0 && (req->mesh || (req->xyz && req->tets)) && req->bc_type && req->bc_value,
                    DEC_EINVAL, "request needs a mesh or xyz and tets, and bc_type and bc_value");
        DEC_REQUIRE(req->n_cracks >= 0 && (req->n_cracks == 0 || req->cracks), DEC_EINVAL, "bad crack array");
        DEC_REQUIRE(estimate_bytes(req->V, req->T) <= (int64_t)s->budget, DEC_EBUDGET,
                    "request does not fit the HBM budget even alone");
    } catch (const DecError& e) {
        s->ctx->last_error = e.msg;
        return e.code;
    }
    ServeReq q;
    try {
        s->ctx->set_device();
        HIP_CHECK(hipEventCreateWithFlags(&q.inputs, hipEventDisableTiming));
        HIP_CHECK(hipEventRecord(q.inputs, s->ctx->stream));
    } catch (const DecError& e) {
        s->ctx->last_error = e.msg;
        return e.code;
    }
    q.ticket = s->next_ticket++;
    q.req = *req;
    q.t_submit = now_ms(s->t0);
    s->pending.push_back(q);
    if (ticket) *ticket = q.ticket;
    return DEC_OK;
}

int dec_server_step(dec_server* s, int32_t* n_active, int32_t* n_pending) {
    if (!s) return DEC_EINVAL;
    try {
        s->ctx->set_device();
        const int ns = (int)s->slots.size();
        ++s->steps;
        double mark = now_ms(s->t0);
        auto phase = [&](int k) {  // host time of a phase of this step
            const double t = now_ms(s->t0);
            s->host_ms[k] += t - mark;
            mark = t;
        };
        // 1. one batch of inner iterations for every system in PH_INNER
        std::vector<int> inner[2];
        for (int k = 0; k < ns; ++k)
            if (s->slots[k].phase == PH_INNER) inner[s->slots[k].mode == DEC_PREC_MIXED ? 1 : 0].push_back(k);
        bool launched = false;
        if (!inner[0].empty() || !inner[1].empty()) {
            upload_slots(s);
            const int n64 = build_items(s, inner[0], s->h_items, s->max_items);
            HIP_CHECK(hipMemcpyAsync(s->d_items64.p, s->h_items, n64 * sizeof(BItem), hipMemcpyHostToDevice,
                                     s->solve_stream));
            const int n32 = build_items(s, inner[1], s->h_items + n64, s->max_items - n64);
            HIP_CHECK(hipMemcpyAsync(s->d_items32.p, s->h_items + n64, n32 * sizeof(BItem), hipMemcpyHostToDevice,
                                     s->solve_stream));
            s->h_n[0] = n32;
            s->h_n[1] = n64;
            HIP_CHECK(hipMemcpyAsync(s->d_n.p, s->h_n, 2 * sizeof(int32_t), hipMemcpyHostToDevice, s->solve_stream));
            for (int prec = 0; prec < 2; ++prec) {  // time the variant again on a batch twice as large
                const int n = prec == 1 ? n32 : n64;
                if (s->tuned[prec] && n >= 2 * s->tuned_items[prec] && s->tunings[prec] < MAX_TUNINGS) {
                    s->tuned[prec] = false;
                    if (s->graph[prec]) HIP_CHECK(hipGraphExecDestroy(s->graph[prec]));
                    s->graph[prec] = nullptr;
                }
                if (n && !s->tuned[prec]) {
                    s->tuned_items[prec] = n;
                    ++s->tunings[prec];
                }
            }
            hipGraphExec_t g32 = n32 ? batched_graph(s, 1) : nullptr;  // captured (and tuned) on first use
            hipGraphExec_t g64 = n64 ? batched_graph(s, 0) : nullptr;
            HIP_CHECK(hipEventRecord(s->ev_b0, s->solve_stream));
            if (g32) HIP_CHECK(hipGraphLaunch(g32, s->solve_stream));
            if (g64) HIP_CHECK(hipGraphLaunch(g64, s->solve_stream));
            HIP_CHECK(hipEventRecord(s->ev_b1, s->solve_stream));
            HIP_CHECK(hipEventRecord(s->ev_chunk, s->solve_stream));
            launched = true;
        }
        phase(0);
        // 2. admissions (setup overlaps the batch on the setup stream)
        while (!s->pending.empty()) {
            int free_k = -1;
            for (int k = 0; k < ns; ++k)
                if (s->slots[k].phase == PH_FREE) {
                    free_k = k;
                    break;
                }
            if (free_k < 0) break;
            const ServeReq& q = s->pending.front();
            if (s->committed + estimate_bytes(q.req.V, q.req.T) > (int64_t)s->budget) break;
            ServeReq qq = q;
            s->pending.pop_front();
            admit(s, qq, free_k);
        }
        phase(1);
        // 3. wait for the batch, then refinement steps for systems whose inner solve ended
        if (launched) HIP_CHECK(hipEventSynchronize(s->ev_chunk));
        HIP_CHECK(hipMemcpyAsync(s->h_st, s->d_st.p, 3 * ns * sizeof(PcgScalars), hipMemcpyDeviceToHost,
                                 s->solve_stream));
        HIP_CHECK(hipStreamSynchronize(s->solve_stream));
        phase(2);
        if (launched) {  // the batch's replay time and the iterations it ran
            float ms = 0.0f;
            HIP_CHECK(hipEventElapsedTime(&ms, s->ev_b0, s->ev_b1));
            s->batch_ms += ms;
            for (int prec = 0; prec < 2; ++prec)
                for (int k : inner[prec]) {
                    ServeSlot& sl = s->slots[k];
                    const int64_t ran = s->h_st[3 * k].iter - sl.iter_mark;
                    s->batch_iterations += ran;
                    s->batch_bytes += (double)ran * batched_iteration_bytes(sl.mesh, sl.mode);
                    sl.iter_mark = s->h_st[3 * k].iter;
                }
        }
        std::vector<int> outer;
        for (int k = 0; k < ns; ++k) {
            ServeSlot& sl = s->slots[k];
            if (sl.phase == PH_INNER && s->h_st[3 * k].done != PCG_RUNNING) sl.phase = PH_OUTER;
            if (sl.phase == PH_OUTER) {
                if (sl.fresh && hipEventQuery(sl.ready) != hipSuccess) continue;  // setup still running
                outer.push_back(k);
            }
        }
        // fresh systems (b.b, x0) first, then the others
        std::vector<int> fresh, old;
        for (int k : outer) (s->slots[k].fresh ? fresh : old).push_back(k);
        outer_steps(s, fresh);
        outer_steps(s, old);
        phase(3);
        int act = 0;
        for (int k = 0; k < ns; ++k) act += s->slots[k].phase != PH_FREE;
        if (n_active) *n_active = act;
        if (n_pending) *n_pending = (int32_t)s->pending.size();
    } catch (const DecError& e) {
        s->ctx->last_error = e.msg;
        return e.code;
    }
    return DEC_OK;
}

int dec_server_poll(dec_server* s, dec_result* out, int32_t max, int32_t* n_out) {
    if (!s || (max > 0 && !out) || !n_out) return DEC_EINVAL;
    const int n = (int)s->done.size() < max ? (int)s->done.size() : max;
    for (int i = 0; i < n; ++i) out[i] = s->done[i];
    s->done.erase(s->done.begin(), s->done.begin() + n);
    *n_out = n;
    return DEC_OK;
}

int dec_server_stats(const dec_server* s, dec_server_counters* out) {
    if (!s || !out) return DEC_EINVAL;
    out->batch_ms = s->batch_ms;
    out->batch_bytes = s->batch_bytes;
    out->batch_iterations = s->batch_iterations;
    for (int k = 0; k < 2; ++k) {
        out->variant[2 * k] = s->tuned[k] ? s->unroll[k] : 0;
        out->variant[2 * k + 1] = s->tuned[k] ? s->nt[k] : 0;
        out->order[k] = s->tuned[k] ? s->order[k] : 0;
    }
    for (int k = 0; k < 4; ++k) out->host_ms[k] = s->host_ms[k];
    out->steps = s->steps;
    return DEC_OK;
}

int dec_server_cancel(dec_server* s, uint64_t ticket) {
    if (!s) return DEC_EINVAL;
    for (auto it = s->pending.begin(); it != s->pending.end(); ++it) {
        if (it->ticket == ticket) {
            dec_result r{};
            r.ticket = ticket;
            r.user_tag = it->req.user_tag;
            r.status = DEC_ECANCELED;
            r.t_submit_ms = it->t_submit;
            r.t_finish_ms = now_ms(s->t0);
            s->done.push_back(r);
            (void)hipEventDestroy(it->inputs);
            s->pending.erase(it);
            return DEC_OK;
        }
    }
    try {
        for (size_t k = 0; k < s->slots.size(); ++k) {
            ServeSlot& sl = s->slots[k];
            if (sl.phase != PH_FREE && sl.ticket == ticket) {
                HIP_CHECK(hipStreamSynchronize(s->solve_stream));
                HIP_CHECK(hipStreamSynchronize(s->setup_stream));
                dec_result r{};
                r.ticket = ticket;
                r.user_tag = sl.req.user_tag;
                r.status = DEC_ECANCELED;
                r.t_submit_ms = sl.t_submit;
                r.t_admit_ms = sl.t_admit;
                r.t_finish_ms = now_ms(s->t0);
                s->done.push_back(r);
                free_slot(s, sl);
                return DEC_OK;
            }
        }
    } catch (const DecError& e) {
        s->ctx->last_error = e.msg;
        return e.code;
    }
    return DEC_EINVAL;
}

int dec_server_destroy(dec_server* s) {
    if (!s) return DEC_EINVAL;
    if (s->solve_stream) (void)hipStreamSynchronize(s->solve_stream);
    if (s->setup_stream) (void)hipStreamSynchronize(s->setup_stream);
    for (auto& sl : s->slots) {
        if (sl.phase != PH_FREE) free_slot(s, sl);
        if (sl.ready) (void)hipEventDestroy(sl.ready);
    }
    for (ServeReq& q : s->pending) (void)hipEventDestroy(q.inputs);
    for (hipGraphExec_t g : s->graph)
        if (g) (void)hipGraphExecDestroy(g);
    s->d_slots.release();
    s->d_items32.release();
    s->d_items64.release();
    s->d_items_aux.release();
    s->d_n.release();
    s->d_ids.release();
    s->d_st.release();
    if (s->h_slots) (void)hipHostFree(s->h_slots);
    if (s->h_items) (void)hipHostFree(s->h_items);
    if (s->h_n) (void)hipHostFree(s->h_n);
    if (s->h_ids) (void)hipHostFree(s->h_ids);
    if (s->h_st) (void)hipHostFree(s->h_st);
    if (s->ev_chunk) (void)hipEventDestroy(s->ev_chunk);
    if (s->ev_b0) (void)hipEventDestroy(s->ev_b0);
    if (s->ev_b1) (void)hipEventDestroy(s->ev_b1);
    if (s->setup_ctx.pinned) (void)hipHostFree(s->setup_ctx.pinned);
    if (s->solve_stream) (void)hipStreamDestroy(s->solve_stream);
    if (s->setup_stream) (void)hipStreamDestroy(s->setup_stream);
    if (s->ctx) s->ctx->live_children -= 1;
    delete s;
    return DEC_OK;
}

}  // extern "C"
