// The sliced-ELL product y = A x (Section 2.3: the solver's matrix-vector
// product), the dominant kernel of every solve.  Kept on its own so that the
// HBM counters recorded for it can be tied to exactly this source.
//
// Layout: slices of SELL_C = 64 consecutive rows, one row per lane of a
// wavefront; entry j of row r of slice s sits at ptr[s] + j * 64 + (r - 64 s),
// so each load instruction of a wavefront reads one contiguous 256 B (column)
// or 512 B (FP64 value) segment.  Padding entries repeat the row's own column
// with value 0.
#pragma once

#include "common.h"

template <class VT>
struct SellView {
    const int64_t* ptr;
    const int32_t* col;
    const VT* val;
    int64_t nslices;
    int64_t V;
};

// Row `lane` of the slice starting at `base` with `width` stored entries per
// row: sum over the row's entries in stored (ascending column) order.  The
// entries go in groups of U: all column and value loads of a group are
// issued before its x gathers, and the last group is predicated (the width
// is uniform across the wavefront), so no entry waits on the one before.
template <class T, bool NT>
__device__ __forceinline__ T stream_load(const T* p) {
    if (NT) return __builtin_nontemporal_load(p);
    return *p;
}

template <class VT, int U, bool NT = true>
__device__ __forceinline__ VT sell_row(const SellView<VT>& A, int64_t base, int width, int lane,
                                       const VT* __restrict__ x) {
    const int32_t* cp = A.col + base + lane;
    const VT* vp = A.val + base + lane;
    VT acc = 0;
    for (int j = 0; j < width; j += U) {
        int32_t c[U];
        VT v[U], xv[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const bool ok = j + u < width;
            c[u] = ok ? stream_load<int32_t, NT>(cp + u * SELL_C) : 0;
            v[u] = ok ? stream_load<VT, NT>(vp + u * SELL_C) : VT(0);
        }
#pragma unroll
        for (int u = 0; u < U; ++u) xv[u] = (j + u < width) ? x[c[u]] : VT(0);
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (j + u < width) acc += v[u] * xv[u];
        cp += U * SELL_C;
        vp += U * SELL_C;
    }
    return acc;
}

enum { MODE_PLAIN = 0, MODE_DOT = 1, MODE_RESID = 2, MODE_DOTB = 3 };

// y = A x (PLAIN), y = A x with per-block partials of x.y (DOT),
// y = b - A x with per-block partials of y.y (RESID), or y = A x with
// per-block partials of b.y (DOTB).  A launch whose `done` flag (if given)
// is set returns at once: inside a batch of PCG iterations that has
// converged, the remaining launches do nothing.
template <class VT, int MODE, int U, bool NT>
__global__ __launch_bounds__(BLOCK) void k_sell(SellView<VT> A, const VT* __restrict__ x, VT* __restrict__ y,
                                                const VT* __restrict__ b, double* __restrict__ partials,
                                                const int32_t* __restrict__ done) {
    __shared__ double lds[BLOCK / 64 + 1];
    if (done != nullptr && *done) return;
    int64_t s0, s1;
    block_range(A.nslices, &s0, &s1);
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    VT d = 0;
    for (int64_t s = s0 + w; s < s1; s += BLOCK / 64) {
        const int64_t base = A.ptr[s];
        const int width = static_cast<int>((A.ptr[s + 1] - base) / SELL_C);
        const int64_t row = s * SELL_C + lane;
        const VT acc = sell_row<VT, U, NT>(A, base, width, lane, x);
        if (row < A.V) {
            if (MODE == MODE_RESID) {
                const VT ri = b[row] - acc;
                y[row] = ri;
                d += ri * ri;
            } else {
                y[row] = acc;
                if (MODE == MODE_DOT) d += x[row] * acc;
                if (MODE == MODE_DOTB) d += b[row] * acc;
            }
        }
    }
    if (MODE == MODE_PLAIN) return;
    const double bs = block_sum(static_cast<double>(d), lds);
    if (threadIdx.x == 0) partials[blockIdx.x] = bs;
}

