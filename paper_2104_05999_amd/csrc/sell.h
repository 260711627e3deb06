// The sliced-ELL product y = A x (Section 2.3: the solver's matrix-vector
// product), the dominant kernel of every solve.  Kept on its own so that the
// HBM counters recorded for it can be tied to exactly this source.
//
// Layout (see sell_index): slices of SELL_C = 64 consecutive rows, one row
// per lane of a wavefront, consecutive entries of a row stored in pairs, so
// each load instruction of a wavefront reads two entries of every row from one
// contiguous 512 B (column) or 1 KiB (FP64 value) segment.  Where every
// entry's column lies within 2^15 of its row, the columns are read as 16-bit
// offsets from the row instead (one 256 B segment per pair): a spatially
// numbered mesh keeps its neighbours that close, and the bytes per stored
// entry fall from 12 to 10 (FP64) and from 8 to 6 (FP32).  Where the stored
// entries take at most 256 distinct offsets (a lattice numbered in order has
// seven, whatever its size), each column is one byte, an index into the
// matrix's table of offsets, which every workgroup stages in LDS: 9 bytes per
// FP64 entry, 5 per FP32 entry, and the same columns.
#pragma once

#include <type_traits>

#include "common.h"

// With `excess` set, the product is taken in difference form,
//     (A x)_i = excess_i x_i + sum_{j != i} a_ij (x_j - x_i),
// where excess_i = a_ii + sum_{j != i} a_ij is kept exactly (from the weights
// that make it up, never as that difference).  For a Laplacian-like matrix
// with weights of very different size this avoids the cancellation of
// a_ii x_i against its neighbours, so the product keeps full relative accuracy
// in the smooth components; the stored diagonal then multiplies x_i - x_i = 0.
template <class VT>
struct SellView {
    const int64_t* ptr;
    const int32_t* col;
    const VT* val;
    int64_t nslices;
    int64_t V;
    const VT* excess = nullptr;  // [V], or null for the plain product
    const int16_t* dcol = nullptr;  // [entries] col - row, or null: the int32 columns
    const uint8_t* tcol = nullptr;  // [entries] index into otab of col - row, or null
    const int32_t* otab = nullptr;  // [ntab] the offsets tcol indexes
    int32_t ntab = 0;
    uint32_t band_plane = 0;  // banded slice order (see banded_slice): slices per plane, 0 for none
    uint32_t band = 0;        // slices per band
};

// How the product reads its columns: int32 columns, 16-bit offsets from the
// row, or one-byte indices into the offset table.
enum { CF_I32 = 0, CF_I16 = 1, CF_U8 = 2 };
constexpr int OTAB_MAX = 256;

// Native two-element vectors for the paired loads.
template <class T>
struct Pair;
template <>
struct Pair<int32_t> {
    typedef int32_t type __attribute__((ext_vector_type(2)));
};
template <>
struct Pair<int16_t> {
    typedef int16_t type __attribute__((ext_vector_type(2)));
};
template <>
struct Pair<uint8_t> {
    typedef uint8_t type __attribute__((ext_vector_type(2)));
};
template <>
struct Pair<double> {
    typedef double type __attribute__((ext_vector_type(2)));
};
template <>
struct Pair<float> {
    typedef float type __attribute__((ext_vector_type(2)));
};

// How a pair of stored columns is loaded (one load per pair) and split: the
// pair is kept as the bits it was loaded as and split only where the columns
// are used, so the load can stay in flight until then.
template <int CF>
struct RawCol;
template <>
struct RawCol<CF_U8> {
    typedef uint16_t pair;  // two one-byte indices
    typedef uint8_t one;
    typedef uint32_t bits;
    static __device__ __forceinline__ int32_t lo(bits b, int32_t row, const int32_t* tab) {
        return row + tab[b & 0xff];
    }
    static __device__ __forceinline__ int32_t hi(bits b, int32_t row, const int32_t* tab) {
        return row + tab[b >> 8];
    }
};
template <>
struct RawCol<CF_I16> {
    typedef uint32_t pair;  // two 16-bit offsets
    typedef int16_t one;
    typedef uint32_t bits;
    static __device__ __forceinline__ int32_t lo(bits b, int32_t row, const int32_t*) {
        return row + static_cast<int16_t>(b & 0xffff);
    }
    static __device__ __forceinline__ int32_t hi(bits b, int32_t row, const int32_t*) {
        return row + (static_cast<int32_t>(b) >> 16);
    }
};
template <>
struct RawCol<CF_I32> {
    typedef Pair<int32_t>::type pair;
    typedef int32_t one;
    typedef Pair<int32_t>::type bits;
    static __device__ __forceinline__ int32_t lo(bits b, int32_t, const int32_t*) { return b.x; }
    static __device__ __forceinline__ int32_t hi(bits b, int32_t, const int32_t*) { return b.y; }
};

template <int CF, class VT>
__device__ __forceinline__ const typename RawCol<CF>::one* raw_cols(const SellView<VT>& A) {
    if constexpr (CF == CF_U8)
        return A.tcol;
    else if constexpr (CF == CF_I16)
        return A.dcol;
    else
        return A.col;
}

// the column of one stored entry from its stored form
template <int CF>
__device__ __forceinline__ int32_t one_col(int32_t raw, int32_t row, const int32_t* tab) {
    return CF == CF_U8 ? row + tab[raw] : CF == CF_I16 ? row + raw : raw;
}

template <class T, bool NT>
__device__ __forceinline__ T stream_load(const T* p) {
    if (NT) return __builtin_nontemporal_load(p);
    return *p;
}

// Row `lane` of the slice starting at `base` with `width` stored entries per
// row: sum over the row's entries in stored (ascending column) order.  x is
// indexed with unsigned 32-bit columns (every column is in [0, V), V < 2^31),
// so a gather's address is the uniform base plus a 32-bit offset.  The
// pairs go in groups of U, each pair's column load next to its value load
// and decoded as it arrives, the group's x gathers after them; the last
// group is predicated (the width is uniform across the wavefront).  Loads
// complete in the order they are issued, so decoding a pair's column also
// waits for the values issued before it: a group's column round trips
// follow one another (sell_row_cfirst issues the columns first instead).
// An odd last entry (rows of 7 entries are the common case on these meshes)
// has its column and value loaded before the first group and its x gathered
// with the last group's.  The terms are added in entry order, so every
// layout, unroll and load order gives the same sum.  DIFF: each term is a_ij (x_j - xi).  CF:
// the columns as int32 (A.col), 16-bit offsets (A.dcol) added to `row`, or
// one-byte indices (A.tcol) into the offset table `tab` (in LDS) added to
// `row`.  A lane past the last row decodes columns that lie inside x: with
// one-byte indices its `row` is the last row and its entries index the
// offset 0; otherwise its `row` is its own (past the end of x) and its
// stored padding offsets or columns name a column inside x.
template <class VT, int U, bool NT = true, bool DIFF = false, int CF = CF_I32>
__device__ __forceinline__ VT sell_row(const SellView<VT>& A, int64_t base, int width, int lane,
                                       const VT* __restrict__ x, VT xi = 0, int32_t row = 0,
                                       const int32_t* tab = nullptr) {
    typedef typename Pair<int32_t>::type C2;
    typedef typename Pair<int16_t>::type D2;
    typedef typename Pair<uint8_t>::type B2;
    typedef typename Pair<VT>::type V2;
    const int np = width >> 1;
    const C2* cp = reinterpret_cast<const C2*>(A.col + base) + lane;
    const D2* dp = reinterpret_cast<const D2*>(A.dcol + base) + lane;
    const B2* bp = reinterpret_cast<const B2*>(A.tcol + base) + lane;
    const V2* vp = reinterpret_cast<const V2*>(A.val + base) + lane;
    const bool odd = width & 1;
    const int64_t ko = base + static_cast<int64_t>(np) * (2 * SELL_C) + lane;
    int32_t oc = 0;  // the odd entry's column as stored (index, offset or column)
    VT vo = 0, xo = 0;
    if (odd) {
        oc = CF == CF_U8    ? static_cast<int32_t>(stream_load<uint8_t, NT>(A.tcol + ko))
             : CF == CF_I16 ? static_cast<int32_t>(stream_load<int16_t, NT>(A.dcol + ko))
                            : stream_load<int32_t, NT>(A.col + ko);
        vo = stream_load<VT, NT>(A.val + ko);
    }
    auto odd_gather = [&]() {
        const int32_t c = CF == CF_U8 ? row + tab[oc] : CF == CF_I16 ? row + oc : oc;
        xo = DIFF ? x[static_cast<uint32_t>(c)] - xi : x[static_cast<uint32_t>(c)];
    };
    VT acc = 0;
    for (int t = 0; t < np; t += U) {
        C2 c[U];
        V2 v[U];
        VT x0[U], x1[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const bool ok = t + u < np;
            if (CF == CF_U8) {
                const B2 d = ok ? stream_load<B2, NT>(bp + u * SELL_C) : B2(0);
                c[u].x = row + tab[d.x];
                c[u].y = row + tab[d.y];
            } else if (CF == CF_I16) {
                const D2 d = ok ? stream_load<D2, NT>(dp + u * SELL_C) : D2(0);
                c[u].x = row + d.x;
                c[u].y = row + d.y;
            } else {
                c[u] = ok ? stream_load<C2, NT>(cp + u * SELL_C) : C2(0);
            }
            v[u] = ok ? stream_load<V2, NT>(vp + u * SELL_C) : V2(0);
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const bool ok = t + u < np;
            x0[u] = ok ? x[static_cast<uint32_t>(c[u].x)] : VT(0);
            x1[u] = ok ? x[static_cast<uint32_t>(c[u].y)] : VT(0);
            if (DIFF) {
                x0[u] -= xi;
                x1[u] -= xi;
            }
        }
        if (odd && t + U >= np) odd_gather();
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (t + u < np) {
                acc += v[u].x * x0[u];
                acc += v[u].y * x1[u];
            }
        cp += U * SELL_C;
        dp += U * SELL_C;
        bp += U * SELL_C;
        vp += U * SELL_C;
    }
    if (odd) {
        if (np == 0) odd_gather();
        acc += vo * xo;
    }
    return acc;
}

// sell_row with each group's loads in another order: all of the group's
// columns first (the first group also takes the odd entry's), then all of its
// values, so that the columns are decoded and the gathers issued while the
// values are still on their way (loads complete in the order they are
// issued).  Where HBM latency is what a row waits for (a matrix far larger
// than the caches) this hides more of it; where the matrix and x come from
// the caches, the interleaved order of sell_row was faster on this GPU, so
// the autotuner times both.  The same terms are added in the same order.
template <class VT, int U, bool NT = true, bool DIFF = false, int CF = CF_I32>
__device__ __forceinline__ VT sell_row_cfirst(const SellView<VT>& A, int64_t base, int width, int lane,
                                       const VT* __restrict__ x, VT xi = 0, int32_t row = 0,
                                       const int32_t* tab = nullptr) {
    typedef RawCol<CF> RC;
    typedef typename RC::pair RP;
    typedef typename Pair<VT>::type V2;
    const int np = width >> 1;
    const bool odd = width & 1;
    const int64_t ko = base + static_cast<int64_t>(np) * (2 * SELL_C) + lane;  // the odd entry
    auto gather = [&](int32_t c) {
        const VT xg = x[static_cast<uint32_t>(c)];
        return DIFF ? xg - xi : xg;
    };
    if (np == 0) {
        if (!odd) return VT(0);
        const int32_t oc = static_cast<int32_t>(stream_load<typename RC::one, NT>(raw_cols<CF>(A) + ko));
        const VT vo = stream_load<VT, NT>(A.val + ko);
        return vo * gather(one_col<CF>(oc, row, tab));
    }
    const RP* rp = reinterpret_cast<const RP*>(raw_cols<CF>(A) + base) + lane;
    const V2* vp = reinterpret_cast<const V2*>(A.val + base) + lane;
    // One group of up to U pairs: its columns first, then its values (loads
    // complete in the order they are issued, so the columns are decoded while
    // the values are still on their way), then the gathers.  Every load is
    // issued whatever the width, so that the waits count them exactly: a pair
    // past the last one is loaded from the group's first pair and not added,
    // and in the first group the odd entry of an even row is loaded from the
    // row's first entry and not used.  The first group also takes the odd
    // entry, so a row of at most 2U + 1 entries costs one round trip for its
    // columns and one for its values and x.
    VT acc = 0, vo = 0, xo = 0;
    auto group = [&](int t, auto first) {
        typename RC::bits rc[U];
        int32_t c0[U], c1[U];
        V2 v[U];
        VT x0[U], x1[U];
        const int64_t ke = odd ? ko : base + lane;
        int32_t oc = 0;
#pragma unroll
        for (int u = 0; u < U; ++u) rc[u] = stream_load<RP, NT>(rp + (t + u < np ? u : 0) * SELL_C);
        if constexpr (first()) oc = static_cast<int32_t>(stream_load<typename RC::one, NT>(raw_cols<CF>(A) + ke));
#pragma unroll
        for (int u = 0; u < U; ++u) v[u] = stream_load<V2, NT>(vp + (t + u < np ? u : 0) * SELL_C);
        if constexpr (first()) vo = stream_load<VT, NT>(A.val + ke);
#pragma unroll
        for (int u = 0; u < U; ++u) {
            c0[u] = RC::lo(rc[u], row, tab);
            c1[u] = RC::hi(rc[u], row, tab);
        }
        // decoded whether or not the row has an odd entry; an even row's stand-in is
        // another row's column, so the gather takes the row's first column instead
        // (a column of this lane's own row: for a lane past the last row the
        // padding's, inside x; the row number itself can lie past the end of x)
        const int32_t cod = one_col<CF>(oc, row, tab);
        const int32_t co = odd ? cod : c0[0];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            x0[u] = gather(c0[u]);
            x1[u] = gather(c1[u]);
        }
        if constexpr (first()) xo = gather(co);
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (t + u < np) {
                acc += v[u].x * x0[u];
                acc += v[u].y * x1[u];
            }
        rp += U * SELL_C;
        vp += U * SELL_C;
    };
    group(0, std::true_type{});
#pragma unroll 1
    for (int t = U; t < np; t += U) group(t, std::false_type{});
    if (odd) acc += vo * xo;
    return acc;
}

// Stage the offset table of a CF_U8 product in LDS (every thread of the block
// calls this before its first row).
__device__ __forceinline__ void stage_offsets(const int32_t* __restrict__ otab, int ntab, int32_t* tab) {
    for (int t = threadIdx.x; t < ntab; t += blockDim.x) tab[t] = otab[t];
    __syncthreads();
}

enum { MODE_PLAIN = 0, MODE_DOT = 1, MODE_RESID = 2, MODE_DOTB = 3 };

// y = A x (PLAIN), y = A x with per-block partials of x.y (DOT),
// y = b - A x with per-block partials of y.y (RESID), or y = A x with
// per-block partials of b.y (DOTB).  A launch whose `done` flag (if given)
// is set returns at once: inside a batch of PCG iterations that has
// converged, the remaining launches do nothing.  DIFF: the difference form
// (A.excess set).  CF: the column format (CF_I16: A.dcol set, CF_U8: A.tcol
// and A.otab set).  ORD: the order of a row's loads (0 sell_row, 1
// sell_row_cfirst).  Up to 3 pairs in flight the kernel is held to 64
// registers, 8 waves per SIMD.
//
// Order of the slices: XCD x (workgroups are dispatched round-robin, so
// blockIdx.x & 7 names it) owns the contiguous x-th eighth of the slices,
// which its workgroups sweep together as a front: wave w of the XCD's j-th
// workgroup takes slices j * 4 + w, then one front width (4 slices per
// workgroup of the XCD) further on, and so on.  At any moment an XCD's waves
// read one contiguous stretch of the matrix, and rows a few front widths
// apart (a neighbour one lattice or cube plane away) are gathered close in
// time, while that part of x is still in the XCD's L2.  (Giving each
// workgroup a contiguous stretch of its own, as the other kernels do, was
// 9% slower at 128^3: 31.2 against 28.6 us.)  A banded matrix has the front
// walk the XCD's share band by band (banded_slice).  gridDim.x must be a
// multiple of 8.
// The slice an XCD takes at step l of its range of n slices.  In plain order
// step l takes slice l.  A banded matrix (band_plane > 0) has its far column
// offsets near one plane of band_plane slices (a lattice or cube plane), and
// an XCD that walked its range in plain order would stream a whole plane of
// the matrix between reading x_j as a row's own value and gathering it for
// the row one plane on, more than its L2 holds.  Its range is then cut into
// planes, the planes into bands of `band` slices, and the XCD takes band 0 of
// every plane, then band 1 of every plane, and so on: the gather one plane on
// comes one band later.  Slices past the last whole plane follow in order.
// A bijection of [0, n) for any plane >= 1 and band >= 1.
__device__ __forceinline__ uint32_t banded_slice(uint32_t l, uint32_t n, uint32_t plane, uint32_t band) {
    if (plane == 0) return l;
    const uint32_t planes = n / plane;
    if (l >= planes * plane) return l;
    const uint32_t stripe = band * planes;  // one band of every plane
    const uint32_t b = l / stripe;
    const uint32_t in = l - b * stripe;
    const uint32_t w = band < plane - b * band ? band : plane - b * band;  // the last band may be narrower
    const uint32_t p = in / w;
    return p * plane + b * band + (in - p * w);
}

// The contribution of row `row` (the product acc of its stored entries) to
// y and to the block's partial sum d.  NT: y is stored non-temporally too
// (the variant for matrices far larger than the caches, where y would not
// stay there for the next kernel either: 256^3 282 -> 268 us).
template <class VT, int MODE, bool DIFF, bool NT = false>
__device__ __forceinline__ void sell_finish(const SellView<VT>& A, int64_t row, VT acc, VT xi, const VT* __restrict__ x,
                                            VT* __restrict__ y, const VT* __restrict__ b, VT& d) {
    // a lane past the last row reads the last row's data and keeps nothing (its loads are
    // unconditional: a load that only some waves issue makes later waits count it)
    const bool in = row < A.V;
    const int64_t rc = in ? row : A.V - 1;
    if (DIFF) acc += A.excess[rc] * xi;
    VT out = acc, t = 0;
    if (MODE == MODE_RESID) {
        out = b[rc] - acc;
        t = out * out;
    } else if (MODE == MODE_DOT) {
        t = xi * acc;
    } else if (MODE == MODE_DOTB) {
        t = b[rc] * acc;
    }
    d += in ? t : VT(0);
    if (in) {
        if (NT)
            __builtin_nontemporal_store(out, y + row);
        else
            y[row] = out;
    }
}

template <class VT, int MODE, int U, bool NT, bool DIFF = false, int CF = CF_I32, int ORD = 0>
__global__ __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(U <= 3 ? 8 : 6))) void k_sell(
    SellView<VT> A, const VT* __restrict__ x, VT* __restrict__ y, const VT* __restrict__ b,
    double* __restrict__ partials, const int32_t* __restrict__ done) {
    __shared__ double lds[BLOCK / 64 + 1];
    __shared__ int32_t tab[CF == CF_U8 ? OTAB_MAX : 1];
    if (done != nullptr && *done) return;
    if (CF == CF_U8) stage_offsets(A.otab, A.ntab, tab);
    constexpr int WAVES = BLOCK / 64;
    // the wave index, uniform across the wavefront (scalar registers for the slice bookkeeping)
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
    const int64_t xcd = blockIdx.x & 7;
    const int64_t s0 = A.nslices * xcd / 8;
    const uint32_t n = static_cast<uint32_t>(A.nslices * (xcd + 1) / 8 - s0);
    const uint32_t step = (gridDim.x >> 3) * WAVES;
    VT d = 0;
    // the row the columns are decoded from (a lane past the last row takes the last row)
    auto decode_row = [&](int64_t row) {
        return static_cast<int32_t>(CF == CF_U8 && row >= A.V ? A.V - 1 : row);
    };
    for (uint32_t l = (blockIdx.x >> 3) * WAVES + w; l < n; l += step) {
        const int64_t s = s0 + banded_slice(l, n, A.band_plane, A.band);
        const int64_t base = A.ptr[s];
        const int width = static_cast<int>((A.ptr[s + 1] - base) / SELL_C);
        const int64_t row = s * SELL_C + lane;
        // the row's own x (DIFF: for the differences, DOT: for x.y), loaded with the matrix
        const VT xr = x[row < A.V ? row : A.V - 1];
        const VT xi = (DIFF || MODE == MODE_DOT) && row < A.V ? xr : VT(0);
        const int32_t drow = decode_row(row);
        const VT acc = ORD == 1 ? sell_row_cfirst<VT, U, NT, DIFF, CF>(A, base, width, lane, x, xi, drow, tab)
                                : sell_row<VT, U, NT, DIFF, CF>(A, base, width, lane, x, xi, drow, tab);
        sell_finish<VT, MODE, DIFF, NT>(A, row, acc, xi, x, y, b, d);
    }
    if (MODE == MODE_PLAIN) return;
    const double bs = block_sum(static_cast<double>(d), lds);
    if (threadIdx.x == 0) partials[blockIdx.x] = bs;
}

