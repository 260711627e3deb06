// Topology of the tetrahedral complex (Section 2.1: cells, incidence, d0):
// vertex -> tet lists, the edge set in lexicographic (lo, hi) order, the
// edge -> tet incidence in ascending tet order, the static CSR pattern of
// L = d0^T *1 d0 (full edge graph plus diagonal) and the boundary faces.
//
// Every list is built per vertex from that vertex's sorted tet list, so the
// result is independent of thread scheduling: integer atomics only count
// (deterministic totals), set bits, or claim slots whose order the per-vertex
// sort then fixes.  Compiled without floating-point contraction: the zero-volume test
// must take the same decision as the FP64 reference.
#include <climits>
#include <type_traits>

#include "common.h"
#include "group_front.h"
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

// Sort each vertex's tet list (ascending tet id).  One 16-lane group per
// vertex: a list of at most 32 distinct ids, two per lane, is ranked in
// registers (rank = number of smaller ids, counted over the group's keys
// brought by the 15 DPP row rotations) and written back; longer lists are
// insertion-sorted by the group's first lane.
constexpr int SG = 16;

template <int R>
__device__ __forceinline__ void rank_rotations(int k0, int k1, int& r0, int& r1) {
    const int o0 = __builtin_amdgcn_mov_dpp(k0, 0x120 + R, 0xf, 0xf, false);  // row_ror:R
    const int o1 = __builtin_amdgcn_mov_dpp(k1, 0x120 + R, 0xf, 0xf, false);
    r0 += (o0 < k0) + (o1 < k0);
    r1 += (o0 < k1) + (o1 < k1);
    if constexpr (R < SG - 1) rank_rotations<R + 1>(k0, k1, r0, r1);
}

__global__ void k_vt_sort(const int64_t* __restrict__ vt_ptr, int32_t* __restrict__ vt_list, int64_t V) {
    const int g = threadIdx.x & (SG - 1);
    GROUP_FRONT_LOOP(v, V, SG) {
        const int64_t b = vt_ptr[v];
        const int d = (int)(vt_ptr[v + 1] - b);
        if (d <= 2 * SG) {
            const int k0 = g < d ? vt_list[b + g] : INT_MAX;
            const int k1 = g + SG < d ? vt_list[b + g + SG] : INT_MAX;
            int r0 = k1 < k0, r1 = k0 < k1;
            rank_rotations<1>(k0, k1, r0, r1);
            if (g < d) vt_list[b + r0] = k0;
            if (g + SG < d) vt_list[b + r1] = k1;
        } else if (g == 0) {
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

// Reductions over one group (a row of 16 lanes, all of them active) with DPP
// row rotations by 8 and 4, then the quad permutations [2,3,0,1] and
// [1,0,3,2]: every lane ends with the result, and no LDS round trip is taken.
template <class Op>
__device__ __forceinline__ int group_reduce(int v, Op op) {
    v = op(v, __builtin_amdgcn_update_dpp(0, v, 0x128, 0xf, 0xf, false));
    v = op(v, __builtin_amdgcn_update_dpp(0, v, 0x124, 0xf, 0xf, false));
    v = op(v, __builtin_amdgcn_update_dpp(0, v, 0x4e, 0xf, 0xf, false));
    v = op(v, __builtin_amdgcn_update_dpp(0, v, 0xb1, 0xf, 0xf, false));
    return v;
}

__device__ __forceinline__ int group_min(int v) {
    return group_reduce(v, [](int a, int b) { return min(a, b); });
}

__device__ __forceinline__ int group_sum(int v) {
    return group_reduce(v, [](int a, int b) { return a + b; });
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

// Vertices of at most 2 * NG tets (every tet of the list in registers) take
// a faster enumeration: each lane keeps the three other vertices of each of
// its two tets as ascending keys w * 8 + tet * 4 + position (tet 0: list
// entry g, tet 1: entry g + NG; INT_MAX past the end).  A round takes the
// group minimum w of the lanes' first keys and each lane drops its keys of w
// -- at most two, a tet holds w at most once, and tet 0's comes first -- so
// the rounds visit the neighbours in ascending order without rescanning the
// tets, and the dropped keys say which of the lane's tets hold w and where.
// Vertex ids must stay below KEY_LIMIT for the keys to fit an int.
constexpr int64_t KEY_LIMIT = (int64_t(1) << 28) - 1;
constexpr int NKEY = 6;
static_assert(NG == 16, "the group reductions work on rows of 16 lanes");

__device__ __forceinline__ void cmp_swap(int& a, int& b) {
    const int lo = min(a, b);
    b = max(a, b);
    a = lo;
}

// the vertices of q other than v as keys, ascending (an absent tet, all -1: four INT_MAX)
__device__ __forceinline__ void tet_keys(const int4& q, int v, int tag, int* k) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int w = vget(q, r);
        k[r] = (w != v && w >= 0) ? (w << 3) | tag | r : INT_MAX;
    }
    cmp_swap(k[0], k[1]);
    cmp_swap(k[2], k[3]);
    cmp_swap(k[0], k[2]);
    cmp_swap(k[1], k[3]);
    cmp_swap(k[1], k[2]);
}

struct LaneKeys {
    int c[NKEY];
    __device__ __forceinline__ void pop_if(bool p) {
#pragma unroll
        for (int i = 0; i < NKEY - 1; ++i) c[i] = p ? c[i + 1] : c[i];
        c[NKEY - 1] = p ? INT_MAX : c[NKEY - 1];
    }
};

__device__ __forceinline__ LaneKeys lane_keys(const GroupTets& gt, int v) {
    int x[8];
    tet_keys(gt.q0, v, 0, x);
    tet_keys(gt.q1, v, 4, x + 4);
    // odd-even merge of the two sorted runs of four (each ends in INT_MAX, so
    // the six smallest are all a lane can hold)
    cmp_swap(x[0], x[4]);
    cmp_swap(x[1], x[5]);
    cmp_swap(x[2], x[6]);
    cmp_swap(x[3], x[7]);
    cmp_swap(x[2], x[4]);
    cmp_swap(x[3], x[5]);
    cmp_swap(x[1], x[2]);
    cmp_swap(x[3], x[4]);
    cmp_swap(x[5], x[6]);
    LaneKeys k;
#pragma unroll
    for (int i = 0; i < NKEY; ++i) k.c[i] = x[i];
    return k;
}

// One round: w is the group's next neighbour (INT_MAX: none left); e0 / e1
// tell whether the lane's first / second dropped key (h0 / h1) was one of w.
struct KeyRound {
    int w = INT_MAX;
    bool e0 = false, e1 = false;
    int h0 = INT_MAX, h1 = INT_MAX;
};

__device__ __forceinline__ KeyRound next_key(LaneKeys& k) {
    KeyRound r;
    r.h0 = k.c[0];
    const int m = group_min(r.h0);
    r.w = m == INT_MAX ? INT_MAX : m >> 3;
    r.e0 = (r.h0 >> 3) == r.w;
    k.pop_if(r.e0);
    r.h1 = k.c[0];
    r.e1 = r.e0 && (r.h1 >> 3) == r.w;
    k.pop_if(r.e1);
    return r;
}

// The count needs the neighbours only: the lane's keys become plain vertex
// ids, a repeat (a vertex in both of the lane's tets, next to each other in
// the sorted keys) is dropped and the six are sorted again, so a round drops
// at most one id per lane.
__device__ __forceinline__ LaneKeys lane_ids(const GroupTets& gt, int v) {
    const LaneKeys k = lane_keys(gt, v);
    int w[NKEY];
#pragma unroll
    for (int i = 0; i < NKEY; ++i) w[i] = k.c[i] == INT_MAX ? INT_MAX : k.c[i] >> 3;
    LaneKeys d;
    d.c[0] = w[0];
#pragma unroll
    for (int i = 1; i < NKEY; ++i) d.c[i] = w[i] == w[i - 1] ? INT_MAX : w[i];
    // sorting network for six
    cmp_swap(d.c[0], d.c[5]);
    cmp_swap(d.c[1], d.c[3]);
    cmp_swap(d.c[2], d.c[4]);
    cmp_swap(d.c[1], d.c[2]);
    cmp_swap(d.c[3], d.c[4]);
    cmp_swap(d.c[0], d.c[3]);
    cmp_swap(d.c[2], d.c[5]);
    cmp_swap(d.c[0], d.c[1]);
    cmp_swap(d.c[2], d.c[3]);
    cmp_swap(d.c[4], d.c[5]);
    cmp_swap(d.c[1], d.c[2]);
    cmp_swap(d.c[3], d.c[4]);
    return d;
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
        int up = 0, all = 0;
        if (d <= 2 * NG && V <= KEY_LIMIT) {
            LaneKeys ids = lane_ids(gt, (int)v);
            while (true) {
                const int w = group_min(ids.c[0]);
                if (w == INT_MAX) break;
                ids.pop_if(ids.c[0] == w);
                ++all;
                up += w > v;
            }
        } else {
            int cur = -1;
            while (true) {
                const int w = group_next(tets, vt_list, b, d, (int)v, cur, g, gt);
                if (w == INT_MAX) break;
                cur = w;
                ++all;
                up += w > v;
            }
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
// tet * 6 + local edge, from inc_ptr[v] on.
__global__ void k_nbr_fill(const int4* __restrict__ tets, const int64_t* __restrict__ vt_ptr,
                           const int32_t* __restrict__ vt_list, int64_t V, const int64_t* __restrict__ up_ptr,
                           const int64_t* __restrict__ row_ptr, const int64_t* __restrict__ inc_ptr,
                           int32_t* __restrict__ edges, int64_t* __restrict__ et_ptr, int32_t* __restrict__ et_inc,
                           int32_t* __restrict__ col, int32_t* __restrict__ nz_edge,
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
        const int64_t row0 = row_ptr[v], up0 = up_ptr[v];
        int64_t ip = inc_ptr[v];
        // Row entries and upper edges are produced one per round; entry j is
        // kept by lane j % NG and every NG of them the group stores together
        // (one coalesced store per array), the rest after the last round.
        int nrow = 0, nup = 0;  // row entries and upper edges so far
        int pcol = 0, pnz = 0;  // this lane's pending row entry: column, edge id
        int phi = 0;            // this lane's pending upper edge: its high end ...
        int64_t pinc = 0;       // ... and its first incidence
        int dpos = -1;          // position of the diagonal in the row
        auto put_row = [&](int c, int z) {
            const bool mine = (nrow & (NG - 1)) == g;
            pcol = mine ? c : pcol;
            pnz = mine ? z : pnz;
            if ((++nrow & (NG - 1)) == 0) {
                col[row0 + nrow - NG + g] = pcol;
                nz_edge[row0 + nrow - NG + g] = pnz;
            }
        };
        auto put_up = [&](int hi, int64_t first) {
            const bool mine = (nup & (NG - 1)) == g;
            phi = mine ? hi : phi;
            pinc = mine ? first : pinc;
            if ((++nup & (NG - 1)) == 0) {
                const int64_t e = up0 + nup - NG + g;
                reinterpret_cast<int2*>(edges)[e] = make_int2((int)v, phi);
                et_ptr[e] = pinc;
            }
        };
        // the rounds, compiled once for waves whose groups all take the fast
        // path (no branch to the general enumeration left) and once for the rest
        const bool fast_group = d <= 2 * NG && V <= KEY_LIMIT;
        auto rounds = [&](auto any_slow) {
            const bool fast = decltype(any_slow)::value ? fast_group : true;
            int cur = -1;
            LaneKeys keys;
            int pv0 = -1, pv1 = -1;  // position of v in the lane's two tets
            if (fast) {
                keys = lane_keys(gt, (int)v);
                pv0 = tet_pos(gt.q0, (int)v);
                pv1 = tet_pos(gt.q1, (int)v);
            }
            while (true) {
                KeyRound r;
                if (fast)
                    r = next_key(keys);
                else
                    r.w = group_next(tets, vt_list, b, d, (int)v, cur, g, gt);
                const int w = r.w;
                if (w == INT_MAX) break;
                cur = w;
                if (w > v && dpos < 0) {
                    dpos = nrow;
                    put_row((int)v, -1);
                }
                put_row(w, w < v ? -2 : (int32_t)(up0 + nup));  // lower entries: k_lower_edge_ids
                if (w < v) continue;
                put_up(w, ip);
                if (fast) {
                    // tet 0 of lane g is list entry g, tet 1 entry g + NG: ascending
                    // tet order is every lane's tet 0 in lane order, then their tets 1
                    const bool in0 = r.e0 && !(r.h0 & 4);
                    const bool in1 = (r.e0 && (r.h0 & 4)) || r.e1;
                    const int p0 = r.h0 & 3, p1 = (r.e1 ? r.h1 : r.h0) & 3;
                    const uint64_t b0 = (__ballot(in0) >> gbase) & ((uint64_t(1) << NG) - 1);
                    const uint64_t b1 = (__ballot(in1) >> gbase) & ((uint64_t(1) << NG) - 1);
                    const int n0 = __popcll(b0);
                    if (in0) {
                        const int slot = gt.t0 * 6 + local_edge(min(pv0, p0), max(pv0, p0));
                        et_inc[ip + __popcll(b0 & below)] = slot;
                    }
                    if (in1) {
                        const int slot = gt.t1 * 6 + local_edge(min(pv1, p1), max(pv1, p1));
                        et_inc[ip + n0 + __popcll(b1 & below)] = slot;
                    }
                    ip += n0 + __popcll(b1);
                    continue;
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
                    }
                    ip += __popcll(ball);
                }
            }
        };
        if (__ballot(!fast_group) == 0)
            rounds(std::false_type{});
        else
            rounds(std::true_type{});
        if (dpos < 0) {
            dpos = nrow;
            put_row((int)v, -1);
        }
        const int rrow = nrow & (NG - 1), rup = nup & (NG - 1);  // entries not stored yet
        if (g < rrow) {
            col[row0 + nrow - rrow + g] = pcol;
            nz_edge[row0 + nrow - rrow + g] = pnz;
        }
        if (g < rup) {
            const int64_t e = up0 + nup - rup + g;
            reinterpret_cast<int2*>(edges)[e] = make_int2((int)v, phi);
            et_ptr[e] = pinc;
        }
        if (g == 0) diag_pos[v] = (int32_t)(row0 + dpos);
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) et_ptr[up_ptr[V]] = inc_ptr[V];
}

// Entries (v, w) with w < v belong to edge (w, v), found among w's upper
// edges (sorted by hi).  One LG-lane group per row, a lane per entry (a row's
// lower entries come first, about half of it); lists of up to 8 upper edges
// are read at once and scanned, longer ones binary searched.
constexpr int LG = 8;

__global__ void k_lower_edge_ids(int64_t V, const int64_t* __restrict__ row_ptr, const int32_t* __restrict__ col,
                                 const int64_t* __restrict__ up_ptr, const int32_t* __restrict__ edges,
                                 int32_t* __restrict__ nz_edge, unsigned* __restrict__ err) {
    const int g = threadIdx.x & (LG - 1);
    GROUP_FRONT_LOOP(v, V, LG) {
        const int64_t k1 = row_ptr[v + 1];
        for (int64_t k = row_ptr[v] + g; k < k1; k += LG) {
            const int w = col[k];
            if (w >= v) break;
            const int64_t lo = up_ptr[w], n = up_ptr[w + 1] - lo;
            int64_t found = -1;
            if (n <= 8) {
                int h[8];
#pragma unroll
                for (int u = 0; u < 8; ++u) h[u] = u < n ? edges[2 * (lo + u) + 1] : -1;
#pragma unroll
                for (int u = 0; u < 8; ++u) found = h[u] == v ? lo + u : found;
            } else {
                int64_t a = lo, b = lo + n - 1;
                while (a <= b) {
                    const int64_t mid = (a + b) >> 1;
                    const int hv = edges[2 * mid + 1];
                    if (hv == v) {
                        found = mid;
                        break;
                    }
                    if (hv < v)
                        a = mid + 1;
                    else
                        b = mid - 1;
                }
            }
            if (found < 0) atomicOr(err, 8u);
            nz_edge[k] = (int32_t)found;
        }
    }
}

// Faces: a face (a, b, x), a < b < x, is counted on its lowest edge (a, b),
// whose incidence list holds every tet of the face.  One lane per edge: the
// ring of tets around (a, b) (up to RING of them in registers, longer rings
// read again from memory) gives each tet's two other vertices; the face
// (a, b, x) with x > b is held by the ring tets that contain x -- one on the
// boundary, two inside, more in an invalid mesh.  Its smallest tet counts it
// once, and a boundary face sets, in its tet's byte, the bit of the local
// vertex opposite it (an atomic OR on the byte's 32-bit word).
constexpr int RING = 8;
constexpr int COUNT_SPREAD = 64;

// the two local vertices off local edge le (the edge opposite it)
__device__ __forceinline__ void off_edge(int le, int* c1, int* c2) {
    *c1 = le == 0 ? 2 : (le <= 2 ? 1 : 0);
    *c2 = (le <= 1 || le == 3) ? 3 : ((le == 2 || le == 4) ? 2 : 1);
}

struct FaceTally {
    unsigned long long owned = 0, bnd = 0;
    __device__ __forceinline__ void add(int t, int opposite, int cnt, int first, uint32_t* bface_words,
                                        unsigned* err) {
        if (cnt > 2) atomicOr(err, 16u);
        owned += first == t;
        if (cnt == 1) {
            ++bnd;
            atomicOr(bface_words + (t >> 2), 1u << (8 * (t & 3) + opposite));
        }
    }
};

__global__ void k_edge_faces(int64_t E, const int32_t* __restrict__ edges, const int64_t* __restrict__ et_ptr,
                             const int32_t* __restrict__ et_inc, const int4* __restrict__ tets,
                             uint32_t* __restrict__ bface_words, unsigned long long* __restrict__ counts,
                             unsigned* __restrict__ err) {
    __shared__ unsigned long long lds[BLOCK / 64];
    FaceTally tally;
    RANGE_LOOP(e, E) {
        const int b = edges[2 * e + 1];
        const int64_t i0 = et_ptr[e];
        const int m = (int)(et_ptr[e + 1] - i0);
        if (m <= RING) {
            int u[RING], x1[RING], x2[RING], o1[RING], o2[RING];
#pragma unroll
            for (int r = 0; r < RING; ++r) {
                const int sl = r < m ? et_inc[i0 + r] : -1;
                int c1, c2;
                off_edge(sl >= 0 ? sl % 6 : 0, &c1, &c2);
                u[r] = sl >= 0 ? sl / 6 : -1;
                const int4 q = sl >= 0 ? tets[u[r]] : make_int4(-1, -1, -1, -1);
                x1[r] = vget(q, c1);  // face (a, b, x1) is opposite c2
                x2[r] = vget(q, c2);
                o1[r] = c2;
                o2[r] = c1;
            }
#pragma unroll
            for (int r = 0; r < RING; ++r) {
#pragma unroll
                for (int j = 0; j < 2; ++j) {
                    const int x = j ? x2[r] : x1[r];
                    if (x > b) {
                        int cnt = 0, first = INT_MAX;
#pragma unroll
                        for (int r2 = 0; r2 < RING; ++r2) {
                            const bool has = x1[r2] == x || x2[r2] == x;
                            cnt += has;
                            first = has ? min(first, u[r2]) : first;
                        }
                        tally.add(u[r], j ? o2[r] : o1[r], cnt, first, bface_words, err);
                    }
                }
            }
        } else {
            for (int r = 0; r < m; ++r) {
                const int sl = et_inc[i0 + r];
                int c1, c2;
                off_edge(sl % 6, &c1, &c2);
                const int4 q = tets[sl / 6];
                for (int j = 0; j < 2; ++j) {
                    const int x = vget(q, j ? c2 : c1);
                    if (x <= b) continue;
                    int cnt = 0, first = INT_MAX;
                    for (int r2 = 0; r2 < m; ++r2) {
                        const int s2 = et_inc[i0 + r2];
                        int d1, d2;
                        off_edge(s2 % 6, &d1, &d2);
                        const int4 q2 = tets[s2 / 6];
                        const bool has = vget(q2, d1) == x || vget(q2, d2) == x;
                        cnt += has;
                        first = has ? min(first, s2 / 6) : first;
                    }
                    tally.add(sl / 6, j ? c1 : c2, cnt, first, bface_words, err);
                }
            }
        }
    }
    // block totals into COUNT_SPREAD counters per sum (summed on the host):
    // thousands of blocks adding to one address would wait on each other
    const unsigned long long owned = block_sum(tally.owned, lds);
    const unsigned long long bnd = block_sum(tally.bnd, lds);
    if (threadIdx.x == 0) {
        const int slot = blockIdx.x % COUNT_SPREAD;
        if (owned) atomicAdd(&counts[slot], owned);
        if (bnd) atomicAdd(&counts[COUNT_SPREAD + slot], bnd);
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
    hipLaunchKernelGGL(k_vt_sort, dim3(grid_xcd(V, BLOCK / SG)), dim3(BLOCK), 0, s, m->vt_ptr.p, m->vt_list.p, V);
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
    m->col.alloc(ctx, nnz);
    m->nz_edge.alloc(ctx, nnz);
    m->diag_pos.alloc(ctx, V);
    hipLaunchKernelGGL(k_nbr_fill, dim3(grid_for(NG * V)), dim3(BLOCK), 0, s, tq, m->vt_ptr.p, m->vt_list.p, V,
                       m->up_ptr.p, row_ptr64.p, inc_ptr.p, m->edges.p, m->et_ptr.p, m->et_inc.p, m->col.p,
                       m->nz_edge.p, m->diag_pos.p);
    // [0, COUNT_SPREAD) owned faces, then as many boundary faces, then the
    // error bits (low word): one read-back for all of them
    DBuf<unsigned long long> fc;
    fc.alloc(ctx, 2 * COUNT_SPREAD + 1);
    fc.zero();
    unsigned* err2 = reinterpret_cast<unsigned*>(fc.p + 2 * COUNT_SPREAD);
    hipLaunchKernelGGL(k_lower_edge_ids, dim3(grid_xcd(V, BLOCK / LG)), dim3(BLOCK), 0, s, V, row_ptr64.p, m->col.p,
                       m->up_ptr.p, m->edges.p, m->nz_edge.p, err2);
    HIP_CHECK(hipGetLastError());
    m->row_ptr.alloc(ctx, V + 1);
    copy_i64_to_i32(ctx, row_ptr64.p, m->row_ptr.p, V + 1);

    // faces; the boundary bytes are set by atomic ORs on their 32-bit words, so
    // the buffer is allocated and cleared in whole words
    m->tet_bface.alloc(ctx, (T + 3) / 4 * 4);
    m->tet_bface.zero();
    hipLaunchKernelGGL(k_edge_faces, dim3(grid_xcd(E)), dim3(BLOCK), 0, s, E, m->edges.p, m->et_ptr.p,
                       m->et_inc.p, tq, reinterpret_cast<uint32_t*>(m->tet_bface.p), fc.p, err2);
    HIP_CHECK(hipGetLastError());
    unsigned long long hc[2 * COUNT_SPREAD + 1];
    std::memcpy(hc, ctx->readback(fc.p, sizeof(hc)), sizeof(hc));
    m->F = m->Fb = 0;
    for (int k = 0; k < COUNT_SPREAD; ++k) {
        m->F += (int64_t)hc[k];
        m->Fb += (int64_t)hc[COUNT_SPREAD + k];
    }
    const unsigned e1 = static_cast<unsigned>(hc[2 * COUNT_SPREAD] & 0xffffffffu);
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
