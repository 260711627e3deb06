// The paper's own unknowns (Section 2.3, eq. 11-13): temperature on the
// tets (Voronoi vertices), flux through the triangles (duals of the Voronoi
// edges).  The (1,1) block (1/kappa) * of eq. 11 is diagonal, so the fluxes
// are eliminated and the Schur complement on the tets is solved: every face
// f between tets t1 and t2 adds W_f (T_t1 - T_t2) to both balances, a
// Dirichlet face W_f (T_t - T0_f), with W_f = kappa_f / *_f and
// *_f = max(h_f / |f|, limiter) (Section 3.1's limiter), h_f the signed
// length of the Voronoi edge through f (to the face's circumcentre on the
// boundary).  Insulated and cracked faces carry no flux (eq. 13).
//
// Faces are numbered by owner tet (the lowest tet holding them), then by the
// local index of the opposite vertex.  A boundary face is Dirichlet when its
// three vertices carry Dirichlet data, with T0 their mean, and Neumann (eq. 13:
// its flux is given) when they carry Neumann data, the vertices' values being
// outward flux densities: its outward flux f0 |f|, f0 their mean, moves to the
// right-hand side.  Tets in parts
// joined to no Dirichlet face over conducting faces are pinned to 0.  The
// system is returned as a mesh whose rows are the tets, so the solver applies
// to it; its solver copy is built for the difference-form product (the
// limited weights are many orders above the rest) and carries the block-Jacobi
// inverse over the clusters of tets that limited faces join.
//
// Compiled without floating-point contraction: the Voronoi-edge end points
// enter the crack predicate, which decides integers.
#include <climits>
#include <cmath>
#include <cstring>
#include <vector>

#include "geom.h"
#include "solver.h"
#include "uf.h"
#include "wave_atomic.h"

void build_sell_copy(dec_ctx* ctx, int64_t V, int64_t nnz, const int32_t* ptr, const int32_t* col, const double* v64,
                     const float* v32, SellMatrix& S);

namespace {

// The tet across each face of every tet (-1 on the boundary), from the edge
// rings of the vertex topology: a face (a, b, x), a < b < x, lies in the ring
// of tets around its lowest edge (a, b), and its tets are the ring tets that
// hold x.  One lane per edge (up to RING ring tets in registers, longer rings
// read again from memory); each tet's face is written by the lane of that
// face's lowest edge, so every entry is written once.
constexpr int RING = 8;

// the two local vertices off local edge le (the edge opposite it)
__device__ __forceinline__ void off_edge(int le, int* c1, int* c2) {
    *c1 = le == 0 ? 2 : (le <= 2 ? 1 : 0);
    *c2 = (le <= 1 || le == 3) ? 3 : ((le == 2 || le == 4) ? 2 : 1);
}

__global__ void k_dual_nbr(int64_t E, const int32_t* __restrict__ edges, const int64_t* __restrict__ et_ptr,
                           const int32_t* __restrict__ et_inc, const int4* __restrict__ tets,
                           int32_t* __restrict__ nbr, unsigned* __restrict__ err) {
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
                        int cnt = 0, other = -1;
#pragma unroll
                        for (int r2 = 0; r2 < RING; ++r2) {
                            const bool has = x1[r2] == x || x2[r2] == x;
                            cnt += has;
                            other = has && r2 != r ? u[r2] : other;
                        }
                        if (cnt > 2) atomicOr(err, 1u);
                        nbr[4 * (int64_t)u[r] + (j ? o2[r] : o1[r])] = other;
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
                    int cnt = 0, other = -1;
                    for (int r2 = 0; r2 < m; ++r2) {
                        const int s2 = et_inc[i0 + r2];
                        int d1, d2;
                        off_edge(s2 % 6, &d1, &d2);
                        const int4 q2 = tets[s2 / 6];
                        const bool has = vget(q2, d1) == x || vget(q2, d2) == x;
                        cnt += has;
                        other = has && r2 != r ? s2 / 6 : other;
                    }
                    if (cnt > 2) atomicOr(err, 1u);
                    nbr[4 * (int64_t)(sl / 6) + (j ? c1 : c2)] = other;
                }
            }
        }
    }
}

// owned[t]: the faces of t that no lower tet holds
__global__ void k_dual_owned(int64_t T, const int32_t* __restrict__ nbr, int32_t* __restrict__ owned) {
    GRID_STRIDE_LOOP(t, T) {
        const int4 n = reinterpret_cast<const int4*>(nbr)[t];
        owned[t] = (n.x < 0 || n.x > t) + (n.y < 0 || n.y > t) + (n.z < 0 || n.z > t) + (n.w < 0 || n.w > t);
    }
}

// Face records in owner order; tet_face[4 t + k] = face of local face k of tet t.
__global__ void k_dual_fill(int64_t T, const int4* __restrict__ tets, const int32_t* __restrict__ nbr,
                            const int64_t* __restrict__ face_ptr, int32_t* __restrict__ t1, int32_t* __restrict__ k1,
                            int32_t* __restrict__ t2, int32_t* __restrict__ k2, int32_t* __restrict__ tet_face) {
    GRID_STRIDE_LOOP(t, T) {
        const int4 q = tets[t];
        int64_t f = face_ptr[t];
        for (int k = 0; k < 4; ++k) {
            const int o = nbr[4 * t + k];
            if (o >= 0 && o < (int)t) continue;  // owned by the lower tet o
            t1[f] = (int32_t)t;
            k1[f] = k;
            t2[f] = o;
            int ko = -1;
            if (o >= 0) {
                // the vertex of o that is not on the face
                const int4 p = tets[o];
                const int a = vget(q, face_local_vertex(k, 0)), b = vget(q, face_local_vertex(k, 1));
                const int c = vget(q, face_local_vertex(k, 2));
                for (int j = 0; j < 4; ++j) {
                    const int v = vget(p, j);
                    if (v != a && v != b && v != c) ko = j;
                }
                if (ko >= 0) tet_face[4 * (int64_t)o + ko] = (int32_t)f;
            }
            k2[f] = ko;
            tet_face[4 * t + k] = (int32_t)f;
            ++f;
        }
    }
}

__global__ void k_dual_circ(int64_t T, const int4* __restrict__ tets, const double* __restrict__ xyz,
                            double* __restrict__ ct) {
    GRID_STRIDE_LOOP(t, T) {
        const int4 q = tets[t];
        const d3 c = tet_circumcentre(load3(xyz + 3 * (int64_t)q.x), load3(xyz + 3 * (int64_t)q.y),
                                      load3(xyz + 3 * (int64_t)q.z), load3(xyz + 3 * (int64_t)q.w));
        ct[3 * t] = c.x;
        ct[3 * t + 1] = c.y;
        ct[3 * t + 2] = c.z;
    }
}

// Per face: the limited Hodge entry, the cut flag (Voronoi edge against the
// discs), boundary kind (0 interior, 1 Dirichlet, 2 insulated, 3 Neumann), the
// Dirichlet value (T0) or the prescribed outward flux of a Neumann face (in
// T0 as well), side and the weight W_f (0 on insulated and Neumann faces).
__global__ void k_dual_faces(int64_t F, const int4* __restrict__ tets, const double* __restrict__ xyz,
                             const double* __restrict__ ct, const int32_t* __restrict__ t1,
                             const int32_t* __restrict__ k1, const int32_t* __restrict__ t2, double limiter,
                             int32_t n_discs, const double* __restrict__ discs, const double* __restrict__ kappa,
                             const int8_t* __restrict__ bc_type, const double* __restrict__ bc_value,
                             const int8_t* __restrict__ side, double* __restrict__ W, double* __restrict__ T0,
                             int8_t* __restrict__ kind, int8_t* __restrict__ fside, uint8_t* __restrict__ cut,
                             uint8_t* __restrict__ limited, unsigned long long* __restrict__ counts) {
    __shared__ int lds[BLOCK / 64];
    int nlim = 0, nbnd = 0;
    RANGE_LOOP(f, F) {
        const int t = t1[f], k = k1[f], o = t2[f];
        const int4 q = tets[t];
        const int va = vget(q, face_local_vertex(k, 0)), vb = vget(q, face_local_vertex(k, 1));
        const int vc = vget(q, face_local_vertex(k, 2));
        const d3 a = load3(xyz + 3 * (int64_t)va), b = load3(xyz + 3 * (int64_t)vb), c = load3(xyz + 3 * (int64_t)vc);
        const d3 opp = load3(xyz + 3 * (int64_t)vget(q, k));
        const d3 n = cross(sub(b, a), sub(c, a));
        const double nn = sqrt(dot(n, n));
        const double sgn = dot(sub(opp, a), n) > 0.0 ? -1.0 : 1.0;  // out of t1
        const double s = sgn / nn;
        const d3 unit = {n.x * s, n.y * s, n.z * s};
        const double area = 0.5 * nn;
        const d3 c1 = load3(ct + 3 * (int64_t)t);
        const d3 far = o >= 0 ? load3(ct + 3 * (int64_t)o) : tri_circumcentre(a, b, c);
        const double h = dot(sub(far, c1), unit);
        const double star = fmax(h / area, limiter);
        const bool lim = !(h / area > limiter);
        nlim += lim;
        // cracks: the Voronoi edge c1 -> far crosses a disc (the predicate of the vertex path)
        uint8_t hit = 0;
        for (int32_t i = 0; i < n_discs && !hit; ++i) {
            const double* d = discs + 7 * (int64_t)i;
            const double cx = d[0], cy = d[1], cz = d[2], nx = d[3], ny = d[4], nz = d[5], r = d[6];
            const double s0 = ((c1.x - cx) * nx + (c1.y - cy) * ny) + (c1.z - cz) * nz;
            const double s1 = ((far.x - cx) * nx + (far.y - cy) * ny) + (far.z - cz) * nz;
            if ((s0 < 0.0) == (s1 < 0.0)) continue;
            const double tt = s0 / (s0 - s1);
            const double qx = c1.x + tt * (far.x - c1.x);
            const double qy = c1.y + tt * (far.y - c1.y);
            const double qz = c1.z + tt * (far.z - c1.z);
            const double d2 = ((qx - cx) * (qx - cx) + (qy - cy) * (qy - cy)) + (qz - cz) * (qz - cz);
            if (d2 <= r * r) hit = 1;
        }
        int8_t kd = 0, sd = 0;
        double t0 = 0.0;
        if (o < 0) {
            ++nbnd;
            kd = 2;
            if (bc_type[va] == 1 && bc_type[vb] == 1 && bc_type[vc] == 1) {
                kd = 1;
                t0 = ((bc_value[va] + bc_value[vb]) + bc_value[vc]) / 3.0;
                if (side) {
                    const int8_t sa = side[va];
                    if ((sa == 1 || sa == 2) && side[vb] == sa && side[vc] == sa) sd = sa;
                }
            } else if (bc_type[va] == 2 && bc_type[vb] == 2 && bc_type[vc] == 2) {
                kd = 3;
                t0 = (((bc_value[va] + bc_value[vb]) + bc_value[vc]) / 3.0) * area;
            }
        }
        const double kap = hit ? 0.0 : (kappa ? kappa[f] : 1.0);
        W[f] = kd >= 2 ? 0.0 : kap * (1.0 / star);
        T0[f] = t0;
        kind[f] = kd;
        fside[f] = sd;
        cut[f] = hit;
        limited[f] = lim;
    }
    const int total = block_sum(nlim, lds);
    if (threadIdx.x == 0 && total) atomicAdd(counts, (unsigned long long)total);
    const int bnd = block_sum(nbnd, lds);
    if (threadIdx.x == 0 && bnd) atomicAdd(counts + 3, (unsigned long long)bnd);
}

__global__ void k_dual_uf_init(int64_t T, int32_t* __restrict__ parent) {
    GRID_STRIDE_LOOP(t, T) parent[t] = (int32_t)t;
}

__global__ void k_dual_uf_hook(int64_t F, const int32_t* __restrict__ t1, const int32_t* __restrict__ t2,
                               const double* __restrict__ W, int32_t* parent) {
    GRID_STRIDE_LOOP(f, F) {
        if (t2[f] < 0 || W[f] == 0.0) continue;
        uf_union(parent, t1[f], t2[f]);
    }
}

__global__ void k_dual_uf_anchor(int64_t F, const int32_t* __restrict__ t1, const int8_t* __restrict__ kind,
                                 const double* __restrict__ W, int32_t* parent, uint32_t* __restrict__ anchored) {
    GRID_STRIDE_LOOP(f, F) {
        if (kind[f] == 1 && W[f] != 0.0) anchored[uf_find(parent, t1[f])] = 1u;
    }
}

__global__ void k_dual_pin(int64_t T, int32_t* parent, const uint32_t* __restrict__ anchored,
                           uint8_t* __restrict__ fixed, int32_t* __restrict__ row_len,
                           const int32_t* __restrict__ nbr, unsigned long long* __restrict__ n_pinned) {
    unsigned long long local = 0;
    GRID_STRIDE_LOOP(t, T) {
        const bool pin = !anchored[uf_find(parent, (int32_t)t)];
        fixed[t] = pin ? 2 : 0;
        local += pin;
        int len = 1;
        for (int k = 0; k < 4; ++k) len += nbr[4 * t + k] >= 0;
        row_len[t] = len;
    }
    if (local) atomicAdd(n_pinned, local);
}

// Row t: the diagonal and the tets across its interior faces, ascending;
// off-diagonal -W_f, diagonal the sum of W over its conducting faces in local
// face order, right-hand side the Dirichlet faces' W_f T0_f less the Neumann
// faces' outward flux (in local face order); pinned rows
// become unit rows with a zero right-hand side.  The row excess (diagonal
// minus the off-diagonal weights) is the sum of the Dirichlet faces' W_f, 1 on
// pinned rows: the solver's product takes the difference form with it, so
// the limited weights (up to kappa / limiter) never cancel against the rest.
__global__ void k_dual_rows(int64_t T, const int32_t* __restrict__ nbr, const int32_t* __restrict__ tet_face,
                            const double* __restrict__ W, const double* __restrict__ T0,
                            const int8_t* __restrict__ kind, const uint8_t* __restrict__ fixed,
                            const int32_t* __restrict__ row_ptr, int32_t* __restrict__ col,
                            int32_t* __restrict__ diag_pos, double* __restrict__ v64, float* __restrict__ v32,
                            double* __restrict__ rhs, double* __restrict__ invd64, float* __restrict__ invd32,
                            double* __restrict__ ex64, float* __restrict__ ex32, int32_t* __restrict__ o_col,
                            double* __restrict__ o64, float* __restrict__ o32) {
    GRID_STRIDE_LOOP(t, T) {
        const bool pin = fixed[t] != 0;
        int cc[5], ff[5], n = 0;
        cc[n] = (int)t;
        ff[n++] = -1;
        double diag = 0.0, b = 0.0, ex = 0.0;
        for (int k = 0; k < 4; ++k) {
            const int f = tet_face[4 * t + k];
            if (kind[f] <= 1) diag += W[f];
            if (kind[f] == 1) {
                b += W[f] * T0[f];
                ex += W[f];
            }
            if (kind[f] == 3) b -= T0[f];
            const int o = nbr[4 * t + k];
            if (o >= 0) {
                cc[n] = o;
                ff[n++] = f;
            }
        }
        for (int i = 1; i < n; ++i) {  // ascending columns
            int j = i;
            while (j > 0 && cc[j - 1] > cc[j]) {
                const int tc = cc[j], tf = ff[j];
                cc[j] = cc[j - 1];
                ff[j] = ff[j - 1];
                cc[j - 1] = tc;
                ff[j - 1] = tf;
                --j;
            }
        }
        const int32_t p = row_ptr[t];
        int32_t q = p - (int32_t)t;  // the row in the off-diagonal copy (one diagonal per row before it)
        for (int i = 0; i < n; ++i) {
            const double v = ff[i] < 0 ? (pin ? 1.0 : diag) : (pin ? 0.0 : -W[ff[i]]);
            col[p + i] = cc[i];
            v64[p + i] = v;
            v32[p + i] = static_cast<float>(v);
            if (ff[i] < 0) {
                diag_pos[t] = p + i;
                invd64[t] = 1.0 / v;
                invd32[t] = 1.0f / static_cast<float>(v);
            } else {
                o_col[q] = cc[i];
                o64[q] = v;
                o32[q] = static_cast<float>(v);
                ++q;
            }
        }
        rhs[t] = pin ? 0.0 : b;
        ex64[t] = pin ? 1.0 : ex;
        ex32[t] = pin ? 1.0f : static_cast<float>(ex);
    }
}

// ---- block Jacobi over the clusters of tets joined by limited faces
// Limited faces carry kappa / limiter, many orders above the rest, so the tets
// they join move together; a preconditioner that inverts each such cluster
// exactly leaves CG the well-conditioned coupling between clusters.  Clusters
// of more than MAX_BLOCK tets are left to Jacobi (one entry per row).
constexpr int MAX_BLOCK = 16;

__global__ void k_dual_cluster_hook(int64_t F, const int32_t* __restrict__ t1, const int32_t* __restrict__ t2,
                                    const double* __restrict__ W, const uint8_t* __restrict__ limited,
                                    int32_t* parent) {
    GRID_STRIDE_LOOP(f, F) {
        if (t2[f] < 0 || W[f] == 0.0 || !limited[f]) continue;
        uf_union(parent, t1[f], t2[f]);
    }
}

// root (smallest tet) of every tet's cluster, and the cluster sizes at the roots
__global__ void k_dual_cluster_size(int64_t T, int32_t* parent, int32_t* __restrict__ root,
                                    int32_t* __restrict__ size) {
    GRID_STRIDE_LOOP(t, T) {
        const int32_t r = uf_find(parent, (int32_t)t);
        root[t] = r;
        (void)wave_claim(size, r);  // a cluster's tets are mostly neighbours
    }
}

__device__ __forceinline__ bool is_block(int s) { return s >= 2 && s <= MAX_BLOCK; }

// Row lengths of the block inverse; member slots per block cluster (at its
// root); the number of block clusters and the largest, reduced per workgroup
// before one atomic each (one per cluster would serialise on two words).
__global__ __launch_bounds__(BLOCK) void k_dual_block_len(int64_t T, const int32_t* __restrict__ root,
                                                          const int32_t* __restrict__ size, int32_t* __restrict__ len,
                                                          int32_t* __restrict__ slots,
                                                          unsigned long long* __restrict__ counts) {
    __shared__ unsigned long long lds[BLOCK / 64];
    __shared__ int wmax[BLOCK / 64];
    unsigned long long leads = 0;
    int smax = 0;
    GRID_STRIDE_LOOP(t, T) {
        const int s = size[root[t]];
        const bool lead = is_block(s) && root[t] == (int32_t)t;
        len[t] = is_block(s) ? s : 1;
        slots[t] = lead ? s : 0;
        if (lead) {
            ++leads;
            smax = max(smax, s);
        }
    }
    const unsigned long long total = block_sum(leads, lds);
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) smax = max(smax, __shfl_xor(smax, off, 64));
    if ((threadIdx.x & 63) == 0) wmax[threadIdx.x >> 6] = smax;
    __syncthreads();
    if (threadIdx.x == 0) {
        int m = 0;
        for (int w = 0; w < BLOCK / 64; ++w) m = max(m, wmax[w]);
        if (total) atomicAdd(counts, total);
        if (m) atomicMax(counts + 1, (unsigned long long)m);
    }
}

__global__ void k_dual_block_members(int64_t T, const int32_t* __restrict__ root, const int32_t* __restrict__ size,
                                     const int64_t* __restrict__ slot_off, int32_t* __restrict__ fill,
                                     int32_t* __restrict__ members) {
    GRID_STRIDE_LOOP(t, T) {
        const int32_t r = root[t];
        if (!is_block(size[r])) continue;
        const int k = wave_claim(fill, r);
        members[slot_off[r] + k] = (int32_t)t;
    }
}

// Rows of tets outside the block clusters: 1 / a_tt.
__global__ void k_dual_block_single(int64_t T, const int32_t* __restrict__ root, const int32_t* __restrict__ size,
                                    const int32_t* __restrict__ diag_pos, const double* __restrict__ v64,
                                    const int32_t* __restrict__ m_ptr, int32_t* __restrict__ m_col,
                                    double* __restrict__ m64, float* __restrict__ m32) {
    GRID_STRIDE_LOOP(t, T) {
        if (is_block(size[root[t]])) continue;
        const int32_t p = m_ptr[t];
        const double inv = 1.0 / v64[diag_pos[t]];
        m_col[p] = (int32_t)t;
        m64[p] = inv;
        m32[p] = static_cast<float>(inv);
    }
}

// One thread per block cluster: gather A restricted to the cluster (members
// ascending), Cholesky A = L L^T, then column b of the inverse from
// L y = e_b, L^T x = y; its entries a >= b go to (a, b) and (b, a).  A pivot
// that is not positive (not expected: the block of an SPD matrix) leaves the
// cluster's rows diagonal (Jacobi).  N bounds the cluster size the launch
// handles (clusters of other sizes are skipped): every loop runs to N with
// the cluster's own size s as a guard, so for N = 8 the matrix stays in
// registers; the operations and their order are those of a loop to s.
template <int N>
__global__ void k_dual_block_inv(int64_t T, int lo, const int32_t* __restrict__ root, const int32_t* __restrict__ size,
                                 const int64_t* __restrict__ slot_off, const int32_t* __restrict__ members,
                                 const int32_t* __restrict__ row_ptr, const int32_t* __restrict__ col,
                                 const double* __restrict__ v64, const int32_t* __restrict__ m_ptr,
                                 int32_t* __restrict__ m_col, double* __restrict__ m64, float* __restrict__ m32) {
    GRID_STRIDE_LOOP(t, T) {
        if (root[t] != (int32_t)t) continue;
        const int s = size[t];
        if (!is_block(s) || s < lo || s > N) continue;
        int mem[N];
#pragma unroll
        for (int a = 0; a < N; ++a) mem[a] = a < s ? members[slot_off[t] + a] : INT_MAX;
#pragma unroll
        for (int a = 1; a < N; ++a)  // insertion sort; the INT_MAX tail stays in place
#pragma unroll
            for (int b = a; b > 0; --b)
                if (mem[b - 1] > mem[b]) {
                    const int x = mem[b];
                    mem[b] = mem[b - 1];
                    mem[b - 1] = x;
                }
        double A[N][N], dg[N], y[N];
#pragma unroll
        for (int a = 0; a < N; ++a)
#pragma unroll
            for (int b = 0; b < N; ++b) A[a][b] = 0.0;
#pragma unroll
        for (int a = 0; a < N; ++a) {
            if (a >= s) continue;
            for (int32_t e = row_ptr[mem[a]]; e < row_ptr[mem[a] + 1]; ++e) {
                const int c = col[e];
                const double v = v64[e];
#pragma unroll
                for (int b = 0; b < N; ++b)
                    if (mem[b] == c) A[a][b] = v;
            }
        }
#pragma unroll
        for (int a = 0; a < N; ++a) dg[a] = A[a][a];
        bool ok = true;
#pragma unroll
        for (int j = 0; j < N; ++j) {
            if (j >= s || !ok) continue;
            double d = A[j][j];
#pragma unroll
            for (int k = 0; k < j; ++k) d -= A[j][k] * A[j][k];
            if (!(d > 0.0) || !isfinite(d)) {
                ok = false;
                continue;
            }
            A[j][j] = sqrt(d);
#pragma unroll
            for (int i = j + 1; i < N; ++i) {
                if (i >= s) continue;
                double v = A[i][j];
#pragma unroll
                for (int k = 0; k < j; ++k) v -= A[i][k] * A[j][k];
                A[i][j] = v / A[j][j];
            }
        }
#pragma unroll
        for (int a = 0; a < N; ++a) {
            if (a >= s) continue;
            const int32_t p = m_ptr[mem[a]];
#pragma unroll
            for (int b = 0; b < N; ++b)
                if (b < s) m_col[p + b] = mem[b];
        }
#pragma unroll
        for (int b = 0; b < N; ++b) {
            if (b >= s) continue;
            if (ok) {
#pragma unroll
                for (int i = 0; i < N; ++i) {  // L y = e_b
                    if (i >= s) continue;
                    double v = i == b ? 1.0 : 0.0;
#pragma unroll
                    for (int k = 0; k < i; ++k) v -= A[i][k] * y[k];
                    y[i] = v / A[i][i];
                }
#pragma unroll
                for (int i = N - 1; i >= 0; --i) {  // L^T x = y, in place
                    if (i >= s) continue;
                    double v = y[i];
#pragma unroll
                    for (int k = i + 1; k < N; ++k)
                        if (k < s) v -= A[k][i] * y[k];
                    y[i] = v / A[i][i];
                }
            } else {
#pragma unroll
                for (int i = 0; i < N; ++i) y[i] = i == b ? 1.0 / dg[b] : 0.0;
            }
#pragma unroll
            for (int a = 0; a < N; ++a) {  // the lower triangle, mirrored: M is exactly symmetric
                if (a < b || a >= s) continue;
                const int32_t pa = m_ptr[mem[a]] + b, pb = m_ptr[mem[b]] + a;
                m64[pa] = m64[pb] = y[a];
                m32[pa] = m32[pb] = static_cast<float>(y[a]);
            }
        }
    }
}

// Row pointer of the off-diagonal copy: row t starts after t diagonals fewer.
__global__ void k_offdiag_ptr(int64_t T, const int32_t* __restrict__ row_ptr, int32_t* __restrict__ o_ptr) {
    GRID_STRIDE_LOOP(t, T + 1) o_ptr[t] = row_ptr[t] - (int32_t)t;
}

// Flux of a tet solution: energy, Q_in, Q_out as per-block partials.
__global__ __launch_bounds__(BLOCK) void k_dual_flux(int64_t F, const int32_t* __restrict__ t1,
                                                     const int32_t* __restrict__ t2, const double* __restrict__ W,
                                                     const double* __restrict__ T0, const int8_t* __restrict__ kind,
                                                     const int8_t* __restrict__ side, const double* __restrict__ T,
                                                     double* __restrict__ partials) {
    __shared__ double lds[BLOCK / 64];
    double en = 0.0, qi = 0.0, qo = 0.0;
    RANGE_LOOP(f, F) {
        const int8_t kd = kind[f];
        if (kd >= 2) continue;  // insulated and Neumann faces (W = 0)
        const double w = W[f], ta = T[t1[f]];
        const double d = kd == 0 ? ta - T[t2[f]] : ta - T0[f];
        en += w * d * d;
        if (kd == 1 && side[f] == 1) qi += w * (T0[f] - ta);
        if (kd == 1 && side[f] == 2) qo += w * (ta - T0[f]);
    }
    const int G = gridDim.x;
    const double a = block_sum(en, lds);
    const double b = block_sum(qi, lds);
    const double c = block_sum(qo, lds);
    if (threadIdx.x == 0) {
        partials[blockIdx.x] = a;
        partials[G + blockIdx.x] = b;
        partials[2 * G + blockIdx.x] = c;
    }
}

__global__ void k_dual_flux_fold(int G, const double* __restrict__ partials, double* __restrict__ out) {
    __shared__ double lds[BLOCK / 64 + 1];
    const double a = reduce_bcast(partials, G, lds);
    const double b = reduce_bcast(partials + G, G, lds);
    const double c = reduce_bcast(partials + 2 * G, G, lds);
    if (threadIdx.x == 0) {
        out[0] = a;
        out[1] = b;
        out[2] = c;
    }
}

// A call for tet systems was given a mesh of vertex unknowns.
int not_dual(dec_ctx* ctx, const char* call) {
    ctx->last_error = std::string(call) + " takes a tet system from dec_dual_build";
    return DEC_ESTATE;
}

}  // namespace

extern "C" {

int dec_dual_build(dec_mesh* m, const double* kappa_face, int32_t n_cracks, const double* cracks,
                   const int8_t* bc_type, const double* bc_value, const int8_t* side, double limiter,
                   dec_mesh** dual_out, int64_t* n_pinned_out) {
    if (!m) return DEC_EINVAL;
    if (!dual_out || !bc_type || !bc_value) return null_argument(m->ctx, "dec_dual_build");
    *dual_out = nullptr;
    dec_ctx* ctx = m->ctx;
    dec_mesh* d = nullptr;
    try {
        DEC_REQUIRE(!m->dual, DEC_ESTATE, "dec_dual_build needs a mesh of vertex unknowns");
        DEC_REQUIRE(m->vt_ptr.p && m->vt_list.p && m->et_inc.p && m->edges.p && m->xyz.p && m->tets.p, DEC_ESTATE,
                    "dec_dual_build needs the topology of dec_build_topology");
        DEC_REQUIRE(n_cracks >= 0 && (n_cracks == 0 || cracks), DEC_EINVAL, "bad crack array");
        DEC_REQUIRE(5 * m->T < (int64_t(1) << 31), DEC_EINVAL, "too many tets for int32 row pointers");
        ctx->set_device();
        hipStream_t s = ctx->stream;
        const int64_t T = m->T, F = m->F;
        const int4* tq = reinterpret_cast<const int4*>(m->tets.p);
        d = new dec_mesh();
        d->ctx = ctx;
        d->owner = ctx;
        ctx->live_children += 1;
        d->dual = new DualData();
        DualData& D = *d->dual;
        d->V = T;
        d->F = F;

        DBuf<int32_t> nbr, owned, tet_face;
        DBuf<unsigned> err;
        nbr.alloc(ctx, 4 * T);
        owned.alloc(ctx, T);
        err.alloc(ctx, 1);
        err.zero();
        hipLaunchKernelGGL(k_dual_nbr, dim3(grid_xcd(m->E)), dim3(BLOCK), 0, s, m->E, m->edges.p, m->et_ptr.p,
                           m->et_inc.p, tq, nbr.p, err.p);
        hipLaunchKernelGGL(k_dual_owned, dim3(grid_for(T)), dim3(BLOCK), 0, s, T, nbr.p, owned.p);
        DBuf<int64_t> face_ptr;
        face_ptr.alloc(ctx, T + 1);
        const int64_t nf = scan_exclusive_i32_to_i64(ctx, owned.p, face_ptr.p, T, true);
        const unsigned e0 = *static_cast<unsigned*>(ctx->readback(err.p, sizeof(unsigned)));
        DEC_REQUIRE(e0 == 0, DEC_ETOPO, "face shared by more than two tets");
        DEC_REQUIRE(nf == F, DEC_ETOPO, "internal: face count mismatch");
        D.F = F;
        for (DBuf<int32_t>* b : {&D.t1, &D.k1, &D.t2, &D.k2}) b->alloc(ctx, F);
        tet_face.alloc(ctx, 4 * T);
        hipLaunchKernelGGL(k_dual_fill, dim3(grid_for(T)), dim3(BLOCK), 0, s, T, tq, nbr.p, face_ptr.p, D.t1.p,
                           D.k1.p, D.t2.p, D.k2.p, tet_face.p);
        DBuf<double> ct;
        ct.alloc(ctx, 3 * T);
        hipLaunchKernelGGL(k_dual_circ, dim3(grid_for(T)), dim3(BLOCK), 0, s, T, tq, m->xyz.p, ct.p);
        D.W.alloc(ctx, F);
        D.T0.alloc(ctx, F);
        D.kind.alloc(ctx, F);
        D.side.alloc(ctx, F);
        D.cut.alloc(ctx, F);
        D.limited.alloc(ctx, F);
        DBuf<unsigned long long> counts;  // limited faces, block clusters, largest block, boundary faces
        counts.alloc(ctx, 4);
        counts.zero();
        hipLaunchKernelGGL(k_dual_faces, dim3(grid_xcd(F)), dim3(BLOCK), 0, s, F, tq, m->xyz.p, ct.p, D.t1.p, D.k1.p,
                           D.t2.p, limiter > 0.0 ? limiter : 1e-8, n_cracks, cracks, kappa_face, bc_type, bc_value,
                           side, D.W.p, D.T0.p, D.kind.p, D.side.p, D.cut.p, D.limited.p, counts.p);
        HIP_CHECK(hipGetLastError());

        // parts cut off from every Dirichlet face
        DBuf<int32_t> parent, row_len;
        DBuf<uint32_t> anchored;
        DBuf<unsigned long long> npin;
        parent.alloc(ctx, T);
        row_len.alloc(ctx, T);
        anchored.alloc(ctx, T);
        anchored.zero();
        npin.alloc(ctx, 1);
        npin.zero();
        d->fixed.alloc(ctx, T);
        hipLaunchKernelGGL(k_dual_uf_init, dim3(grid_for(T)), dim3(BLOCK), 0, s, T, parent.p);
        hipLaunchKernelGGL(k_dual_uf_hook, dim3(grid_for(F)), dim3(BLOCK), 0, s, F, D.t1.p, D.t2.p, D.W.p, parent.p);
        hipLaunchKernelGGL(k_dual_uf_anchor, dim3(grid_for(F)), dim3(BLOCK), 0, s, F, D.t1.p, D.kind.p, D.W.p,
                           parent.p, anchored.p);
        hipLaunchKernelGGL(k_dual_pin, dim3(grid_for(T)), dim3(BLOCK), 0, s, T, parent.p, anchored.p, d->fixed.p,
                           row_len.p, nbr.p, npin.p);
        HIP_CHECK(hipGetLastError());

        // the tet operator (CSR, then its sliced-ELL copy)
        DBuf<int64_t> rp64;
        rp64.alloc(ctx, T + 1);
        const int64_t nnz = scan_exclusive_i32_to_i64(ctx, row_len.p, rp64.p, T, true);
        d->nnz = nnz;
        d->row_ptr.alloc(ctx, T + 1);
        copy_i64_to_i32(ctx, rp64.p, d->row_ptr.p, T + 1);
        d->col.alloc(ctx, nnz);
        d->diag_pos.alloc(ctx, T);
        d->val64.alloc(ctx, nnz);
        d->val32.alloc(ctx, nnz);
        d->rhs.alloc(ctx, T);
        d->invdiag64.alloc(ctx, T);
        d->invdiag32.alloc(ctx, T);
        d->bc_value.alloc(ctx, T);
        d->bc_value.zero();
        // the solver's copy holds the off-diagonal entries only: in the difference form the
        // diagonal multiplies x_i - x_i = 0
        DBuf<double> ex64, o64;
        DBuf<float> ex32, o32;
        DBuf<int32_t> o_ptr, o_col;
        ex64.alloc(ctx, T);
        ex32.alloc(ctx, T);
        o_ptr.alloc(ctx, T + 1);
        o_col.alloc(ctx, nnz - T > 0 ? nnz - T : 1);
        o64.alloc(ctx, nnz - T > 0 ? nnz - T : 1);
        o32.alloc(ctx, nnz - T > 0 ? nnz - T : 1);
        hipLaunchKernelGGL(k_dual_rows, dim3(grid_for(T)), dim3(BLOCK), 0, s, T, nbr.p, tet_face.p, D.W.p, D.T0.p,
                           D.kind.p, d->fixed.p, d->row_ptr.p, d->col.p, d->diag_pos.p, d->val64.p, d->val32.p,
                           d->rhs.p, d->invdiag64.p, d->invdiag32.p, ex64.p, ex32.p, o_col.p, o64.p, o32.p);
        hipLaunchKernelGGL(k_offdiag_ptr, dim3(grid_for(T + 1)), dim3(BLOCK), 0, s, T, d->row_ptr.p, o_ptr.p);
        HIP_CHECK(hipGetLastError());
        build_sell_copy(ctx, T, nnz - T, o_ptr.p, o_col.p, o64.p, o32.p, d->sell);
        d->sell.excess64 = std::move(ex64);
        d->sell.excess32 = std::move(ex32);

        // block Jacobi: clusters over limited faces, their inverses as a sparse matrix
        {
            DBuf<int32_t> cpar, root, size, len, slots, fill, members;
            for (DBuf<int32_t>* b : {&cpar, &root, &size, &len, &slots, &fill}) b->alloc(ctx, T);
            size.zero();
            fill.zero();
            hipLaunchKernelGGL(k_dual_uf_init, dim3(grid_for(T)), dim3(BLOCK), 0, s, T, cpar.p);
            hipLaunchKernelGGL(k_dual_cluster_hook, dim3(grid_for(F)), dim3(BLOCK), 0, s, F, D.t1.p, D.t2.p, D.W.p,
                               D.limited.p, cpar.p);
            hipLaunchKernelGGL(k_dual_cluster_size, dim3(grid_for(T)), dim3(BLOCK), 0, s, T, cpar.p, root.p, size.p);
            hipLaunchKernelGGL(k_dual_block_len, dim3(grid_for(T, BLOCK, 1024)), dim3(BLOCK), 0, s, T, root.p, size.p, len.p,
                               slots.p, counts.p + 1);
            DBuf<int64_t> mp64, slot_off;
            mp64.alloc(ctx, T + 1);
            slot_off.alloc(ctx, T + 1);
            const int64_t mnnz = scan_exclusive_i32_to_i64(ctx, len.p, mp64.p, T, true);
            const int64_t nmem = scan_exclusive_i32_to_i64(ctx, slots.p, slot_off.p, T, true);
            DEC_REQUIRE(mnnz < (int64_t(1) << 31), DEC_EINVAL, "block preconditioner too large for int32 offsets");
            members.alloc(ctx, nmem > 0 ? nmem : 1);
            DBuf<int32_t> m_ptr, m_col;
            DBuf<double> m64;
            DBuf<float> m32;
            m_ptr.alloc(ctx, T + 1);
            copy_i64_to_i32(ctx, mp64.p, m_ptr.p, T + 1);
            m_col.alloc(ctx, mnnz);
            m64.alloc(ctx, mnnz);
            m32.alloc(ctx, mnnz);
            hipLaunchKernelGGL(k_dual_block_members, dim3(grid_for(T)), dim3(BLOCK), 0, s, T, root.p, size.p,
                               slot_off.p, fill.p, members.p);
            hipLaunchKernelGGL(k_dual_block_single, dim3(grid_for(T)), dim3(BLOCK), 0, s, T, root.p, size.p,
                               d->diag_pos.p, d->val64.p, m_ptr.p, m_col.p, m64.p, m32.p);
            // clusters of up to 8 tets (the Kuhn cube's 6) in registers, larger ones apart
            hipLaunchKernelGGL(k_dual_block_inv<8>, dim3(grid_for(T)), dim3(BLOCK), 0, s, T, 2, root.p, size.p,
                               slot_off.p, members.p, d->row_ptr.p, d->col.p, d->val64.p, m_ptr.p, m_col.p, m64.p,
                               m32.p);
            hipLaunchKernelGGL(k_dual_block_inv<MAX_BLOCK>, dim3(grid_for(T)), dim3(BLOCK), 0, s, T, 9, root.p,
                               size.p, slot_off.p, members.p, d->row_ptr.p, d->col.p, d->val64.p, m_ptr.p, m_col.p,
                               m64.p, m32.p);
            HIP_CHECK(hipGetLastError());
            build_sell_copy(ctx, T, mnnz, m_ptr.p, m_col.p, m64.p, m32.p, d->blockinv);
            ctx->sync();  // the temporaries above are released on return
            unsigned long long h[4];
            std::memcpy(h, ctx->readback(counts.p, sizeof(h)), sizeof(h));
            D.n_limited = (int64_t)h[0];
            D.n_blocks = (int64_t)h[1];
            D.max_block = (int64_t)h[2];
            d->Fb = (int64_t)h[3];
        }
        d->n_pinned = (int64_t) * static_cast<unsigned long long*>(ctx->readback(npin.p, sizeof(unsigned long long)));
        d->assembled = true;
        d->bc_ready = true;
        if (n_pinned_out) *n_pinned_out = d->n_pinned;
    } catch (const DecError& e) {
        ctx->last_error = e.msg;
        if (d) {
            ctx->sync();
            delete d;
        }
        return e.code;
    }
    *dual_out = d;
    return DEC_OK;
}

int dec_dual_faces(const dec_mesh* d, int32_t* face_tets, int32_t* face_local, double* weight, uint8_t* cut) {
    if (!d) return DEC_EINVAL;
    if (!d->dual) return not_dual(d->ctx, "dec_dual_faces");
    try {
        const DualData& D = *d->dual;
        hipStream_t s = d->ctx->stream;
        const size_t F = (size_t)D.F;
        if (face_tets) {
            HIP_CHECK(hipMemcpy2DAsync(face_tets, 2 * sizeof(int32_t), D.t1.p, sizeof(int32_t), sizeof(int32_t), F,
                                       hipMemcpyDeviceToDevice, s));
            HIP_CHECK(hipMemcpy2DAsync(face_tets + 1, 2 * sizeof(int32_t), D.t2.p, sizeof(int32_t), sizeof(int32_t),
                                       F, hipMemcpyDeviceToDevice, s));
        }
        if (face_local) {
            HIP_CHECK(hipMemcpy2DAsync(face_local, 2 * sizeof(int32_t), D.k1.p, sizeof(int32_t), sizeof(int32_t), F,
                                       hipMemcpyDeviceToDevice, s));
            HIP_CHECK(hipMemcpy2DAsync(face_local + 1, 2 * sizeof(int32_t), D.k2.p, sizeof(int32_t), sizeof(int32_t),
                                       F, hipMemcpyDeviceToDevice, s));
        }
        if (weight) HIP_CHECK(hipMemcpyAsync(weight, D.W.p, F * sizeof(double), hipMemcpyDeviceToDevice, s));
        if (cut) HIP_CHECK(hipMemcpyAsync(cut, D.cut.p, F, hipMemcpyDeviceToDevice, s));
    } catch (const DecError& e) {
        d->ctx->last_error = e.msg;
        return e.code;
    }
    return DEC_OK;
}

int dec_dual_info(const dec_mesh* d, int64_t* n_faces, int64_t* n_limited, int64_t* n_blocks, int64_t* max_block) {
    if (!d) return DEC_EINVAL;
    if (!d->dual) return not_dual(d->ctx, "dec_dual_info");
    const DualData& D = *d->dual;
    if (n_faces) *n_faces = D.F;
    if (n_limited) *n_limited = D.n_limited;
    if (n_blocks) *n_blocks = D.n_blocks;
    if (max_block) *max_block = D.max_block;
    return DEC_OK;
}

int dec_dual_flux(dec_mesh* d, const double* T, double length, double area, double dT, double* k_eff, double* q_in,
                  double* q_out, double* energy) {
    if (!d) return DEC_EINVAL;
    if (!d->dual) return not_dual(d->ctx, "dec_dual_flux");
    if (!T) return null_argument(d->ctx, "dec_dual_flux");
    dec_ctx* ctx = d->ctx;
    try {
        DEC_REQUIRE(area > 0.0 && length > 0.0 && dT != 0.0, DEC_EINVAL, "bad length/area/dT");
        ctx->set_device();
        const DualData& D = *d->dual;
        const unsigned G = grid_xcd(D.F, BLOCK, 1024);
        DBuf<double> part, out;
        part.alloc(ctx, 3 * (int64_t)G);
        out.alloc(ctx, 3);
        hipLaunchKernelGGL(k_dual_flux, dim3(G), dim3(BLOCK), 0, ctx->stream, D.F, D.t1.p, D.t2.p, D.W.p, D.T0.p,
                           D.kind.p, D.side.p, T, part.p);
        hipLaunchKernelGGL(k_dual_flux_fold, dim3(1), dim3(BLOCK), 0, ctx->stream, (int)G, part.p, out.p);
        HIP_CHECK(hipGetLastError());
        double h[3];
        std::memcpy(h, ctx->readback(out.p, sizeof(h)), sizeof(h));
        if (energy) *energy = h[0];
        if (q_in) *q_in = h[1];
        if (q_out) *q_out = h[2];
        if (k_eff) *k_eff = h[0] * length / (area * dT * dT);
    } catch (const DecError& e) {
        ctx->last_error = e.msg;
        return e.code;
    }
    return DEC_OK;
}

}  // extern "C"
