/*
 * dec.h -- C ABI of the MI355X (gfx950) DEC steady-diffusion library.
 *
 * The library solves the steady conduction problem of the paper's
 * Section 2.1 (Fourier law f = -kappa grad T, conservation div f = 0,
 * Dirichlet T = T0, Neumann f.n = f0; eqs. 1-4) in its exterior-calculus
 * form (eqs. 5-8) with the temperature a primal 0-form on the vertices of a
 * tetrahedral mesh:
 *
 *     L T = b,   L = d0^T *1 d0,
 *
 * d0 the vertex-to-edge coboundary (Section 2.1, eqs. 9-10) and *1 the
 * diagonal circumcentric Hodge star on edges (dual-area / edge-length,
 * Section 2.1), scaled per edge by the conductivity of the dual face
 * (Section 2.1) and set to zero on edges a crack cuts (Section 2.5).
 *
 * Conventions, common to every call:
 *  - Every function returns an int status (DEC_OK = 0 or a negative
 *    DEC_E* code); dec_last_error() gives a message for the last failure on
 *    a context.  No C++ exception crosses this interface.
 *  - Array arguments are DEVICE pointers unless stated otherwise; scalar
 *    outputs (k_eff, counts, stats) are HOST pointers.
 *  - Work is ordered on the context's HIP stream.  Calls that return a
 *    count or a scalar to the host synchronise that stream before returning.
 *    Input buffers only need to stay valid until the call returns (the
 *    server, dec_server_submit, is the exception).
 *  - The caller owns every buffer it passes; the library copies what it
 *    keeps.  The library's own device memory comes from the alloc/free
 *    callbacks given to dec_create (hipMalloc/hipFree when they are NULL).
 *  - Indices are 0-based int32 (V, E and nnz below 2^31); offsets inside the
 *    library are int64 where counts may exceed that.
 *  - One context per host thread; a context and its meshes must not be used
 *    from two threads at once.
 */
#ifndef DEC_H
#define DEC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ---------------------------------------------------- */
#define DEC_OK 0
#define DEC_EINVAL (-1)      /* bad argument (NULL, negative size, bad option)        */
#define DEC_ENOMEM (-2)      /* device allocation failed                               */
#define DEC_EHIP (-3)        /* a HIP runtime call failed                              */
#define DEC_ENOTCONV (-4)    /* max_iters reached before the tolerance                 */
#define DEC_EBREAKDOWN (-5)  /* CG breakdown: p.Ap <= 0 or a non-finite scalar         */
#define DEC_ETOPO (-6)       /* invalid mesh: index out of range, repeated vertex,
                                non-finite coordinate, zero-volume tet, face shared by
                                more than two tets                                       */
#define DEC_EBUDGET (-7)     /* request does not fit the server's HBM budget           */
#define DEC_ESTATE (-8)      /* call out of order (e.g. solve before apply_bc)         */
#define DEC_ECANCELED (-9)   /* a served request was cancelled                          */

typedef struct dec_ctx dec_ctx;
typedef struct dec_mesh dec_mesh;

typedef void* (*dec_alloc_fn)(size_t bytes, void* user);
typedef void (*dec_free_fn)(void* ptr, void* user);

/* Create a context on HIP device `device`, ordering work on `stream`
 * (a hipStream_t; NULL = the device's null stream).  `alloc`/`free` provide
 * the library's device memory (both NULL: hipMalloc/hipFree). */
int dec_create(dec_ctx** out, int device, void* stream, dec_alloc_fn alloc, dec_free_fn free_fn,
               void* user);
/* DEC_ESTATE while meshes or servers created on ctx are still alive. */
int dec_destroy(dec_ctx* ctx);
const char* dec_status_string(int status);
/* Message of the last failure on ctx; with ctx NULL, of the last failed call
 * that takes no context on this thread (dec_tetgen_read). */
const char* dec_last_error(const dec_ctx* ctx);

/* ---- topology (Section 2.1: cells, incidence, coboundary d) ------------
 * xyz: [V x 3] float64, tets: [T x 4] int32, device.  Builds the edge set
 * (unique vertex pairs (lo < hi), numbered in lexicographic order, oriented
 * lo -> hi so (d0 a)_e = a_hi - a_lo), the edge-to-tet incidence in
 * ascending tet order, the static CSR pattern of L (full edge graph plus
 * diagonal, columns ascending) and the boundary faces.  Returns DEC_ETOPO
 * for an invalid mesh.  Synchronises the stream. */
int dec_build_topology(dec_ctx* ctx, int64_t V, const double* xyz, int64_t T, const int32_t* tets,
                       dec_mesh** out);
/* Counts of vertices, tets, edges, faces, boundary faces and nonzeros of L (host outputs; any
 * may be NULL). */
int dec_mesh_info(const dec_mesh* m, int64_t* V, int64_t* T, int64_t* E, int64_t* F,
                  int64_t* F_boundary, int64_t* nnz);
/* Copy the edge list [E x 2] int32 (lo, hi) into a device buffer. */
int dec_get_edges(const dec_mesh* m, int32_t* edges);
/* Copy the CSR of the current system matrix into device buffers (any may be NULL):
 * row_ptr [V+1] int32, col [nnz] int32, val64 [nnz] float64, val32 [nnz] float32.  Before
 * dec_apply_bc the values are those of L; after, those of the eliminated system A. */
int dec_get_csr(const dec_mesh* m, int32_t* row_ptr, int32_t* col, double* val64, float* val32);
int dec_mesh_destroy(dec_mesh* m);

/* ---- TetGen mesh files (Section 2.2: the input is TetGen's Delaunay mesh) --
 * Host only (no GPU call, no context).  node_path: the .node file (header
 * "<points> 3 <attributes> <marker flag>", then "<index> x y z [attributes]
 * [marker]" per point); ele_path: the .ele file (header "<tets> <4|10>
 * <attributes>", then "<index> n1 .. n4 [n5 .. n10] [attributes]" per tet).
 * '#' starts a comment.  The first point index (0 or 1) is the numbering
 * base; points and tets must be numbered consecutively from it; ten-node tets
 * keep their corners.  *V_out, *T_out (host, NULL ok) receive the counts;
 * with xyz, tets and node_marker all NULL only the headers are read.
 * Otherwise xyz [V x 3] float64, tets [T x 4] int32 (0-based) and node_marker
 * [V] int32 (0 without markers) are HOST buffers the caller sized from a first
 * call (any may be NULL).  DEC_EINVAL on a missing file or a malformed line;
 * dec_last_error(NULL) names the file and line. */
int dec_tetgen_read(const char* node_path, const char* ele_path, int64_t* V_out, int64_t* T_out,
                    double* xyz, int32_t* tets, int32_t* node_marker);

/* ---- spatial numbering (Section 2.2: nodes numbered by location, z first,
 * then y, then x) ------------------------------------------------------------
 * For points off a lattice the order is taken on cells: the bounding box is
 * cut into B^3 cells, B the smallest integer with B^3 >= V; a point's cell on
 * axis a is floor((x_a - lo_a) * (B / (hi_a - lo_a))) clamped to [0, B-1]
 * (0 on a flat axis); points go by (x cell, y cell, z cell), z cell fastest,
 * ties by original index.  Tets then go by their smallest new vertex number,
 * ties by original index, keeping their vertex order.  On a lattice with one
 * point per cell (a Kuhn cube) this is the lattice order.
 * order: DEC_ORDER_LEXICOGRAPHIC (the above, the paper's) or DEC_ORDER_MORTON
 * (cells by the interleaved bits of (x cell, y cell, z cell), z in the lowest
 * bit, which keeps neighbours in all three directions close in memory; ties
 * and tets as above).
 * xyz [V x 3] float64, tets [T x 4] int32 device inputs; xyz_out, tets_out
 * device outputs of the same shapes (not aliasing the inputs), tets_out
 * renumbered; vperm_out [V] (new -> old vertex) and tperm_out [T] (new -> old
 * tet) int32 device outputs, NULL ok.  DEC_ETOPO for a vertex index out of
 * range, DEC_EINVAL for non-finite coordinates.  Synchronises the stream. */
#define DEC_ORDER_LEXICOGRAPHIC 0
#define DEC_ORDER_MORTON 1
int dec_reorder(dec_ctx* ctx, int32_t order, int64_t V, const double* xyz, int64_t T, const int32_t* tets,
                double* xyz_out, int32_t* tets_out, int32_t* vperm_out, int32_t* tperm_out);

/* ---- Hodge star *1 with conductivity and cracks (Sections 2.1, 2.5) ----
 * |*e| = sum over the edge's tets (ascending tet id) of the signed area of
 * the circumcentric dual quadrilateral (m_e, c_f1, c_T, c_f2); |*e| is
 * snapped to 0 when |*e| <= 1e-12 |e|^2.  *1_e = kappa_e * (|*e| / |e|),
 * and 0 on edges cut by a crack disc.
 * kappa: [E] float64 (NULL: kappa = 1).  cracks: [n_cracks x 7] float64 rows
 * (cx, cy, cz, nx, ny, nz, r), unit normal (NULL when n_cracks == 0).  An
 * edge (p0 = lo, p1 = hi) is cut when (s0 < 0) != (s1 < 0) with
 * s = (p - c).n, and the crossing point q = p0 + s0/(s0 - s1) (p1 - p0)
 * has |q - c|^2 <= r^2 (FP64, fixed operation order, no contraction).
 * cut_out: [E] uint8 (NULL ok), star1_out: [E] float64 (NULL ok).  The mesh
 * keeps *1 for dec_assemble and the flux. */
int dec_hodge1(dec_mesh* m, const double* kappa, int32_t n_cracks, const double* cracks,
               uint8_t* cut_out, double* star1_out);

/* ---- assembly of L = d0^T *1 d0 ---------------------------------------
 * L_ij = -*1_e for e = (i, j), L_ii = sum of *1_e over the row's edges in
 * ascending column order, pattern fixed (zeros kept), no atomics.  Fills the
 * FP64 and FP32 CSR (full static pattern) and the sliced-ELL copies the
 * solver multiplies with.  By default the sliced-ELL copy leaves out edges
 * whose geometric dual area is exactly zero (L_ij = -0 for every kappa and
 * crack set), which leaves every product bit-for-bit unchanged;
 * DEC_ASM_FULL_PATTERN keeps them.  Beside its int32 columns the
 * sliced-ELL copy holds two compact encodings where they fit: 16-bit
 * offsets j - i when every stored column lies within 2^15 of its row, and
 * one-byte indices into a table of the matrix's distinct offsets (sorted,
 * at most 256; on a Kuhn lattice the 14 neighbour offsets and 0).  The
 * solver's product reads whichever encoding the autotuner timed fastest on
 * the matrix (the same columns, so the same sums). */
#define DEC_ASM_DEFAULT 0u
#define DEC_ASM_FULL_PATTERN 1u
int dec_assemble(dec_mesh* m, uint32_t flags);

/* ---- boundary data (eqs. 3-4, 12-13) -----------------------------------
 * bc_type [V] int8: 0 free, 1 Dirichlet (T = bc_value), 2 Neumann vertex
 * (outward flux density neumann_f0[v]).  bc_value [V] float64.
 * neumann_f0 [V] float64 or NULL.  Dirichlet rows and columns are
 * eliminated symmetrically (identity rows, b_i -= L_ij T_j); a boundary face
 * whose vertices are all Neumann or Dirichlet, at least one Neumann, loads
 * b_v -= f0_v A*_{v,f} on its Neumann vertices (A*_{v,f}: v's circumcentric
 * part of the face); connected parts of the graph of edges with *1 != 0
 * that hold no Dirichlet vertex are pinned to T = 0.  n_pinned_out (host,
 * NULL ok) receives their vertex count; b_out [V] float64 device (NULL ok)
 * the right-hand side.  A later call on the same assembly replaces the
 * earlier boundary data (the operator is rebuilt from *1 first); after a
 * failed call the mesh has no system until a call succeeds.
 * Synchronises the stream. */
int dec_apply_bc(dec_mesh* m, const int8_t* bc_type, const double* bc_value,
                 const double* neumann_f0, int64_t* n_pinned_out, double* b_out);

/* ---- solve ------------------------------------------------------------- */
#define DEC_PREC_FP64 0   /* FP64 PCG                                              */
#define DEC_PREC_MIXED 1  /* FP32 PCG inner solves inside FP64 iterative refinement */
#define DEC_PRECOND_JACOBI 0
#define DEC_PRECOND_FSAI 1 /* factored sparse approximate inverse, pattern lower(L)  */
#define DEC_PRECOND_BLOCK 2 /* tet systems only: block Jacobi, the exact inverse of A on
                               each cluster of <= 16 tets joined by limited faces
                               (conducting interior faces whose *_f the limiter set),
                               1 / a_ii on every other tet                          */
#define DEC_FMT_AUTO 0
#define DEC_FMT_CSR 1
#define DEC_FMT_SELL 2
#define DEC_NORM_RESIDUAL 0 /* stop on ||b - A T||_2 <= tol ||b||_2                      */
#define DEC_NORM_ENERGY 1   /* FP64 only: stop when the error in the A-norm,
                               ||T* - T||_A <= tol ||T*||_A, by the Hestenes-Stiefel
                               estimate: PCG step j removes alpha_j rho_j from
                               ||T* - T||_A^2, so the sum over a window of 16 steps
                               bounds the error of the iterate 15 steps back from
                               below, and ||T*||_A^2 = T0.(b + r0) + all steps.  For
                               systems whose weights span many orders (the tet
                               system's limited faces): there rounding T to FP64
                               alone leaves ||b - A T||_2 near eps ||A|| ||T||, far
                               above a useful tolerance, while CG keeps reducing the
                               A-norm error                                          */

typedef struct dec_solve_opts {
    int32_t precision;           /* DEC_PREC_*                                     */
    int32_t precond;             /* DEC_PRECOND_*                                  */
    double tol;                  /* stop at ||b - A T|| <= tol ||b|| (FP64), norm below */
    double inner_tol;            /* mixed: relative tolerance of each FP32 solve   */
    int32_t adaptive_final_inner;/* mixed: inner tol max(inner_tol, 0.5 tol||b||/||r||) */
    int32_t warm_start;          /* T holds the initial guess (Dirichlet values are imposed) */
    int64_t max_iters;           /* cap on PCG iterations (FP64) / inner iterations (mixed;
                                    one FP32 solve gets at most max(max_iters / 8, 64)) */
    int32_t format;              /* DEC_FMT_* for the SpMV                         */
    int32_t chunk;               /* iterations per launch batch (0: default)       */
    int32_t use_graph;           /* capture each batch in a hipGraph               */
    int32_t profile;             /* 0: off; k > 0: time SpMV launches with HIP events,
                                    every k-th one of each launch batch, the batch's
                                    launches k-1, 2k-1, ... (1: all)               */
    int32_t norm;                /* DEC_NORM_* of the stopping test                */
} dec_solve_opts;

typedef struct dec_solve_stats {
    int64_t iterations;       /* FP64: PCG iterations. mixed: sum of inner iterations    */
    int64_t outer_iterations; /* mixed: refinement steps (FP64 residuals)                */
    int64_t restarts;         /* FP64: restarts from the true residual                    */
    int32_t fp64_fallback;    /* mixed: 1 when FP64 PCG finished: refinement stagnated (a
                                 correction that raised the residual is undone first) or an
                                 FP32 solve broke down or hit its cap (it is not applied)   */
    int32_t status;           /* DEC_OK / DEC_ENOTCONV / DEC_EBREAKDOWN                   */
    double rel_residual;      /* true FP64 ||b - A T|| / ||b|| at exit; with DEC_NORM_ENERGY
                                 and DEC_OK, the final A-norm error estimate instead       */
    double solve_ms;          /* wall time of the call on the stream (HIP events)          */
    int64_t spmv_launches;    /* profile: SpMV launches timed                              */
    double spmv_ms;           /* profile: summed duration of those launches                */
    double spmv_bytes;        /* bytes one SpMV must move: CSR definition over the entries
                                 the product uses (nnz (s+c) + 4 (V+1) + 2 V s, plus V s
                                 for the row excess of a difference-form product; c = 2
                                 with 16-bit column offsets, else 4)                       */
    int64_t spmv_nnz;         /* entries the product uses (full pattern or pruned)       */
    double plain_residual;    /* true FP64 ||b - A T||_2 / ||b||_2 at exit                 */
    int32_t spmv_unroll;      /* the product variant of the iteration's precision: entry
                                 pairs in flight per lane (2, 3, 4; timed by the autotuner) */
    int32_t spmv_nontemporal; /* 1 when its matrix loads and y stores are non-temporal     */
    int32_t spmv_col_bytes;   /* its column encoding: 1 one-byte offset-table index, 2
                                 16-bit offset, 4 int32 column                             */
    int32_t spmv_band;        /* slices per band of its banded slice order, 0 for plain    */
    int32_t spmv_order;       /* 1 when each row issues its column loads ahead of its value
                                 loads (the tuner's pick where HBM latency dominates), 0
                                 for the two interleaved                                   */
} dec_solve_stats;

/* Solver knobs read from the environment when a mesh's solver state is
 * first created (first dec_solve or dec_spmv on it), for tests and timing.
 * The first three change no result; the others change rounding (the split
 * form's arithmetic, or how the reductions are partitioned):
 *   DEC_SELL_UNROLL=2|3|4, DEC_SELL_NT=0|1, DEC_SELL_ORDER=0|1  pin the
 *       sliced-ELL variant the autotuner would pick (entry pairs in flight,
 *       non-temporal loads, a row's loads interleaved or columns first);
 *   DEC_SELL_COLS=8|16|32 read the columns through the one-byte offset
 *       table, the 16-bit offsets or the int32 columns (when the matrix
 *       lacks that encoding, the next wider one it holds);
 *   DEC_SELL_BAND=plane,band | auto  read at assembly: the product walks
 *       each XCD's share of slices band by band across planes of `plane`
 *       slices (`auto`: planes of the farthest column offset, bands of about
 *       1 MiB of matrix, where that offset spans more than 2 MiB of matrix),
 *       so a gather one plane back stays in L2; unset, plain order (on this
 *       GPU the bands cut the fetched bytes but not the time).  Changes the
 *       grouping of the product's partial sums, so the rounding of solves;
 *   DEC_VEC_PAIRS=0       FP32 vector kernels one row per lane instead of
 *       two (float2 elements);
 *   DEC_JACOBI_SPLIT=0|1  run Jacobi PCG on A, or always in split form (CG
 *       on D^-1/2 A D^-1/2); unset, the split form is taken for plain
 *       systems of 65,536 rows or more with a positive diagonal;
 *   DEC_BLOCKS_PER_CU, DEC_SPMV_BLOCKS_PER_CU  workgroups per CU of the
 *       vector kernels (default 4; 8 from 2^22 rows) and of the SpMV
 *       (default 8). */

/* Fill opts (host) with the defaults: FP64, Jacobi, tol 1e-10 (the relative
 * tolerance of Section 3.1's solves), inner_tol 1e-5, adaptive final inner
 * tolerance on, cold start, max_iters 100000, auto format, chunk 32, graphs
 * on, profiling off, plain residual norm.  DEC_EINVAL when opts is NULL. */
int dec_solve_opts_default(dec_solve_opts* opts);
/* The iterative solve of the assembled system (Section 2.3: the paper solves
 * its system with a preconditioned Krylov method, FGMRES with a
 * sparse-approximate-inverse preconditioner; the vertex system here is
 * symmetric positive definite, so the method is preconditioned conjugate
 * gradients with Jacobi, FSAI or block-Jacobi preconditioning, in FP64 or as
 * FP32 inner solves inside FP64 iterative refinement).  Solves A T = b after
 * dec_apply_bc.  opts (host, read during the call).  T [V] float64 device,
 * owned by the caller: initial guess when opts->warm_start, solution on
 * return.  stats (host) may be NULL.  Returns DEC_OK, DEC_ENOTCONV or
 * DEC_EBREAKDOWN (T then holds the last iterate), DEC_ESTATE before
 * dec_apply_bc, DEC_EINVAL for a bad option.  The solver keeps its Krylov
 * vectors with the mesh (allocated on first use).  Synchronises the stream. */
int dec_solve(dec_mesh* m, const dec_solve_opts* opts, double* T, dec_solve_stats* stats);

/* The same FP64 Jacobi PCG as dec_solve, for callers that cannot allocate
 * device memory (code running while other work is captured into a graph,
 * tight serving loops, harnesses that forbid hipMalloc): it calls no
 * allocator.  Its Krylov vectors r, p, q, the partial sums of its reductions
 * and its scalar state live in one static device array of the library, held
 * on every GPU the library runs on from library load to process end:
 * 3 x 8 B x DEC_NOALLOC_MAX_ROWS (96 MiB) plus 64 KiB; x is T itself.
 * m: after dec_apply_bc, at most DEC_NOALLOC_MAX_ROWS rows (DEC_EINVAL with a
 * message naming both counts beyond that).  opts: precision DEC_PREC_FP64,
 * precond DEC_PRECOND_JACOBI, norm DEC_NORM_RESIDUAL and profile 0, else
 * DEC_EINVAL; tol, warm_start, max_iters and chunk as in dec_solve; format and
 * use_graph are ignored (sliced-ELL product, no graphs).  T [V] float64
 * device: initial guess when warm_start, solution on return.  stats (host,
 * NULL ok): iterations, restarts, residuals, solve_ms (host clock).  Returns
 * as dec_solve.  Every call on one GPU uses that GPU's one array: calls from
 * this process are serialised per device, and the array keeps the last
 * call's contents (each call initialises what it reads).  It is ordered on
 * the context's stream and synchronises it before returning. */
#define DEC_NOALLOC_MAX_ROWS 4194304
int dec_solve_noalloc(dec_mesh* m, const dec_solve_opts* opts, double* T, dec_solve_stats* stats);

/* y = A x with the current system matrix: the solver's matrix-vector product
 * (Section 2.3), the dominant kernel of every solve.  precision DEC_PREC_FP64
 * (x, y float64) or DEC_PREC_MIXED (x, y float32), format DEC_FMT_CSR (the
 * full static pattern) or DEC_FMT_SELL / DEC_FMT_AUTO (the solver's
 * sliced-ELL copy; the same sums).  x, y: device vectors of length V owned
 * by the caller, not aliasing.  DEC_ESTATE before dec_assemble, DEC_EINVAL
 * for a NULL vector or a bad precision.  Asynchronous on the stream. */
int dec_spmv(dec_mesh* m, int32_t precision, int32_t format, const void* x, void* y);

/* The FSAI factor G of the current system (built on first use): nnz_out
 * (host) receives its entry count; g_ptr [V+1] int32, g_col [nnz] int32,
 * g_val [nnz] float64 device buffers (any may be NULL).  Row i holds
 * y / sqrt(y_i) with A[S_i,S_i] y = e_i over S_i = {j <= i : A_ij stored}
 * (Kolotilina-Yeremin factored sparse approximate inverse, the role
 * ParaSails has in Section 2.3).  Synchronises the stream. */
int dec_get_fsai(dec_mesh* m, int64_t* nnz_out, int32_t* g_ptr, int32_t* g_col, double* g_val);

/* ---- flux and effective conductivity (Section 2.5) ---------------------
 * T [V] float64, side [V] int8 (1 inflow face, 2 outflow face, 0 other).
 * Q_in = sum over side 1 of (L T)_v, Q_out = -sum over side 2, with L before
 * boundary elimination; energy E = sum_e *1_e (T_hi - T_lo)^2.  k_eff is the
 * flux density through the inflow face over the gradient, Section 2.5's
 * definition: without a Neumann load (the last dec_apply_bc had neumann_f0
 * NULL) it is taken in the energy form k_eff = E length / (area dT^2), equal
 * to Q_in length / (area dT) at the exact solution and second order in the
 * solution's error; with a Neumann load k_eff = Q length / (area dT), Q the
 * flux through a Dirichlet side: Q_in when side marks inflow vertices, else
 * Q_out, NaN when it marks neither.
 * Host scalar outputs (NULL ok);
 * edge_flux_out [E] float64 device (NULL ok): *1_e (T_lo - T_hi).
 * Synchronises the stream. */
int dec_flux_effective_conductivity(dec_mesh* m, const double* T, const int8_t* side,
                                    double length, double area, double dT, double* k_eff,
                                    double* q_in, double* q_out, double* energy,
                                    double* edge_flux_out);

/* ---- verification error (eq. 15) ----------------------------------------
 * RMS = sqrt(sum_i w_i (T_i - a - g.p_i)^2) against the linear field with
 * field = {a, g_x, g_y, g_z} (HOST array of 4).  m: the mesh of vertices and
 * tets (not a tet system).  on_tets = 1: T [T] float64 device holds one
 * value per tet (a tet system's solution), p_i the tet's circumcentre, w_i
 * its volume, as in the paper; on_tets = 0: T [V] per vertex, p_i the vertex,
 * w_i = sum over its tets of vol / 4.  *rms host.  Synchronises the stream. */
int dec_rms_error(dec_mesh* m, int32_t on_tets, const double* T, const double* field, double* rms);

/* ---- cracking (Section 3, deterministic cracking process) --------------
 * The face with the largest heat-flux density: over the edges e with
 * eligible[e] != 0 (eligible [E] uint8 device, or NULL for every edge whose
 * dual cell has nonzero area and whose *1_e is not zero, i.e. the faces not
 * cracked yet), the largest |*1_e (T_hi - T_lo)| / |*e| for the solution
 * T [V] float64 device, |*e| the edge's dual area.  Ties go to the smallest
 * edge id.  *edge_out (host) receives the edge, -1 when no eligible edge has
 * a finite density; *density_out (host, NULL ok) its density.  A crack is
 * then a zero in the conductivity given to dec_hodge1.  Needs dec_hodge1.
 * Synchronises the stream. */
int dec_max_flux_edge(dec_mesh* m, const double* T, const uint8_t* eligible, int64_t* edge_out,
                      double* density_out);

/* ---- temperature on the tets, flux through the triangles ---------------
 * The paper's own unknowns (Section 2.3, eq. 11-13): one temperature per tet
 * (the Voronoi vertex at its circumcentre), one flux per triangle (the dual
 * of a Voronoi edge).  The flux block (1/kappa) * is diagonal, so it is
 * eliminated and the Schur complement on the tets is assembled: a face f
 * between tets t1 and t2 couples them with W_f = kappa_f / *_f, a Dirichlet
 * face adds W_f to its tet's diagonal and W_f T0_f to its right-hand side,
 * a Neumann face subtracts its prescribed outward flux from it, insulated and
 * cracked faces carry nothing.  *_f = max(h_f / |f|, limiter):
 * h_f the signed length of the Voronoi edge through f (t1's circumcentre to
 * t2's, or to the face's circumcentre on the boundary, positive along the
 * normal out of t1), |f| the face area; the limiter is Section 3.1's (1e-8
 * when limiter <= 0).
 *
 * Faces are numbered by owner tet (the lowest tet holding the face), then by
 * local index (the tet's vertex opposite the face).  A boundary face is
 * Dirichlet when its three vertices have bc_type 1, with T0 their mean
 * bc_value, and inflow/outflow when all three vertices carry side 1/2; it is
 * Neumann (eq. 13) when all three have bc_type 2, whose bc_value is then an
 * outward flux density: the face's outward flux f0 |f|, f0 their mean, moves
 * to its tet's right-hand side.  Other boundary faces are insulated.
 * A face is cracked when its Voronoi edge crosses a disc (cracks as in
 * dec_hodge1) or kappa_face is 0.
 *
 * m: a mesh from dec_build_topology.  kappa_face [F] float64 device (NULL
 * for 1), cracks [n_cracks x 7] device, bc_type/bc_value/side [V] device
 * (side NULL ok), all read during the call.  *dual_out receives a new mesh
 * whose rows are the tets (V = T of m, F the faces), assembled and with its
 * boundary data applied: dec_solve, dec_spmv, dec_get_csr, dec_get_fsai and
 * dec_mesh_info apply to it; the vertex calls (dec_hodge1, dec_assemble,
 * dec_apply_bc, dec_flux_effective_conductivity, dec_max_flux_edge) return
 * DEC_ESTATE.  Tets in parts joined to no Dirichlet face over conducting
 * faces are pinned to 0 (*n_pinned_out, host, NULL ok).  The limiter puts
 * weights up to kappa / limiter beside weights of order |f| / h, so the
 * solver's (sliced-ELL) product of this system takes the difference form
 * (L x)_i = e_i x_i + sum_j L_ij (x_j - x_i), with e_i the exact sum of the
 * tet's Dirichlet-face weights (1 on pinned rows): the diagonal never cancels
 * against the limited couplings, so residuals keep full FP64 (and FP32)
 * relative accuracy; dec_spmv with DEC_FMT_CSR applies the stored matrix
 * as is.  Free it with
 * dec_mesh_destroy; it does not refer to m.  Synchronises the stream.
 * DEC_ETOPO if a face is shared by more than two tets. */
int dec_dual_build(dec_mesh* m, const double* kappa_face, int32_t n_cracks, const double* cracks,
                   const int8_t* bc_type, const double* bc_value, const int8_t* side, double limiter,
                   dec_mesh** dual_out, int64_t* n_pinned_out);

/* Counts of a tet system (host outputs, each NULL ok): faces, limited faces,
 * clusters inverted as blocks by DEC_PRECOND_BLOCK, the largest of them.
 * This call, dec_dual_faces and dec_dual_flux return DEC_ESTATE for a mesh
 * of vertex unknowns. */
int dec_dual_info(const dec_mesh* d, int64_t* n_faces, int64_t* n_limited, int64_t* n_blocks,
                  int64_t* max_block);

/* Face records of a tet system, device outputs (each NULL ok):
 * face_tets [F x 2] int32 (t1, t2 or -1), face_local [F x 2] int32 (local
 * index of the face in t1 and t2, or -1), weight [F] float64 (W_f, 0 on
 * insulated and cracked faces), cut [F] uint8.  Stream-ordered. */
int dec_dual_faces(const dec_mesh* d, int32_t* face_tets, int32_t* face_local, double* weight,
                   uint8_t* cut);

/* Flux of a tet solution T [T] float64 device: energy
 * E = sum_f W_f (T_t1 - T_t2)^2 over interior faces plus W_f (T_t1 - T0_f)^2
 * over Dirichlet faces, k_eff = E length / (area dT^2), Q_in = sum of
 * W_f (T0_f - T_t1) over inflow faces, Q_out = sum of W_f (T_t1 - T0_f) over
 * outflow faces.  Host outputs (NULL ok).  Synchronises the stream. */
int dec_dual_flux(dec_mesh* d, const double* T, double length, double area, double dT, double* k_eff,
                  double* q_in, double* q_out, double* energy);

/* ---- serving: many solves, batched on the device ----------------------
 * A server admits requests (one full problem each: mesh, conductivity,
 * cracks, boundary data) while the HBM budget allows, runs their setup on a
 * side stream while the systems already admitted keep iterating, keeps each
 * admitted system's matrix and Krylov state resident, and advances all of
 * them together: one dec_server_step replays `chunk` PCG iterations of every
 * admitted system in three batched kernels (captured in a hipGraph), then
 * runs the FP64 refinement steps of systems whose inner solve ended, retires
 * converged systems (solution copied to T_out, flux and k_eff computed) and
 * admits new ones.  Each system's reductions depend only on that system, so
 * its result is bit-for-bit the same alone and in any mix.  Not thread-safe:
 * call from the context's thread. */
typedef struct dec_server dec_server;

typedef struct dec_request {
    int64_t V;                 /* vertices                                              */
    const double* xyz;         /* [V x 3] device                                        */
    int64_t T;                 /* tets                                                  */
    const int32_t* tets;       /* [T x 4] device                                        */
    const double* kappa;       /* [E] device or NULL (kappa = 1), canonical edge order   */
    int32_t n_cracks;
    const double* cracks;      /* [n_cracks x 7] device or NULL                          */
    const int8_t* bc_type;     /* [V] device, as dec_apply_bc                            */
    const double* bc_value;    /* [V] device                                            */
    const double* neumann_f0;  /* [V] device or NULL                                    */
    const int8_t* side;        /* [V] device or NULL: faces for Q_in / Q_out             */
    double length, area, dT;   /* k_eff scaling (0: 1)                                   */
    double* T_out;             /* [V] device or NULL: receives the solution              */
    uint64_t user_tag;
    const double* T0;          /* [V] device or NULL: initial guess (warm start, e.g. the
                                  previous step of a cracking path); Dirichlet values and
                                  pinned zeros are imposed on it                          */
    const dec_mesh* mesh;      /* NULL, or a mesh of vertex unknowns from dec_build_topology
                                  on the server's device with V and T as above: the server
                                  copies its topology (and its geometry and solver pattern
                                  when it has them, after dec_hodge1 / dec_assemble)
                                  instead of building them from xyz and tets, which may then
                                  be NULL; many requests on one mesh (the steps of cracking
                                  paths) share that work                                  */
} dec_request;
/* The request's input arrays must stay valid until its result is polled
 * (they are read when the request is admitted); T_out likewise, and the
 * request's mesh, which must not change or be destroyed before then. */

typedef struct dec_result {
    uint64_t ticket;
    uint64_t user_tag;
    int32_t status;             /* DEC_OK, DEC_ENOTCONV, DEC_EBREAKDOWN (an FP64 inner
                                   solve broke down or the residual is not finite),
                                   DEC_ECANCELED, or a setup error                         */
    int32_t fp64_fallback;      /* mixed: 1 when FP64 PCG finished (an FP32 solve broke down
                                   or reached its cap of max(max_iters / 8, 64) iterations and
                                   was not applied, or refinement stagnated: a correction that
                                   raised the residual is taken back first), as dec_solve  */
    double k_eff, q_in, q_out, energy;
    double rel_residual;        /* FP64 ||b - A T|| / ||b|| at retirement                  */
    int64_t inner_iterations;   /* PCG iterations (FP32 inner, or FP64)                    */
    int64_t outer_iterations;   /* refinement steps                                       */
    double t_submit_ms, t_admit_ms, t_start_ms, t_finish_ms; /* host clock since creation  */
} dec_result;

typedef struct dec_server_opts {
    int32_t precision;            /* DEC_PREC_MIXED (FP32 inner, FP64 refinement) or DEC_PREC_FP64 */
    int32_t max_slots;            /* systems resident at once (<= 1024)                    */
    double tol;                   /* ||b - A T|| <= tol ||b|| (FP64)                        */
    double inner_tol;             /* mixed: relative tolerance of each FP32 solve            */
    int32_t adaptive_final_inner; /* as dec_solve_opts                                      */
    int32_t chunk;                /* iterations per batch step (even, 2..1024)              */
    int64_t max_iters;            /* per request, inner iterations; one FP32 solve gets at
                                     most max(max_iters / 8, 64)                            */
} dec_server_opts;

/* Defaults: mixed precision, 64 slots, tol 1e-10, inner_tol 1e-5, adaptive
 * final inner tolerance, chunk 16, max_iters 100000. */
int dec_server_opts_default(dec_server_opts* opts);
/* hbm_budget_bytes bounds the estimated device memory of the admitted
 * requests (setup peak included). */
int dec_server_create(dec_ctx* ctx, size_t hbm_budget_bytes, const dec_server_opts* opts, dec_server** out);
/* Queue a request (FIFO).  DEC_EBUDGET when it cannot fit the budget even alone.
 * Unlike the other calls, the request's arrays are read later, when a
 * dec_server_step admits it (its setup runs on a stream of the server, after
 * the work queued on the context's stream before this call), and T_out is
 * written when it retires: the caller keeps every array of the request valid
 * and unchanged until its result has been polled or it was cancelled. */
int dec_server_submit(dec_server* s, const dec_request* req, uint64_t* ticket);
/* Advance the server: one batch of iterations, refinement steps, retirements,
 * admissions.  n_active / n_pending (host, NULL ok) receive the counts after
 * the step.  Synchronises its streams. */
int dec_server_step(dec_server* s, int32_t* n_active, int32_t* n_pending);
/* Move up to max finished results (retirement order) into out; n_out receives the count. */
int dec_server_poll(dec_server* s, dec_result* out, int32_t max, int32_t* n_out);
/* Cancel a pending or admitted request; its result has status DEC_ECANCELED.
 * DEC_EINVAL when the ticket is unknown or already finished. */
int dec_server_cancel(dec_server* s, uint64_t ticket);
/* Counters since the server was created, for the roofline of serving. */
typedef struct dec_server_counters {
    double batch_ms;          /* time of the steps' graph replays (HIP events on the server's stream) */
    double batch_bytes;       /* algorithmic bytes of the iterations they ran, per system and iteration
                                 kept entries x (value + column bytes) + 4 (V + 1) + 12 V values (the
                                 product's x and y; the update's r, q, D^-1 and r; the closing kernel's
                                 D^-1, r, p, x, x and p)                                              */
    int64_t batch_iterations; /* system-iterations run in them                                        */
    int32_t variant[4];       /* the batched product's entry pairs in flight and non-temporal loads
                                 (0/1) for FP64, then for FP32 (0 where that precision has not run);
                                 the server picks them per precision by timing its product on the
                                 first batch of that precision; the choice changes no result         */
    double host_ms[4];        /* host wall time of dec_server_step's phases: building and launching
                                 the batch, admissions, waiting for the batch, refinement steps       */
    int64_t steps;            /* dec_server_step calls                                                */
    int32_t order[2];         /* the batched product's load order for FP64, then FP32: 1 when a row's
                                 column loads go out ahead of its value loads, 0 interleaved (timed
                                 with the variant above)                                            */
} dec_server_counters;
/* Fill *out (host).  DEC_EINVAL when s or out is NULL. */
int dec_server_stats(const dec_server* s, dec_server_counters* out);
int dec_server_destroy(dec_server* s);

#ifdef __cplusplus
}
#endif

#endif /* DEC_H */
