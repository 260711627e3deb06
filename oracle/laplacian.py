"""Oracle operator and boundary data: L = d0^T *1 d0, Dirichlet/Neumann, isolated parts (test infrastructure).

Section 2.1: with temperature a primal 0-form alpha, the flux is the dual
2-form omega = *1 d alpha and conservation is d^T omega = 0 on the dual,
so the discrete steady problem at the vertices is L T = b with
L = d0^T *1 d0.  Entrywise, for edge e = (i, j): L_ij = L_ji = -*1_e and
L_ii = sum of *1_e over the edges at i.  The sparsity pattern is the full
edge graph plus the diagonal and is kept fixed even where *1_e = 0 (the
paper keeps the system matrix's form fixed when it inserts cracks,
Section 2.3).

Boundary data (eqs. 3-4 and 12-13, restated for vertex unknowns):
* Dirichlet vertices are eliminated symmetrically: for a free row i,
  b_i -= L_ij T_j over Dirichlet j; Dirichlet rows and columns become the
  identity with b_j = T_j (pattern kept, as in the paper's zero-and-unit-
  diagonal treatment);
* Neumann data f0 (outward normal flux density) enters as b_v -= f0_v A*_v,
  A*_v the area of v's dual cell on the Neumann faces (see
  geometry.neumann_load); faces without data are insulated, which is the
  natural condition of the truncated dual cells;
* a connected part of the graph of edges with *1_e != 0 that holds no
  Dirichlet vertex (cut off by cracks) has no unique solution; its vertices
  are pinned to T = 0 (identity rows and columns, b = 0).
"""
import numpy as np
import scipy.sparse as sp
from scipy.sparse.csgraph import connected_components


def assemble(V, edges, star1):
    """CSR of L with columns ascending per row, diagonal included, explicit zeros kept.

    Returns ``(L, entry_edge)``: ``entry_edge[k]`` is the edge of stored
    entry k, or -1 for a diagonal entry.  The diagonal sums *1_e over the
    row's off-diagonal entries in ascending column order.
    """
    edges = np.asarray(edges, dtype=np.int64)
    star1 = np.asarray(star1, dtype=np.float64)
    E = len(edges)
    lo, hi = edges[:, 0], edges[:, 1]
    rows = np.concatenate([lo, hi, np.arange(V)])
    cols = np.concatenate([hi, lo, np.arange(V)])
    eid = np.concatenate([np.arange(E), np.arange(E), -np.ones(V, dtype=np.int64)])
    order = np.lexsort((cols, rows))
    rows, cols, eid = rows[order], cols[order], eid[order]
    off = eid >= 0
    vals = np.zeros(len(rows))
    vals[off] = -star1[eid[off]]
    vals[~off] = np.bincount(rows[off], weights=star1[eid[off]], minlength=V)
    indptr = np.concatenate([[0], np.cumsum(np.bincount(rows, minlength=V))])
    L = sp.csr_matrix((vals, cols, indptr), shape=(V, V))
    L.has_sorted_indices = True
    return L, eid


def isolated_components(V, edges, star1, dirichlet):
    """Boolean mask of vertices in connected parts (over edges with *1_e != 0) that hold no Dirichlet vertex."""
    edges = np.asarray(edges, dtype=np.int64)
    nz = np.asarray(star1) != 0.0
    g = sp.coo_matrix((np.ones(int(nz.sum())), (edges[nz, 0], edges[nz, 1])), shape=(V, V))
    _, label = connected_components(g, directed=False)
    anchored = np.zeros(label.max() + 1 if V else 0, dtype=bool)
    anchored[label[np.asarray(dirichlet, dtype=bool)]] = True
    return ~anchored[label]


def apply_bc(L, bc_type, bc_value, edges=None, star1=None, neumann=None, pin_isolated=True):
    """System (A, b) after Dirichlet elimination, Neumann data and pinning of isolated parts.

    Returns ``(A, b, pinned)`` with ``pinned`` the mask of pinned vertices.
    ``bc_type`` is 1 on Dirichlet vertices, ``bc_value`` their temperature;
    ``neumann`` is the load g of ``geometry.neumann_load`` (b -= g) or None.
    """
    V = L.shape[0]
    dirichlet = np.asarray(bc_type) == 1
    if pin_isolated:
        pinned = isolated_components(V, edges, star1, dirichlet)
    else:
        pinned = np.zeros(V, dtype=bool)
    pinned &= ~dirichlet
    fixed = dirichlet | pinned
    xd = np.where(dirichlet, np.asarray(bc_value, dtype=np.float64), 0.0)
    b = np.zeros(V)
    if neumann is not None:
        b -= np.asarray(neumann, dtype=np.float64)
    b = b - L @ xd
    b[fixed] = xd[fixed]
    A = L.copy()
    rows = np.repeat(np.arange(V), np.diff(A.indptr))
    cols = A.indices
    kill = fixed[rows] | fixed[cols]
    A.data = np.where(kill, 0.0, A.data)
    A.data = np.where(kill & (rows == cols), 1.0, A.data)
    return A, b, pinned


def lumped_vertex_volumes(xyz, tets):
    """V*_v = sum over the tets at v of vol(T)/4 (weights of the RMS error)."""
    from .geometry import tet_volumes

    vol = tet_volumes(xyz, tets)
    return np.bincount(np.asarray(tets, dtype=np.int64).ravel(), weights=np.repeat(vol / 4.0, 4),
                       minlength=len(xyz))


def rms_error(T, T_exact, weights):
    """Volume-weighted RMS error of eq. 15, with vertex unknowns and vertex volumes as weights."""
    d = np.asarray(T) - np.asarray(T_exact)
    return float(np.sqrt((weights * d * d).sum()))
