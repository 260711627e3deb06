"""Oracle topology: cells, incidence and the coboundary operators (test infrastructure).

Section 2.1 (chain and cochain complexes): the topology of the simplicial
3-complex, i.e. its cells and their orientations, defines the coboundary
operators d0 (nodes -> edges) and d1 (edges -> faces) with d1 d0 = 0.

Conventions fixed here (the paper leaves them to the implementation):
* an edge is the unordered vertex pair stored as (lo, hi), lo < hi, oriented
  lo -> hi; edges are numbered in lexicographic (lo, hi) order;
* a face is the sorted triple (a, b, c) oriented a -> b -> c; faces are
  numbered in lexicographic order;
* the six local edges of a tet (v0, v1, v2, v3) are taken in the order
  LOCAL_EDGES.
"""
import numpy as np
import scipy.sparse as sp

LOCAL_EDGES = ((0, 1), (0, 2), (0, 3), (1, 2), (1, 3), (2, 3))
LOCAL_FACES = ((1, 2, 3), (0, 2, 3), (0, 1, 3), (0, 1, 2))  # face k is opposite vertex k


def _edge_keys(tets, V):
    tets = np.asarray(tets, dtype=np.int64)
    a = tets[:, [p for p, _ in LOCAL_EDGES]]
    b = tets[:, [q for _, q in LOCAL_EDGES]]
    return np.minimum(a, b) * V + np.maximum(a, b)  # [T, 6]


def edges_of(tets, V):
    """Unique edges (lo < hi) of the tets, sorted lexicographically. int64 [E, 2]."""
    keys = np.unique(_edge_keys(tets, V).ravel())
    return np.stack([keys // V, keys % V], axis=1)


def tet_edge_ids(tets, V, edges):
    """Edge id of each of the 6 local edges of every tet. int64 [T, 6]."""
    keys = edges[:, 0] * V + edges[:, 1]
    return np.searchsorted(keys, _edge_keys(tets, V))


def faces_of(tets):
    """Unique faces as sorted triples, lexicographic order, with the tets incident to each.

    Returns ``(faces [F,3] int64, count [F] int64)`` where ``count`` is the
    number of tets sharing the face (1 on the boundary, 2 inside).
    """
    tets = np.asarray(tets, dtype=np.int64)
    tri = np.sort(tets[:, list(LOCAL_FACES)], axis=2).reshape(-1, 3)
    uniq, count = np.unique(tri, axis=0, return_counts=True)
    return uniq, count


def boundary_faces(tets):
    """Faces shared by exactly one tet: list of (tet, local face k) pairs in ascending tet order."""
    tets = np.asarray(tets, dtype=np.int64)
    tri = np.sort(tets[:, list(LOCAL_FACES)], axis=2).reshape(-1, 3)
    _, inv, count = np.unique(tri, axis=0, return_inverse=True, return_counts=True)
    inv = inv.ravel()
    sel = np.nonzero(count[inv] == 1)[0]
    return np.stack([sel // 4, sel % 4], axis=1)


def d0_matrix(edges, V):
    """Coboundary d0: (d0 a)_e = a_hi - a_lo for e = (lo, hi).  Sparse E x V."""
    E = len(edges)
    rows = np.repeat(np.arange(E), 2)
    cols = edges.reshape(-1)
    vals = np.tile([-1.0, 1.0], E)
    return sp.csr_matrix((vals, (rows, cols)), shape=(E, V))


def d1_matrix(faces, edges, V):
    """Coboundary d1 on oriented faces (a<b<c): boundary = [b,c] - [a,c] + [a,b].  Sparse F x E."""
    keys = edges[:, 0] * V + edges[:, 1]
    a, b, c = faces[:, 0], faces[:, 1], faces[:, 2]
    e_bc = np.searchsorted(keys, b * V + c)
    e_ac = np.searchsorted(keys, a * V + c)
    e_ab = np.searchsorted(keys, a * V + b)
    F = len(faces)
    rows = np.repeat(np.arange(F), 3)
    cols = np.stack([e_bc, e_ac, e_ab], axis=1).ravel()
    vals = np.tile([1.0, -1.0, 1.0], F)
    return sp.csr_matrix((vals, (rows, cols)), shape=(F, len(edges)))


def vertex_degrees(edges, V):
    """Number of edges at each vertex."""
    return np.bincount(edges.ravel(), minlength=V)


def check_mesh(xyz, tets):
    """Validity of a tet mesh as the path requires it.

    Returns a string naming the first problem found, or None: an index out of
    [0, V), a tet repeating a vertex, a tet with a non-finite vertex
    coordinate, a tet of zero volume, or a face shared by more than two tets
    (not a 3-manifold with boundary).
    """
    xyz = np.asarray(xyz, dtype=np.float64)
    tets = np.asarray(tets, dtype=np.int64)
    V = len(xyz)
    if tets.size and (tets.min() < 0 or tets.max() >= V):
        return "index out of range"
    s = np.sort(tets, axis=1)
    if np.any(s[:, 1:] == s[:, :-1]):
        return "repeated vertex"
    p = xyz[tets]
    with np.errstate(invalid="ignore"):  # inf - inf in a tet with an infinite coordinate
        a, b, c = p[:, 1] - p[:, 0], p[:, 2] - p[:, 0], p[:, 3] - p[:, 0]
        det = (a * np.cross(b, c)).sum(axis=1)
    if not np.all(np.isfinite(det)):
        return "non-finite coordinate"
    if np.any(det == 0.0):
        return "zero volume"
    if len(tets):
        _, count = faces_of(tets)
        if count.max() > 2:
            return "face shared by more than two tets"
    return None
