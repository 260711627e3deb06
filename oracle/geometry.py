"""Oracle geometry: circumcentres, circumcentric dual areas and the Hodge star *1 (test infrastructure).

Section 2.1: on a Delaunay tetrahedral complex with its circumcentric
(Voronoi) dual, the discrete Hodge stars are diagonal, each entry the ratio
of a dual cell's volume to its primal cell's volume; the conductivity is a
property of the (primal edge, dual face) pair, so *1 for edge e is
kappa_e |*e| / |e| with |*e| the area of the dual 2-cell of e.

The dual 2-cell of an edge is assembled tet by tet.  Inside a tet, the part
belonging to edge e = (i, j) is the planar quadrilateral (m_e, c_f1, c_T,
c_f2) in the bisector plane of e, where m_e is the edge midpoint (its
circumcentre), c_f1 and c_f2 the circumcentres of the two faces of the tet
that contain e, and c_T the tet's circumcentre.  Its signed area is
    1/2 [ h(e->f1) h(f1->T) + h(e->f2) h(f2->T) ],
h(e->f) the signed distance from m_e to c_f inside face f, positive toward
f's third vertex, and h(f->T) the signed distance from c_f to c_T along
f's normal, positive toward the tet's fourth vertex.  This is the signed
circumcentric convention of Hirani's DEC, which the paper's geometry
follows.  Dual cells of boundary edges are truncated at the boundary.
"""
import numpy as np

from .topology import LOCAL_EDGES, LOCAL_FACES, tet_edge_ids

# |*e| <= SNAP_REL * |e|^2 is taken as exactly zero (reading of the paper's
# near-zero limiter, Section 3.1; see the design notes for why it is a snap).
SNAP_REL = 1e-12


def _dot(a, b):
    return a[..., 0] * b[..., 0] + a[..., 1] * b[..., 1] + a[..., 2] * b[..., 2]


def _cross(a, b):
    return np.stack([a[..., 1] * b[..., 2] - a[..., 2] * b[..., 1],
                     a[..., 2] * b[..., 0] - a[..., 0] * b[..., 2],
                     a[..., 0] * b[..., 1] - a[..., 1] * b[..., 0]], axis=-1)


def _norm(a):
    return np.sqrt(_dot(a, a))


def circumcenter_tet(p0, p1, p2, p3):
    """Circumcentre of a tetrahedron (textbook closed form), vectorised over leading axes.

    With a, b, c = p1-p0, p2-p0, p3-p0:
    c_T = p0 + (|a|^2 (b x c) + |b|^2 (c x a) + |c|^2 (a x b)) / (2 a.(b x c)).
    """
    a, b, c = p1 - p0, p2 - p0, p3 - p0
    num = (_dot(a, a)[..., None] * _cross(b, c) + _dot(b, b)[..., None] * _cross(c, a)
           + _dot(c, c)[..., None] * _cross(a, b))
    den = 2.0 * _dot(a, _cross(b, c))
    return p0 + num / den[..., None]


def circumcenter_tri(p0, p1, p2):
    """Circumcentre of a triangle in 3D (textbook closed form).

    With a, b = p1-p0, p2-p0: c_f = p0 + ((|a|^2 b - |b|^2 a) x (a x b)) / (2 |a x b|^2).
    """
    a, b = p1 - p0, p2 - p0
    axb = _cross(a, b)
    num = _cross(_dot(a, a)[..., None] * b - _dot(b, b)[..., None] * a, axb)
    return p0 + num / (2.0 * _dot(axb, axb))[..., None]


def _edge_to_face(pi, pj, pk, cf):
    """h(e->f): signed in-plane distance from the midpoint of (pi, pj) to c_f, positive toward pk."""
    m = 0.5 * (pi + pj)
    e = pj - pi
    w = pk - pi
    u = w - (_dot(w, e) / _dot(e, e))[..., None] * e
    u = u / _norm(u)[..., None]
    return _dot(cf - m, u)


def _face_to_tet(pi, pj, pk, pl, cf, ct):
    """h(f->T): signed distance from c_f to c_T along the normal of face (pi,pj,pk), positive toward pl."""
    n = _cross(pj - pi, pk - pi)
    s = np.where(_dot(n, pl - pi) < 0.0, -1.0, 1.0)
    n = n * (s / _norm(n))[..., None]
    return _dot(ct - cf, n)


def elementary_dual_areas(xyz, tets):
    """Signed area of the part of each local edge's dual 2-cell inside each tet.  float64 [T, 6].

    Column q belongs to local edge LOCAL_EDGES[q].  Independent of the order
    in which a tet lists its vertices.
    """
    p = np.asarray(xyz, dtype=np.float64)[np.asarray(tets, dtype=np.int64)]  # [T, 4, 3]
    ct = circumcenter_tet(p[:, 0], p[:, 1], p[:, 2], p[:, 3])
    out = np.empty((len(p), 6))
    for q, (i, j) in enumerate(LOCAL_EDGES):
        k, l = [r for r in range(4) if r not in (i, j)]
        pi, pj, pk, pl = p[:, i], p[:, j], p[:, k], p[:, l]
        cf1 = circumcenter_tri(pi, pj, pk)
        cf2 = circumcenter_tri(pi, pj, pl)
        t1 = _edge_to_face(pi, pj, pk, cf1) * _face_to_tet(pi, pj, pk, pl, cf1, ct)
        t2 = _edge_to_face(pi, pj, pl, cf2) * _face_to_tet(pi, pj, pl, pk, cf2, ct)
        out[:, q] = 0.5 * (t1 + t2)
    return out


def tet_volumes(xyz, tets):
    """Unsigned tet volumes |a.(b x c)| / 6."""
    p = np.asarray(xyz, dtype=np.float64)[np.asarray(tets, dtype=np.int64)]
    a, b, c = p[:, 1] - p[:, 0], p[:, 2] - p[:, 0], p[:, 3] - p[:, 0]
    return np.abs(_dot(a, _cross(b, c))) / 6.0


def edge_lengths(xyz, edges):
    xyz = np.asarray(xyz, dtype=np.float64)
    return _norm(xyz[edges[:, 1]] - xyz[edges[:, 0]])


def dual_areas(xyz, tets, edges, snap=True):
    """|*e| for every edge: sum over the edge's tets, in ascending tet order, then the snap."""
    V = len(xyz)
    ids = tet_edge_ids(tets, V, edges)
    elem = elementary_dual_areas(xyz, tets)
    # bincount accumulates in input order, i.e. tet by tet in ascending tet id
    area = np.bincount(ids.ravel(), weights=elem.ravel(), minlength=len(edges))
    if snap:
        length = edge_lengths(xyz, edges)
        area = np.where(np.abs(area) <= SNAP_REL * length * length, 0.0, area)
    return area


def hodge1(xyz, tets, edges, kappa=None, cut=None, snap=True):
    """Diagonal of *1 with conductivity: star1_e = kappa_e * (|*e| / |e|), 0 on cut edges.

    Section 2.1 (Hodge star as the dual/primal volume ratio, conductivity on
    the edge/dual-face pair); cut edges model cracks, whose conductivity is
    set to zero (Section 2.5).
    """
    area = dual_areas(xyz, tets, edges, snap=snap)
    length = edge_lengths(xyz, edges)
    geo = area / length
    k = np.ones(len(edges)) if kappa is None else np.asarray(kappa, dtype=np.float64)
    star = k * geo
    if cut is not None:
        star = np.where(np.asarray(cut).astype(bool), 0.0, star)
    return star


def _face_vertex_areas(pts):
    """Signed area of each vertex's part of triangle pts[0..2] (circumcentric split)."""
    cf = circumcenter_tri(pts[0], pts[1], pts[2])
    out = []
    for a in range(3):
        b, c = [r for r in range(3) if r != a]
        lab = float(_norm(pts[b] - pts[a]))
        lac = float(_norm(pts[c] - pts[a]))
        hab = float(_edge_to_face(pts[a], pts[b], pts[c], cf))
        hac = float(_edge_to_face(pts[a], pts[c], pts[b], cf))
        out.append(0.5 * (0.5 * lab) * hab + 0.5 * (0.5 * lac) * hac)
    return out


def boundary_dual_areas(xyz, tets, bfaces, V):
    """A*_v: area of the part of the whole boundary surface belonging to vertex v's dual cell.

    For a boundary triangle (a, b, c) with circumcentre c_f, vertex a owns
    1/2 (|ab|/2) h(ab->f) + 1/2 (|ac|/2) h(ac->f) (signed, the 2D analogue
    of the elementary dual area).
    """
    xyz = np.asarray(xyz, dtype=np.float64)
    tets = np.asarray(tets, dtype=np.int64)
    out = np.zeros(V)
    for t, k in bfaces:
        verts = [int(tets[t, r]) for r in LOCAL_FACES[k]]
        for v, a in zip(verts, _face_vertex_areas([xyz[v] for v in verts])):
            out[v] += a
    return out


def neumann_load(xyz, tets, bfaces, bc_type, f0):
    """Right-hand-side load g of the Neumann data (eq. 4): the system gets b -= g.

    ``f0`` is the prescribed outward normal flux density sampled at vertices
    flagged Neumann (bc_type 2).  A boundary face carries Neumann data when
    each of its vertices is flagged Neumann or Dirichlet (bc_type 1) and at
    least one is Neumann; every Neumann vertex v of such a face gets
    g_v += f0_v * (v's circumcentric part of the face).  Other boundary faces
    are insulated.  Faces are visited in ascending (tet, local face) order.
    """
    xyz = np.asarray(xyz, dtype=np.float64)
    tets = np.asarray(tets, dtype=np.int64)
    bc_type = np.asarray(bc_type)
    f0 = np.asarray(f0, dtype=np.float64)
    g = np.zeros(len(xyz))
    for t, k in bfaces:
        verts = [int(tets[t, r]) for r in LOCAL_FACES[k]]
        kinds = [int(bc_type[v]) for v in verts]
        if not all(q in (1, 2) for q in kinds) or 2 not in kinds:
            continue
        for v, q, a in zip(verts, kinds, _face_vertex_areas([xyz[v] for v in verts])):
            if q == 2:
                g[v] += f0[v] * a
    return g
