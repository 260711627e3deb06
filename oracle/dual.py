"""Oracle of the paper's own unknowns: temperature on the tets, flux through the triangles
(test infrastructure only).

Section 2.1 puts the temperature 0-form on the nodes of one complex and the flux
2-form on the faces of its dual; the numerical implementation (Section 2.3,
eq. 11) takes the Voronoi complex for the temperature, so the unknowns are one
temperature per Delaunay tet (its circumcentre is the Voronoi node) and one
flux per Delaunay triangle (the dual of a Voronoi edge):

    [ (1/kappa) *   d^T ] [ omega ]   [ 0 ]
    [      d         0  ] [ alpha ] = [ 0 ],

with * the diagonal Hodge star of the triangles, *_f = |f*| / |f| (length of
the Voronoi edge through f over the triangle's area).  Dirichlet faces (eq. 12)
keep the incomplete Voronoi edge from the tet's circumcentre to the face's
circumcentre and move kappa-weighted T0 to the right-hand side; Neumann faces
(eq. 13) prescribe their flux: the face's row fixes omega_f and the known
flux moves to its tet's balance; insulated faces (zero flux) and cracked faces
(kappa = 0) have their rows and columns replaced by a unit diagonal, so their
flux is zero.  Section 3.1 limits
Hodge entries at 1e-8 (zero-length Voronoi edges occur wherever tets share a
circumcentre).

Eliminating omega (the (1,1) block is diagonal) leaves the Schur complement on
the tets: L = d diag(kappa_f / *_f) d^T, i.e. every face f between tets t1, t2
contributes W_f (T_t1 - T_t2) to both balances, with W_f = kappa_f / *_f, a
Dirichlet face W_f (T_t - T0), and a Neumann face its prescribed outward flux
g_f = f0 |f| (moved to the right-hand side).  `mixed_system` writes eq. 11-13
out literally (used to pin `dual_system`).

Readings (where the paper is silent): faces are numbered by their owner tet
(the lowest-numbered tet holding them), then by the local index of the
opposite vertex; a signed Voronoi-edge length (positive along the normal from
t1 to t2) and the limiter *_f := max(*_f, 1e-8) (negative entries included); a
boundary face is Dirichlet when all three vertices carry Dirichlet data, with
T0 the mean of the three vertex values, and its side (inflow / outflow) is the
vertices' common side; a boundary face is Neumann when all three vertices
carry Neumann data (type 2), the vertices' values being outward flux
densities, with f0 their mean; tets in parts joined to no Dirichlet face are
pinned to 0 and their Neumann data ignored.
"""
import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .cracks import _cut_by_disc
from .geometry import circumcenter_tet, circumcenter_tri
from .laplacian import isolated_components
from .topology import LOCAL_FACES

LIMITER = 1e-8


def faces_by_owner(tets):
    """Faces in owner order: arrays t1 (owner tet), k1 (local face index in t1, the index of
    the opposite vertex), t2 (the other tet or -1), k2 (its local index or -1), verts [F,3]
    (the face's vertices in t1's local order)."""
    tets = np.asarray(tets, dtype=np.int64)
    where = {}
    for t in range(len(tets)):
        for k, loc in enumerate(LOCAL_FACES):
            key = tuple(sorted(int(tets[t, j]) for j in loc))
            where.setdefault(key, []).append((t, k))
    t1, k1, t2, k2, verts = [], [], [], [], []
    for t in range(len(tets)):
        for k, loc in enumerate(LOCAL_FACES):
            key = tuple(sorted(int(tets[t, j]) for j in loc))
            hold = where[key]
            if hold[0][0] != t:  # owned by a lower tet
                continue
            assert len(hold) <= 2, "face shared by more than two tets"
            t1.append(t)
            k1.append(k)
            other = hold[1] if len(hold) == 2 else (-1, -1)
            t2.append(other[0])
            k2.append(other[1])
            verts.append([int(tets[t, j]) for j in loc])
    return (np.array(t1), np.array(k1), np.array(t2), np.array(k2), np.array(verts, dtype=np.int64))


def face_geometry(xyz, tets, faces, limiter=LIMITER):
    """Per face: area |f|, signed Voronoi-edge length h (interior: (c_t2 - c_t1).n;
    boundary: (c_f - c_t1).n, n the unit normal pointing out of t1), the Hodge entry
    *_f = max(h / |f|, limiter), and the geometric weight 1 / *_f."""
    xyz = np.asarray(xyz, dtype=np.float64)
    tets = np.asarray(tets, dtype=np.int64)
    t1, k1, t2, _, verts = faces
    p = xyz[tets]
    ct = circumcenter_tet(p[:, 0], p[:, 1], p[:, 2], p[:, 3])
    a, b, c = xyz[verts[:, 0]], xyz[verts[:, 1]], xyz[verts[:, 2]]
    n = np.cross(b - a, c - a)
    nn = np.sqrt((n * n).sum(axis=1))
    opp = p[t1, k1]
    sgn = np.where(((opp - a) * n).sum(axis=1) > 0.0, -1.0, 1.0)  # away from t1's opposite vertex
    unit = n * (sgn / nn)[:, None]
    area = 0.5 * nn
    cf = circumcenter_tri(a, b, c)
    far = np.where((t2 >= 0)[:, None], ct[np.maximum(t2, 0)], cf)
    h = ((far - ct[t1]) * unit).sum(axis=1)
    star = np.maximum(h / area, limiter)
    return {"area": area, "h": h, "star": star, "gw": 1.0 / star, "ct": ct, "cf": cf, "far": far}


def face_cut(xyz, tets, faces, geo, cracks):
    """A face is cut when its Voronoi edge (t1's circumcentre to t2's, or to the face's
    circumcentre on the boundary) crosses a penny disc (the predicate of the vertex path)."""
    cut = np.zeros(len(faces[0]), dtype=bool)
    if cracks is None or len(cracks) == 0:
        return cut
    p0 = geo["ct"][faces[0]]
    p1 = geo["far"]
    for d in np.asarray(cracks, dtype=np.float64).reshape(-1, 7):
        cut |= _cut_by_disc(p0, p1, d)
    return cut


def face_bc(faces, bc_type, bc_value, side):
    """Per boundary face: Dirichlet flag, T0 (mean of the vertex values), side (1/2/0),
    Neumann flag and f0 (mean of the vertices' outward flux densities)."""
    t2, verts = faces[2], faces[4]
    bt = np.asarray(bc_type)[verts]
    bv = np.asarray(bc_value, dtype=np.float64)[verts]
    sd = np.asarray(side)[verts] if side is not None else np.zeros_like(bt)
    dirichlet = (t2 < 0) & (bt == 1).all(axis=1)
    mean = ((bv[:, 0] + bv[:, 1]) + bv[:, 2]) / 3.0
    T0 = np.where(dirichlet, mean, 0.0)
    fside = np.where(dirichlet & (sd == 1).all(axis=1), 1, np.where(dirichlet & (sd == 2).all(axis=1), 2, 0))
    neumann = (t2 < 0) & (bt == 2).all(axis=1)
    f0 = np.where(neumann, mean, 0.0)
    return dirichlet, T0, fside, neumann, f0


def dual_system(xyz, tets, bc_type, bc_value, side=None, kappa=None, cracks=None, limiter=LIMITER):
    """The Schur complement on the tets: returns dict(L, b, W, pinned, faces, geo, dirichlet, T0,
    side).  Tets in parts joined to no Dirichlet face (over faces with W != 0) are pinned to 0."""
    tets = np.asarray(tets, dtype=np.int64)
    T = len(tets)
    faces = faces_by_owner(tets)
    t1, _, t2, _, _ = faces
    geo = face_geometry(xyz, tets, faces, limiter)
    kap = np.ones(len(t1)) if kappa is None else np.asarray(kappa, dtype=np.float64)
    kap = np.where(face_cut(xyz, tets, faces, geo, cracks), 0.0, kap)
    dirichlet, T0, fside, neumann, f0 = face_bc(faces, bc_type, bc_value, side)
    g = f0 * geo["area"]  # prescribed outward flux of the Neumann faces
    inner = t2 >= 0
    W = np.where(inner | dirichlet, kap * geo["gw"], 0.0)
    # pinning over the faces that conduct
    anchored = np.zeros(T, dtype=bool)
    anchored[t1[dirichlet & (W != 0.0)]] = True
    pinned = isolated_components(T, np.stack([t1[inner], t2[inner]], axis=1), W[inner], anchored)
    rows = np.concatenate([t1[inner], t2[inner], t1[inner], t2[inner], t1[dirichlet]])
    cols = np.concatenate([t2[inner], t1[inner], t1[inner], t2[inner], t1[dirichlet]])
    vals = np.concatenate([-W[inner], -W[inner], W[inner], W[inner], W[dirichlet]])
    L = sp.csr_matrix((vals, (rows, cols)), shape=(T, T))
    b = np.bincount(t1[dirichlet], weights=W[dirichlet] * T0[dirichlet], minlength=T)
    b = b - np.bincount(t1[neumann], weights=g[neumann], minlength=T)
    # pinned parts: unit rows, zero right-hand side (they touch no conducting face)
    L = L.tolil()
    for t in np.flatnonzero(pinned):
        L.rows[t], L.data[t] = [t], [1.0]
    L = L.tocsr()
    b[pinned] = 0.0
    return {"L": L, "b": b, "W": W, "pinned": pinned, "faces": faces, "geo": geo, "dirichlet": dirichlet,
            "T0": T0, "side": fside, "kappa": kap, "neumann": neumann, "g": g}


def mixed_system(xyz, tets, bc_type, bc_value, side=None, kappa=None, cracks=None, limiter=LIMITER):
    """Eq. 11-13 written out: unknowns [omega (faces); alpha (tets)], the (1,1) block
    (1/kappa_f) *_f, d the tet-face incidence (+1 for the owner t1, -1 for t2), Dirichlet
    faces moving T0 to the right-hand side, Neumann faces fixing omega_f = -g_f (omega
    is the flux into t1) in their own row and keeping their entry in t1's balance,
    insulated and cracked faces replaced by unit rows and columns (zero flux).  Pinned
    tets (as in dual_system) get unit rows, and their Neumann faces count as insulated."""
    s = dual_system(xyz, tets, bc_type, bc_value, side, kappa, cracks, limiter)
    t1, _, t2, _, _ = s["faces"]
    F, T = len(t1), len(tets)
    star, kap = s["geo"]["star"], s["kappa"]
    inner = t2 >= 0
    live = (inner | s["dirichlet"]) & (kap != 0.0)
    rows, cols, vals = [], [], []
    rhs = np.zeros(F + T)
    for f in range(F):
        if s["neumann"][f] and not s["pinned"][t1[f]]:
            rows += [f, F + t1[f]]
            cols += [f, f]
            vals += [1.0, 1.0]
            rhs[f] = -s["g"][f]
            continue
        if not live[f]:
            rows.append(f), cols.append(f), vals.append(1.0)
            continue
        rows.append(f), cols.append(f), vals.append(star[f] / kap[f])
        # (d^T alpha)_f = alpha_t1 - alpha_t2, or alpha_t1 - T0 on a Dirichlet face
        rows += [f, F + t1[f]]
        cols += [F + t1[f], f]
        vals += [1.0, 1.0]
        if inner[f]:
            rows += [f, F + t2[f]]
            cols += [F + t2[f], f]
            vals += [-1.0, -1.0]
        else:
            rhs[f] = s["T0"][f]
    for t in np.flatnonzero(s["pinned"]):
        rows.append(F + t), cols.append(F + t), vals.append(1.0)
    K = sp.csr_matrix((vals, (rows, cols)), shape=(F + T, F + T))
    return K, rhs, s


def solve(s):
    """Direct solve of the tet system (library sparse LU)."""
    return spla.spsolve(s["L"].tocsc(), s["b"])


def flux(T, s, length=1.0, area=1.0, dT=1.0):
    """k_eff (energy form), Q_in, Q_out of the tet solution."""
    T = np.asarray(T, dtype=np.float64)
    t1, _, t2, _, _ = s["faces"]
    W, dirichlet, T0, side = s["W"], s["dirichlet"], s["T0"], s["side"]
    inner = t2 >= 0
    d_in = T[t1[inner]] - T[t2[inner]]
    d_bc = T[t1[dirichlet]] - T0[dirichlet]
    energy = float((W[inner] * d_in * d_in).sum() + (W[dirichlet] * d_bc * d_bc).sum())
    q_in = float((W * (T0 - T[t1]))[dirichlet & (side == 1)].sum())
    q_out = float((W * (T[t1] - T0))[dirichlet & (side == 2)].sum())
    return {"k_eff": energy * length / (area * dT * dT), "q_in": q_in, "q_out": q_out, "energy": energy}


def rms_error_tets(xyz, tets, T, field=(1.0, -1.0, 0.0, 0.0)):
    """Eq. 15, the paper's verification error: sqrt(sum over tets of V_t (T_t - T_exact)^2), T_exact
    the linear field a + g.p at the tet's circumcentre (its Voronoi vertex), V_t its volume."""
    xyz = np.asarray(xyz, dtype=np.float64)
    p = xyz[np.asarray(tets, dtype=np.int64)]
    c = circumcenter_tet(p[:, 0], p[:, 1], p[:, 2], p[:, 3])
    vol = np.abs(np.einsum("ij,ij->i", np.cross(p[:, 1] - p[:, 0], p[:, 2] - p[:, 0]), p[:, 3] - p[:, 0])) / 6.0
    a, g = field[0], np.asarray(field[1:], dtype=np.float64)
    d = np.asarray(T, dtype=np.float64) - (a + c @ g)
    return float(np.sqrt((vol * d * d).sum()))
