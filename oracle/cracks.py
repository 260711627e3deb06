"""Oracle crack predicate: which edges a penny-shaped crack cuts (test infrastructure).

Section 2.5: a crack is an internal surface that stops heat transfer; it is
introduced by setting the conductivity of the dual faces it crosses to zero.
With penny-shaped discs (centre c, unit normal n, radius r), the dual face
of edge e = (p0, p1) is crossed when the segment p0 -> p1 passes through the
disc.  Predicate, evaluated in FP64 in exactly this operation order (both
implementations take the same integer decision):
    s0 = (p0x-cx)*nx + (p0y-cy)*ny + (p0z-cz)*nz, s1 likewise for p1;
    the endpoints are on different sides when (s0 < 0) != (s1 < 0)
    (an endpoint exactly on the plane counts as the non-negative side);
    t = s0 / (s0 - s1); q = p0 + t*(p1 - p0) per axis;
    cut when |q - c|^2 = (qx-cx)^2 + (qy-cy)^2 + (qz-cz)^2 <= r*r (rim inclusive).
p0 is the edge's lower vertex.
"""
import numpy as np


def _cut_by_disc(p0, p1, d):
    cx, cy, cz, nx, ny, nz, r = (float(v) for v in d)
    s0 = (p0[:, 0] - cx) * nx + (p0[:, 1] - cy) * ny + (p0[:, 2] - cz) * nz
    s1 = (p1[:, 0] - cx) * nx + (p1[:, 1] - cy) * ny + (p1[:, 2] - cz) * nz
    sides = (s0 < 0.0) != (s1 < 0.0)
    with np.errstate(divide="ignore", invalid="ignore"):
        t = s0 / (s0 - s1)
        qx = p0[:, 0] + t * (p1[:, 0] - p0[:, 0])
        qy = p0[:, 1] + t * (p1[:, 1] - p0[:, 1])
        qz = p0[:, 2] + t * (p1[:, 2] - p0[:, 2])
        d2 = (qx - cx) * (qx - cx) + (qy - cy) * (qy - cy) + (qz - cz) * (qz - cz)
    return sides & (d2 <= r * r)


def crack_cut(xyz, edges, cracks, edge_ids=None):
    """Boolean cut mask over ``edges`` (or over the subset ``edge_ids``) for a set of discs.

    ``cracks`` is [N, 7] rows (cx, cy, cz, nx, ny, nz, r).  An edge is cut if
    any disc cuts it.  Discs are tested against candidate edges whose
    midpoint x lies within r plus half the longest edge of the disc centre
    (plus a margin); no edge outside that slab can reach the disc, so the
    filter changes no result.
    """
    xyz = np.asarray(xyz, dtype=np.float64)
    edges = np.asarray(edges, dtype=np.int64)
    if edge_ids is not None:
        edges = edges[np.asarray(edge_ids, dtype=np.int64)]
    cut = np.zeros(len(edges), dtype=bool)
    cracks = np.asarray(cracks, dtype=np.float64).reshape(-1, 7)
    if len(edges) == 0 or len(cracks) == 0:
        return cut
    p0 = xyz[edges[:, 0]]
    p1 = xyz[edges[:, 1]]
    mx = 0.5 * (p0[:, 0] + p1[:, 0])
    half = 0.5 * np.sqrt(((p1 - p0) ** 2).sum(axis=1)).max()
    order = np.argsort(mx, kind="stable")
    mxs = mx[order]
    for d in cracks:
        reach = abs(float(d[6])) + half + 1e-9
        lo = np.searchsorted(mxs, d[0] - reach, side="left")
        hi = np.searchsorted(mxs, d[0] + reach, side="right")
        if hi <= lo:
            continue
        sel = order[lo:hi]
        hit = _cut_by_disc(p0[sel], p1[sel], d)
        cut[sel[hit]] = True
    return cut
