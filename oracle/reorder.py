"""Oracle of the spatial numbering (test infrastructure only).

Section 2.2: a pre-processing step numbers the Delaunay nodes by their
location in space, z first, then y, then x, so that blocks of consecutive
nodes are compact.  Reading for points off a lattice: the bounding box is cut
into B^3 cells, B the smallest integer with B^3 >= V; a point's cell on axis a
is floor((x_a - lo_a) * (B / (hi_a - lo_a))) clamped to [0, B-1] (0 on a flat
axis); points are sorted by (x cell, y cell, z cell) with the z cell varying
fastest, ties by original index.  Tets are sorted by their smallest new vertex
number, ties by original index, and keep their vertex order.  The Z (Morton)
order is offered beside it: cells by the interleaved bits of (x cell, y cell,
z cell), z in the lowest bit.
"""
import numpy as np


def cells_per_axis(V):
    """The smallest B with B^3 >= V (exact integer search)."""
    B = max(1, int(round(float(V) ** (1.0 / 3.0))))
    while B ** 3 < V:
        B += 1
    while B > 1 and (B - 1) ** 3 >= V:
        B -= 1
    return B


def point_cells(xyz, B):
    """[V, 3] cell coordinates of every point."""
    xyz = np.asarray(xyz, dtype=np.float64)
    lo, hi = xyz.min(axis=0), xyz.max(axis=0)
    ext = hi - lo
    s = np.where(ext > 0.0, float(B) / np.where(ext > 0.0, ext, 1.0), 0.0)
    c = np.floor((xyz - lo) * s)
    return np.clip(np.nan_to_num(c, nan=0.0), 0, B - 1).astype(np.int64)


def morton_key(c):
    """Interleaved bits of the [N, 3] cell coordinates: bit b of x at 3b + 2, of y at 3b + 1,
    of z at 3b."""
    c = np.asarray(c, dtype=np.uint64)
    key = np.zeros(len(c), dtype=np.uint64)
    for b in range(21):
        for axis, shift in ((0, 2), (1, 1), (2, 0)):
            bit = (c[:, axis] >> np.uint64(b)) & np.uint64(1)
            key |= bit << np.uint64(3 * b + shift)
    return key


def spatial_order(xyz, tets, order="lexicographic"):
    """(xyz_new, tets_new, vperm, tperm): vperm[new] = old vertex, tperm[new] = old tet."""
    xyz = np.asarray(xyz, dtype=np.float64)
    tets = np.asarray(tets, dtype=np.int64)
    V = len(xyz)
    c = point_cells(xyz, cells_per_axis(V))
    if order == "morton":
        vperm = np.lexsort((np.arange(V), morton_key(c)))
    else:
        vperm = np.lexsort((np.arange(V), c[:, 2], c[:, 1], c[:, 0]))  # last key is the primary one
    inv = np.empty(V, dtype=np.int64)
    inv[vperm] = np.arange(V)
    relabel = inv[tets]
    tperm = np.lexsort((np.arange(len(tets)), relabel.min(axis=1)))
    return xyz[vperm], relabel[tperm].astype(np.int32), vperm.astype(np.int32), tperm.astype(np.int32)
