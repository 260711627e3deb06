"""Pins of the spatial-numbering oracle (Section 2.2's location sort).  CPU only."""
import numpy as np

import oracle as O
import workloads as W
from oracle.reorder import cells_per_axis, point_cells


def test_cells_per_axis_is_the_first_cube():
    for V, B in [(1, 1), (2, 2), (8, 2), (9, 3), (27, 3), (28, 4), (4913, 17), (4914, 18), (2146689, 129)]:
        assert cells_per_axis(V) == B


def test_kuhn_lattice_order_is_kept():
    """Kuhn vertices are numbered k + (n+1)(j + (n+1) i) (z fastest) and cube-major tets: the
    sort gives both numberings back unchanged."""
    for n in (1, 2, 5, 8):
        xyz, tets = W.kuhn_cube(n)
        x2, t2, vp, tp = O.spatial_order(xyz, tets)
        assert np.array_equal(vp, np.arange(len(xyz))) and np.array_equal(tp, np.arange(len(tets)))
        assert np.array_equal(x2, xyz) and np.array_equal(t2, tets)


def test_shuffled_lattice_is_restored():
    n = 6
    xyz, tets = W.kuhn_cube(n)
    rng = np.random.Generator(np.random.PCG64(3))
    p = rng.permutation(len(xyz))       # new position of old vertex
    q = rng.permutation(len(tets))
    inv = np.argsort(p)
    xs = xyz[inv]                        # vertex p[v] holds old v
    ts = p[tets][q]
    x2, t2, vp, tp = O.spatial_order(xs, ts)
    assert np.array_equal(x2, xyz)      # one point per cell: the lattice order again
    # the same tets (as vertex sets) in cube order; within a cube, by shuffled index
    assert sorted(map(tuple, np.sort(t2, axis=1))) == sorted(map(tuple, np.sort(tets, axis=1)))
    assert np.array_equal(np.sort(t2.min(axis=1)), t2.min(axis=1))
    assert np.array_equal(xs[vp], x2) and np.array_equal(t2, np.argsort(vp)[ts[tp]])


def test_order_is_by_cell_then_index():
    """Random points: the cell keys of the new order are non-decreasing in (x, y, z) cell order
    and equal keys keep their original order; every tet keeps its vertex order."""
    xyz, tets = W.delaunay_cube(400, 40, 5)
    x2, t2, vp, tp = O.spatial_order(xyz, tets)
    B = cells_per_axis(len(xyz))
    c = point_cells(xyz, B)[vp]
    key = (c[:, 0] * B + c[:, 1]) * B + c[:, 2]
    assert (np.diff(key) >= 0).all()
    same = np.diff(key) == 0
    assert (np.diff(vp)[same] > 0).all()
    inv = np.argsort(vp)
    assert np.array_equal(t2, inv[tets[tp]])
    m = t2.min(axis=1)
    assert (np.diff(m) >= 0).all() and (np.diff(tp)[np.diff(m) == 0] > 0).all()


def test_flat_and_degenerate_boxes():
    xyz = np.array([[0.0, 0.0, 0.5], [1.0, 0.0, 0.5], [0.0, 1.0, 0.5], [1.0, 1.0, 0.5]])
    c = point_cells(xyz, 2)
    assert (c[:, 2] == 0).all() and np.array_equal(c[:, 0], [0, 1, 0, 1])


def test_morton_keys_and_octants():
    """The interleave against bit-by-bit Python arithmetic; on a 4^3 lattice the Z order visits
    each 2x2x2 octant as one run of 8 points, octants in Z order themselves."""
    from oracle.reorder import morton_key
    rng = np.random.Generator(np.random.PCG64(2))
    c = rng.integers(0, 1 << 20, size=(50, 3))
    for row, k in zip(c, morton_key(c)):
        want = 0
        for b in range(21):
            want |= ((int(row[0]) >> b) & 1) << (3 * b + 2)
            want |= ((int(row[1]) >> b) & 1) << (3 * b + 1)
            want |= ((int(row[2]) >> b) & 1) << (3 * b)
        assert int(k) == want
    xyz, tets = W.kuhn_cube(3)
    x2, t2, vp, tp = O.spatial_order(xyz, tets, order="morton")
    cells = np.rint(x2 * 3).astype(int)  # lattice coordinates in the new order
    octant = (cells // 2) @ np.array([4, 2, 1])
    assert np.array_equal(octant, np.repeat(np.arange(8), 8))
    assert np.array_equal(np.sort(vp), np.arange(len(xyz)))
    m = t2.min(axis=1)
    assert (np.diff(m) >= 0).all() and np.array_equal(t2, np.argsort(vp)[tets[tp]])
