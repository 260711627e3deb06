"""Pins of the oracle's topology against closed forms, invariants and brute force (CPU)."""
import itertools

import numpy as np
import pytest

import oracle as O
import workloads as W


@pytest.mark.parametrize("n", [1, 2, 3, 4, 5, 8])
def test_kuhn_counts_closed_form(n):
    xyz, tets = W.kuhn_cube(n)
    V = len(xyz)
    E = O.edges_of(tets, V)
    F, count = O.faces_of(tets)
    c = W.kuhn_counts(n)
    assert (V, len(tets), len(E), len(F)) == (c["V"], c["T"], c["E"], c["F"])
    # Euler characteristic of a ball: V - E + F - T = 1
    assert V - len(E) + len(F) - len(tets) == 1
    # boundary faces: 2 triangles per boundary square, 6 n^2 squares
    assert int((count == 1).sum()) == 12 * n * n
    assert count.max() == 2


def test_kuhn_counts_table_sizes():
    # sizes of the 16^3, 128^3 and 256^3 workloads
    assert W.kuhn_counts(16)["E"] == 31024 and W.kuhn_counts(16)["nnz"] == 66961
    assert W.kuhn_counts(128)["E"] == 14827904 and W.kuhn_counts(128)["nnz"] == 31802497
    assert W.kuhn_counts(256)["V"] == 16974593 and W.kuhn_counts(256)["E"] == 118031104


@pytest.mark.parametrize("n", [1, 2, 3])
def test_edges_brute_force(n):
    xyz, tets = W.kuhn_cube(n)
    want = set()
    for t in tets:
        for a, b in itertools.combinations([int(v) for v in t], 2):
            want.add((min(a, b), max(a, b)))
    got = O.edges_of(tets, len(xyz))
    assert [tuple(e) for e in got.tolist()] == sorted(want)
    ids = O.tet_edge_ids(tets, len(xyz), got)
    for t, row in zip(tets, ids):
        for q, (i, j) in enumerate(O.LOCAL_EDGES):
            lo, hi = sorted((int(t[i]), int(t[j])))
            assert tuple(got[row[q]]) == (lo, hi)


@pytest.mark.parametrize("n", [2, 3, 4])
def test_d1_d0_is_zero(n):
    xyz, tets = W.kuhn_cube(n)
    V = len(xyz)
    E = O.edges_of(tets, V)
    F, _ = O.faces_of(tets)
    d0 = O.d0_matrix(E, V)
    d1 = O.d1_matrix(F, E, V)
    assert abs(d1 @ d0).max() == 0
    # every face has three edges with coefficients +1, -1, +1
    assert np.all(np.diff(d1.indptr) == 3)
    assert sorted(np.unique(d1.data).tolist()) == [-1.0, 1.0]


def test_degree_histogram_n3():
    xyz, tets = W.kuhn_cube(3)
    E = O.edges_of(tets, len(xyz))
    deg = O.vertex_degrees(E, len(xyz))
    hist = dict(zip(*np.unique(deg, return_counts=True)))
    assert {int(k): int(v) for k, v in hist.items()} == {4: 6, 6: 12, 7: 2, 8: 12, 10: 24, 14: 8}


def test_degree_interior_and_corners():
    n = 4
    xyz, tets = W.kuhn_cube(n)
    E = O.edges_of(tets, len(xyz))
    deg = O.vertex_degrees(E, len(xyz))
    i, j, k = W.lattice_index(n)
    interior = (i > 0) & (i < n) & (j > 0) & (j < n) & (k > 0) & (k < n)
    assert np.all(deg[interior] == 14)
    corners = {(0, 0, 0): 7, (n, n, n): 7}
    for c in itertools.product([0, n], repeat=3):
        v = c[2] + (n + 1) * (c[1] + (n + 1) * c[0])
        assert deg[v] == corners.get(c, 4)


def test_check_mesh_errors():
    xyz, tets = W.kuhn_cube(2)
    assert O.check_mesh(xyz, tets) is None
    bad = tets.copy()
    bad[3, 2] = len(xyz)
    assert O.check_mesh(xyz, bad) == "index out of range"
    bad = tets.copy()
    bad[5, 1] = bad[5, 0]
    assert O.check_mesh(xyz, bad) == "repeated vertex"
    flat = xyz.copy()
    flat[:, 2] = 0.0
    assert O.check_mesh(flat, tets) == "zero volume"
    dup = np.concatenate([tets, tets[:1]])
    assert O.check_mesh(xyz, dup) == "face shared by more than two tets"
    for v in (np.nan, np.inf):
        odd = xyz.copy()
        odd[7, 1] = v
        assert O.check_mesh(odd, tets) == "non-finite coordinate"


def test_boundary_faces_match_face_counts():
    xyz, tets = W.kuhn_cube(3)
    bf = O.boundary_faces(tets)
    assert len(bf) == 12 * 9
    # every boundary face lies in one of the planes x, y or z in {0, 1}
    for t, k in bf:
        verts = [int(tets[t, r]) for r in O.topology.LOCAL_FACES[k]]
        p = xyz[verts]
        assert any(np.all(p[:, a] == p[0, a]) and p[0, a] in (0.0, 1.0) for a in range(3))
