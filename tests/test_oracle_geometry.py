"""Pins of the oracle's circumcentres, dual areas and *1 (CPU)."""
import numpy as np
import pytest

import oracle as O
import workloads as W


def _rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


def _near_regular_tets(count, seed, amp=0.15):
    reg = np.array([[1, 1, 1], [1, -1, -1], [-1, 1, -1], [-1, -1, 1]], dtype=float)
    rng = _rng(seed)
    P = reg[None] + amp * rng.uniform(-1, 1, size=(count, 4, 3))
    return P.reshape(-1, 3), np.arange(4 * count).reshape(-1, 4)


def test_circumcentres_equidistant():
    rng = _rng(1)
    P = rng.normal(size=(200, 4, 3))
    c = O.circumcenter_tet(P[:, 0], P[:, 1], P[:, 2], P[:, 3])
    d = np.linalg.norm(P - c[:, None, :], axis=2)
    assert np.allclose(d, d[:, :1], rtol=1e-8)
    cf = O.circumcenter_tri(P[:, 0], P[:, 1], P[:, 2])
    df = np.linalg.norm(P[:, :3] - cf[:, None, :], axis=2)
    assert np.allclose(df, df[:, :1], rtol=1e-9)
    # the triangle's circumcentre lies in its plane
    nrm = np.cross(P[:, 1] - P[:, 0], P[:, 2] - P[:, 0])
    off = np.abs(((cf - P[:, 0]) * nrm).sum(1)) / np.linalg.norm(nrm, axis=1)
    assert off.max() < 1e-9 * np.abs(P).max()


def test_regular_tet_weights():
    # all six weights equal l / (12 sqrt 2); edge length 2 sqrt 2 gives 1/6
    p = np.array([[1, 1, 1], [1, -1, -1], [-1, 1, -1], [-1, -1, 1]], dtype=float)
    area = O.elementary_dual_areas(p, np.array([[0, 1, 2, 3]]))[0]
    l = 2 * np.sqrt(2)
    assert np.allclose(area / l, l / (12 * np.sqrt(2)), rtol=1e-14)


def test_well_centred_area_equals_polygon_area():
    xyz, tets = _near_regular_tets(300, 2)
    area = O.elementary_dual_areas(xyz, tets)
    P = xyz[tets]
    ct = O.circumcenter_tet(P[:, 0], P[:, 1], P[:, 2], P[:, 3])
    # well-centred: circumcentre inside (positive barycentric coordinates)
    M = np.stack([P[:, 1] - P[:, 0], P[:, 2] - P[:, 0], P[:, 3] - P[:, 0]], axis=2)
    lam = np.linalg.solve(M, (ct - P[:, 0])[..., None])[..., 0]
    assert np.all(lam > 0) and np.all(lam.sum(1) < 1)
    for q, (i, j) in enumerate(O.LOCAL_EDGES):
        k, l = [r for r in range(4) if r not in (i, j)]
        m = 0.5 * (P[:, i] + P[:, j])
        c1 = O.circumcenter_tri(P[:, i], P[:, j], P[:, k])
        c2 = O.circumcenter_tri(P[:, i], P[:, j], P[:, l])
        # quadrilateral (m, c1, cT, c2) as two triangles, unsigned areas by cross products
        a1 = 0.5 * np.linalg.norm(np.cross(c1 - m, ct - m), axis=1)
        a2 = 0.5 * np.linalg.norm(np.cross(ct - m, c2 - m), axis=1)
        assert np.allclose(area[:, q], a1 + a2, rtol=1e-11, atol=0)


def test_volume_identity_any_tet():
    # each tet splits into four signed vertex regions, each a union of pyramids of height |e|/2
    # over the edge's dual piece: vol(T) = (1/3) sum_e A_e^T |e|, also for obtuse tets
    rng = _rng(3)
    P = rng.normal(size=(500, 4, 3))
    xyz = P.reshape(-1, 3)
    tets = np.arange(2000).reshape(-1, 4)
    area = O.elementary_dual_areas(xyz, tets)
    lens = np.stack([np.linalg.norm(P[:, j] - P[:, i], axis=1) for i, j in O.LOCAL_EDGES], axis=1)
    vol = O.tet_volumes(xyz, tets)
    R = np.linalg.norm(P[:, 0] - O.circumcenter_tet(P[:, 0], P[:, 1], P[:, 2], P[:, 3]), axis=1)
    lhs = (area * lens).sum(1) / 3
    # rounding scales with circumradius^2 times edge length
    assert np.all(np.abs(lhs - vol) <= 1e-12 * (R * R * lens.max(1) + vol))
    assert (area < 0).any()  # the sample does contain non-well-centred tets


def test_orientation_independent():
    xyz, tets = _near_regular_tets(50, 4, amp=0.4)
    a = O.elementary_dual_areas(xyz, tets)
    perm = tets[:, [2, 0, 3, 1]]
    b = O.elementary_dual_areas(xyz, perm)
    # map local edges of the permuted tet back to the original local edges
    for q, (i, j) in enumerate(O.LOCAL_EDGES):
        oi, oj = sorted(([2, 0, 3, 1][i], [2, 0, 3, 1][j]))
        assert np.allclose(b[:, q], a[:, O.LOCAL_EDGES.index((oi, oj))], rtol=1e-12, atol=1e-15)


def _kuhn_star_expected(n, edges, xyz):
    """Closed forms on a Kuhn cube: axis edges h, h/2 on a boundary face, h/4 on a domain edge;
    face and body diagonals 0."""
    h = 1.0 / n
    d = xyz[edges[:, 1]] - xyz[edges[:, 0]]
    axis = (np.abs(d) > 0).sum(1) == 1
    m = 0.5 * (xyz[edges[:, 0]] + xyz[edges[:, 1]])
    on_bdry = ((m == 0.0) | (m == 1.0)).sum(1)  # boundary planes containing the edge
    want = np.where(axis, h / (2.0 ** on_bdry), 0.0)
    return want


@pytest.mark.parametrize("n", [2, 3, 4, 5, 6, 8, 16, 24])
def test_kuhn_star1_closed_forms(n):
    xyz, tets = W.kuhn_cube(n)
    E = O.edges_of(tets, len(xyz))
    s = O.hodge1(xyz, tets, E)
    want = _kuhn_star_expected(n, E, xyz)
    assert np.allclose(s, want, rtol=1e-12, atol=0)
    # zero-dual-area diagonals are exactly zero after the snap
    assert np.all(s[want == 0.0] == 0.0)


def test_snap_only_removes_rounding():
    n = 24  # not a power of two: diagonal dual areas come out as rounding noise
    xyz, tets = W.kuhn_cube(n)
    E = O.edges_of(tets, len(xyz))
    raw = O.dual_areas(xyz, tets, E, snap=False)
    snapped = O.dual_areas(xyz, tets, E, snap=True)
    l = O.edge_lengths(xyz, E)
    changed = raw != snapped
    assert changed.any()
    assert np.all(np.abs(raw[changed]) < 1e-14 * l[changed] ** 2)
    assert np.all(np.abs(snapped[snapped != 0]) > 0.1 * l[snapped != 0] ** 2)


def test_kappa_and_cut_scale_star1():
    n = 3
    xyz, tets = W.kuhn_cube(n)
    E = O.edges_of(tets, len(xyz))
    kap = W.lognormal_kappa(len(E), 1.0, 5)
    cut = np.zeros(len(E), dtype=bool)
    cut[::7] = True
    s0 = O.hodge1(xyz, tets, E)
    s = O.hodge1(xyz, tets, E, kappa=kap, cut=cut)
    assert np.all(s[cut] == 0.0)
    assert np.allclose(s[~cut], (kap * s0)[~cut], rtol=1e-15)


def test_boundary_dual_areas_partition_surface():
    for n in (2, 3, 5):
        xyz, tets = W.kuhn_cube(n)
        bf = O.boundary_faces(tets)
        A = O.boundary_dual_areas(xyz, tets, bf, len(xyz))
        assert abs(A.sum() - 6.0) < 1e-13  # surface of the unit cube
        i, j, k = W.lattice_index(n)
        # a vertex in the middle of a boundary face owns h^2 of it
        mid = (i == 0) & (j > 0) & (j < n) & (k > 0) & (k < n)
        assert np.allclose(A[mid], 1.0 / n ** 2, rtol=1e-13)
