"""Pins of the oracle of the paper's own unknowns (temperature on the tets, flux through the
triangles; Section 2.3, eq. 11-13; the 1e-8 Hodge limiter of Section 3.1).  CPU only."""
import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

import oracle as O
import workloads as W
from oracle import dual as D


def _kuhn(n):
    xyz, tets = W.kuhn_cube(n)
    bt, bv, side = W.x_sides(n)
    return xyz, tets, bt, bv, side


def _with_neumann(xyz, bt, bv, seed):
    """Neumann data (type 2, outward flux densities) on the vertices of the face y = 0 that carry
    no Dirichlet data."""
    bt, bv = bt.copy(), bv.copy()
    on = (np.abs(xyz[:, 1]) < 1e-12) & (bt != 1)
    bt[on] = 2
    bv[on] = np.random.Generator(np.random.PCG64(seed)).normal(0.0, 1.0, on.sum())
    return bt, bv


def _neumann_inflow(n):
    """T = 0 on x = 1 (Dirichlet), outward flux density -1 on x = 0 (an inflow of 1 through the
    unit face), insulated elsewhere: the continuous solution is 1 - x."""
    xyz, tets = W.kuhn_cube(n)
    i = W.lattice_index(n)[0]
    bt = np.where(i == n, 1, np.where(i == 0, 2, 0)).astype(np.int8)
    bv = np.where(i == 0, -1.0, 0.0)
    side = np.where(i == n, 2, 0).astype(np.int8)
    return xyz, tets, bt, bv, side


def test_faces_by_owner():
    for n in (1, 2, 3):
        xyz, tets, *_ = _kuhn(n)
        t1, k1, t2, k2, verts = D.faces_by_owner(tets)
        assert len(t1) == W.kuhn_counts(n)["F"] and int((t2 < 0).sum()) == 12 * n * n
        inner = t2 >= 0
        assert (t1[inner] < t2[inner]).all()
        for f in np.flatnonzero(inner)[:50]:
            a = set(tets[t1[f]]) - {tets[t1[f], k1[f]]}
            b = set(tets[t2[f]]) - {tets[t2[f], k2[f]]}
            assert a == b == set(verts[f])
        assert sorted(zip(t1, k1)) == list(zip(t1, k1))  # owner order


def test_kuhn_dual_edge_lengths_and_the_limited_faces():
    """Kuhn cubes: the six tets of a cube share its centre as circumcentre, so exactly the 6 n^3
    faces inside the cubes have zero Voronoi length (and are limited); the others measure the
    lattice spacing h between cube centres, h/2 from a cube centre to a boundary face."""
    for n in (2, 3, 5):
        xyz, tets, bt, bv, side = _kuhn(n)
        s = D.dual_system(xyz, tets, bt, bv, side)
        h, area, t2 = s["geo"]["h"], s["geo"]["area"], s["faces"][2]
        limited = h / area < D.LIMITER
        assert limited.sum() == 6 * n ** 3 and np.abs(h[limited]).max() < 1e-14
        assert np.allclose(h[~limited & (t2 >= 0)], 1.0 / n, rtol=1e-12)
        assert np.allclose(h[t2 < 0], 0.5 / n, rtol=1e-12)
        assert np.array_equal(s["geo"]["star"][limited], np.full(limited.sum(), D.LIMITER))


def test_schur_complement_of_the_mixed_system():
    """Eliminating the face fluxes from eq. 11-13 (the (1,1) block is diagonal) gives exactly
    the tet operator and right-hand side: S = -L, r = -b (jittered mesh, lognormal
    conductivity, cracks, Dirichlet and Neumann faces, limited entries)."""
    n = 3
    xyz, tets, bt, bv, side = _kuhn(n)
    xj = W.jitter_interior(xyz, n, 0.2, 3)
    cr = W.penny_cracks(6, 2, 0.1, 0.3)
    F = W.kuhn_counts(n)["F"]
    kap = np.random.Generator(np.random.PCG64(1)).lognormal(0.0, 1.0, F)
    bt, bv = _with_neumann(xj, bt, bv, 4)
    K, rhs, s = D.mixed_system(xj, tets, bt, bv, side, kappa=kap, cracks=cr)
    assert (s["kappa"] == 0).any() and (s["geo"]["h"] < 0).any() and s["neumann"].sum() == 2 * (n - 2) * n
    K = K.tocsr()
    # a Neumann face's row fixes its flux and has no tet column, so the tets' rows are
    # taken as they stand (B2) rather than as the transpose of the faces' columns
    A, B, B2, C = K[:F, :F], K[:F, F:], K[F:, :F], K[F:, F:]
    Ainv = sp.diags(1.0 / A.diagonal())
    S = (C - B2 @ Ainv @ B).toarray()
    L = s["L"].toarray()
    assert np.abs(S + L).max() <= 1e-14 * np.abs(L).max()
    assert np.abs(rhs[F:] - B2 @ (Ainv @ rhs[:F]) + s["b"]).max() <= 1e-14 * np.abs(s["b"]).max()
    assert np.allclose(L, L.T, rtol=0, atol=1e-15 * np.abs(L).max())


def test_limiter_sets_the_error_of_the_linear_solution():
    """Homogeneous Kuhn cube: with the limited Voronoi lengths the saddle system's solution
    deviates from the exact linear field by an amount proportional to the limit (the paper's
    non-machine-zero error), and k_eff = 1 up to the same order."""
    n = 3
    xyz, tets, bt, bv, side = _kuhn(n)
    errs = []
    for lim in (1e-6, 1e-8, 1e-10):
        K, rhs, s = D.mixed_system(xyz, tets, bt, bv, side, limiter=lim)
        T = spla.spsolve(K.tocsc(), rhs)[len(s["W"]):]
        err = np.abs(T - (1.0 - s["geo"]["ct"][:, 0])).max()
        errs.append(err)
        assert 0.05 * lim < err < 0.5 * lim
        assert abs(D.flux(T, s)["k_eff"] - 1.0) < 3.0 * lim
    assert 80 < errs[0] / errs[1] < 120 and 80 < errs[1] / errs[2] < 120


def test_neumann_inflow_is_conserved_and_gives_the_linear_field():
    """A prescribed inflow (outward flux density -1 on x = 0) with T = 0 on x = 1: summing the
    tet balances, the interior faces cancel, so the Dirichlet outflow equals the inflow, 1, on
    any mesh and conductivity (jittered, lognormal, cracked), up to the direct solve's
    residual (the limited weights, ~kappa / 1e-8, leave it near 1e-8 of the inflow); on the
    homogeneous cube the solution is the linear field 1 - x up to the limiter's error."""
    n = 4
    xyz, tets, bt, bv, side = _neumann_inflow(n)
    s = D.dual_system(xyz, tets, bt, bv, side)
    assert s["neumann"].sum() == 2 * n * n and abs(s["g"][s["neumann"]].sum() + 1.0) < 1e-14
    T = D.solve(s)
    assert np.abs(T - (1.0 - s["geo"]["ct"][:, 0])).max() < 1e-6
    assert abs(D.flux(T, s)["q_out"] - 1.0) < 1e-6
    xj = W.jitter_interior(xyz, n, 0.2, 8)
    kap = np.random.Generator(np.random.PCG64(2)).lognormal(0.0, 1.0, W.kuhn_counts(n)["F"])
    s2 = D.dual_system(xj, tets, bt, bv, side, kappa=kap, cracks=W.penny_cracks(3, 5, 0.05, 0.15))
    assert not s2["pinned"].any()
    T2 = D.solve(s2)
    assert abs(D.flux(T2, s2)["q_out"] - 1.0) < 1e-6
    # the literal saddle system gives the same solution, up to what rounding leaves of two
    # direct solves beside weights near kappa / 1e-8 (about 1e-7 here, as with Dirichlet data
    # on both sides; the matrices themselves agree to 1e-14, test_schur_complement_...)
    K, rhs, s3 = D.mixed_system(xj, tets, bt, bv, side, kappa=kap, cracks=W.penny_cracks(3, 5, 0.05, 0.15))
    T3 = spla.spsolve(K.tocsc(), rhs)[len(s3["W"]):]
    assert np.abs(T3 - T2).max() < 1e-5 * np.abs(T2).max()


def test_energy_identity_and_cracks_lower_the_conductivity():
    n = 4
    xyz, tets, bt, bv, side = _kuhn(n)
    xj = W.jitter_interior(xyz, n, 0.15, 5)
    K, rhs, s = D.mixed_system(xj, tets, bt, bv, side)
    T = spla.spsolve(K.tocsc(), rhs)[len(s["W"]):]
    f = D.flux(T, s)
    assert abs(f["q_in"] - f["energy"]) < 1e-6 * f["energy"] and abs(f["q_out"] - f["energy"]) < 1e-6 * f["energy"]
    K2, rhs2, s2 = D.mixed_system(xj, tets, bt, bv, side, cracks=W.penny_cracks(5, 4, 0.15, 0.3))
    T2 = spla.spsolve(K2.tocsc(), rhs2)[len(s2["W"]):]
    assert (s2["kappa"] == 0).any() and D.flux(T2, s2)["k_eff"] < f["k_eff"]


def test_rms_error_of_eq15():
    """Zero on the exact linear values, |delta| for a constant shift on the unit cube (the
    volumes sum to 1), and one tet by hand."""
    xyz, tets, *_ = _kuhn(3)
    p = xyz[tets]
    ct = O.circumcenter_tet(p[:, 0], p[:, 1], p[:, 2], p[:, 3])
    exact = 1.0 - ct[:, 0]
    assert D.rms_error_tets(xyz, tets, exact) == 0.0
    assert abs(D.rms_error_tets(xyz, tets, exact + 1e-3) - 1e-3) < 1e-15
    one = np.array([[0.0, 0, 0], [2, 0, 0], [0, 2, 0], [0, 0, 2]])
    # circumcentre (1, 1, 1), volume 8/6; field 2x + 3y: exact 5 there, T = 7
    assert abs(D.rms_error_tets(one, [[0, 1, 2, 3]], [7.0], (0.0, 2.0, 3.0, 0.0)) - 2.0 * np.sqrt(8 / 6)) < 1e-14


def _linear_residual(xyz, tets, g=(0.3, -0.7, 0.55), a=0.2):
    """(L u)_t for u = a + g.c_t (the linear field at the Voronoi nodes) over the tets whose four
    faces are interior and unlimited, with the scale sum_f W_f |u_t - u_t'|, and that count."""
    bt, bv, side = W.x_faces(xyz)
    s = D.dual_system(xyz, tets, bt, bv, side)
    t1, _, t2, _, _ = s["faces"]
    geo = s["geo"]
    lim = geo["h"] / geo["area"] <= D.LIMITER
    excluded = np.zeros(len(tets), dtype=bool)
    excluded[t1[(t2 < 0) | lim]] = True
    excluded[t2[(t2 >= 0) & lim]] = True
    u = a + geo["ct"] @ np.asarray(g)
    Lu = s["L"] @ u
    inner = t2 >= 0
    d = np.abs(u[t1[inner]] - u[t2[inner]]) * s["W"][inner]
    scale = np.zeros(len(tets))
    np.add.at(scale, t1[inner], d)
    np.add.at(scale, t2[inner], d)
    keep = ~excluded
    return Lu[keep], scale[keep], int(keep.sum())


def test_linear_fields_are_exact_at_interior_voronoi_nodes():
    """Off the lattice (Delaunay meshes of a jittered lattice and of random points): for a tet
    whose four faces are interior and unlimited, the flux balance of a linear field u = a + g.x
    taken at the circumcentres vanishes, (L u)_t = sum_f (|f| / h_f)(u_t - u_t') = -g . sum_f |f| n_f
    = 0, because the Voronoi edge through a face is orthogonal to it (c_t' - c_t = h_f n_f with n_f
    the unit normal out of t) and the outward area vectors of a closed surface sum to zero
    (Section 3.1: exact for linear solutions where nothing is limited).  A wrong normal sign
    limits almost every face (the count below), a wrong area or length breaks the balance."""
    for xyz, tets in (W.delaunay_lattice(8, 0.2, 1), W.delaunay_lattice(8, 0.2, 2), W.delaunay_cube(600, 60, 3)):
        Lu, scale, count = _linear_residual(xyz, tets)
        assert count >= 0.7 * len(tets), (count, len(tets))
        assert (np.abs(Lu) <= 1e-9 * scale).all(), np.max(np.abs(Lu) / scale)
        assert np.median(np.abs(Lu) / scale) <= 1e-13


def test_one_interior_face_by_hand():
    """Two tets sharing the face (1,0,0), (0,1,0), (0,0,1): t1 has the origin as its fourth vertex
    and circumcentre (1/2, 1/2, 1/2); t2 has (2,2,2), and its circumcentre s(1,1,1) satisfies
    (s - 1)^2 + 2 s^2 = 3 (s - 2)^2, s = 11/10.  Face area sqrt(3)/2; the unit normal out of t1 is
    (1,1,1)/sqrt(3), so h = 0.6 sqrt(3) and *_f = h / |f| = 1.2.  A boundary face of t1, the one in
    the plane x = 0: area 1/2, circumcentre (0, 1/2, 1/2), h = 1/2 along (-1, 0, 0), *_f = 1."""
    xyz = np.array([[0.0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1], [2, 2, 2]])
    tets = np.array([[0, 1, 2, 3], [1, 2, 3, 4]])
    faces = D.faces_by_owner(tets)
    geo = D.face_geometry(xyz, tets, faces)
    t1, k1, t2, _, verts = faces
    assert np.allclose(geo["ct"], [[0.5, 0.5, 0.5], [1.1, 1.1, 1.1]], rtol=0, atol=1e-15)
    f = int(np.flatnonzero(t2 >= 0)[0])
    assert (t1[f], t2[f], set(verts[f])) == (0, 1, {1, 2, 3})
    assert abs(geo["area"][f] - np.sqrt(3) / 2) <= 1e-15
    assert abs(geo["h"][f] - 0.6 * np.sqrt(3)) <= 1e-15
    assert abs(geo["star"][f] - 1.2) <= 1e-15
    b = [i for i in np.flatnonzero(t2 < 0) if t1[i] == 0 and set(verts[i]) == {0, 2, 3}][0]
    assert abs(geo["area"][b] - 0.5) <= 1e-16 and abs(geo["h"][b] - 0.5) <= 1e-16
    assert np.allclose(geo["cf"][b], [0.0, 0.5, 0.5], rtol=0, atol=1e-16) and abs(geo["star"][b] - 1.0) <= 1e-15
