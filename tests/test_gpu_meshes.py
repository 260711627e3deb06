"""General tetrahedral meshes on the GPU: TetGen files in, the spatial numbering of Section 2.2,
and the eq. 15 verification error, against the oracle.

The numbering is integer work and must equal the oracle's bit for bit (permutations and the
reordered arrays).  A mesh read from TetGen files, renumbered and solved must give the oracle's
solution on the same arrays (FP64 Jacobi PCG to 1e-13 on both sides, T to 1e-9, k_eff to 1e-10),
and the same k_eff and temperatures as the unnumbered mesh (a renumbering only permutes the
system).  RMS errors agree with the oracle's to 1e-12 relative (a reduction in another order).
"""

import numpy as np
import pytest
import torch

import oracle as O
import workloads as W
from oracle import dual as D

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx(dev):
    import paper_2104_05999_amd as dec
    c = dec.Context(dev)
    yield c
    c.close()


def _t(a, dev):
    return torch.as_tensor(np.ascontiguousarray(a), device=dev)


def _shuffled_kuhn(n, seed):
    xyz, tets = W.kuhn_cube(n)
    rng = np.random.Generator(np.random.PCG64(seed))
    p = rng.permutation(len(xyz))
    q = rng.permutation(len(tets))
    return xyz[np.argsort(p)], p[tets][q].astype(np.int32)


CASES = {
    "kuhn5": lambda: W.kuhn_cube(5),
    "kuhn6_shuffled": lambda: _shuffled_kuhn(6, 3),
    "kuhn6_jittered": lambda: (W.jitter_interior(W.kuhn_cube(6)[0], 6, 0.2, 1), W.kuhn_cube(6)[1]),
    "delaunay": lambda: W.delaunay_cube(1500, 80, 7),
    # strongly graded towards one corner: 44% of the points share the first cell, so the ties by
    # original index decide most of the order
    "graded": lambda: (W.kuhn_cube(20)[0] ** 12, W.kuhn_cube(20)[1]),
}


@pytest.mark.parametrize("order", ["lexicographic", "morton"])
@pytest.mark.parametrize("name", list(CASES))
def test_reorder_matches_oracle(ctx, dev, name, order):
    xyz, tets = CASES[name]()
    xo, to, vp, tp = O.spatial_order(xyz, tets, order=order)
    xg, tg, vg, tpg = (a.cpu().numpy() for a in ctx.reorder(_t(xyz, dev), _t(tets, dev), order))
    assert np.array_equal(vg, vp) and np.array_equal(tpg, tp)
    assert np.array_equal(xg, xo) and np.array_equal(tg, to)


@pytest.mark.parametrize("order", ["lexicographic", "morton"])
def test_reorder_large_matches_oracle(ctx, dev, order):
    """The hand-written radix sort behind the numbering at a size where its blocks take long tiles
    (a shuffled Kuhn 112^3: 1.44M vertices, 8.43M tets, more tiles than the sort's block cap):
    vertex and tet permutations equal the oracle's bit for bit."""
    xyz, tets = _shuffled_kuhn(112, 5)
    xo, to, vp, tp = O.spatial_order(xyz, tets, order=order)
    xg, tg, vg, tpg = (a.cpu().numpy() for a in ctx.reorder(_t(xyz, dev), _t(tets, dev), order))
    assert np.array_equal(vg, vp) and np.array_equal(tpg, tp)
    assert np.array_equal(tg, to)


def test_reorder_rejects_bad_index(ctx, dev):
    import paper_2104_05999_amd as dec
    xyz, tets = W.kuhn_cube(2)
    bad = tets.copy()
    bad[5, 2] = len(xyz)
    with pytest.raises(dec.DecError):
        ctx.reorder(_t(xyz, dev), _t(bad, dev))
    # the context still works
    ctx.reorder(_t(xyz, dev), _t(tets, dev))


def _gpu_solve(ctx, dev, xyz, tets, kappa):
    bt, bv, side = W.x_faces(xyz)
    m = ctx.mesh(_t(xyz, dev), _t(tets, dev))
    try:
        edges = m.edges().cpu().numpy()
        m.hodge1(_t(kappa(edges), dev), want_cut=False, want_star=False)
        m.assemble()
        m.apply_bc(_t(bt, dev), _t(bv, dev), want_rhs=False)
        T, st, rc = m.solve(tol=1e-13, check=False)
        assert rc == 0, st
        f = m.flux(T, _t(side, dev))
        rms = m.rms_error(T)
        return T.cpu().numpy(), f, rms, edges
    finally:
        m.close()


def _oracle_solve(xyz, tets, kappa):
    bt, bv, side = W.x_faces(xyz)
    E = O.edges_of(tets, len(xyz))
    star = O.hodge1(xyz, tets, E, kappa=kappa(E))
    L, _ = O.assemble(len(xyz), E, star)
    A, b, _ = O.apply_bc(L, bt, bv, E, star)
    res = O.pcg(A, b, precond="jacobi", tol=1e-13)
    return res.x, O.flux_effective_conductivity(res.x, E, star, side)


def test_tetgen_mesh_renumbered_and_solved(ctx, dev, tmp_path):
    """A jittered Kuhn mesh with scrambled numbering -> TetGen files (1-based, with markers) -> read
    -> renumber -> the whole vertex path, against the oracle on the same arrays and against the
    unnumbered mesh.  (On random-point Delaunay meshes some circumcentric dual areas are negative
    and the vertex operator is indefinite; those meshes are the tet path's, below.)"""
    from paper_2104_05999_amd import read_tetgen
    n = 8
    xk, tk = W.kuhn_cube(n)
    xk = W.jitter_interior(xk, n, 0.15, 4)
    rng = np.random.Generator(np.random.PCG64(9))
    p = rng.permutation(len(xk))
    xyz0 = xk[np.argsort(p)]
    tets0 = p[tk][rng.permutation(len(tk))].astype(np.int32)
    node, ele = str(tmp_path / "cube.node"), str(tmp_path / "cube.ele")
    with open(node, "w") as f:
        f.write(f"{len(xyz0)} 3 0 1\n")
        for i, p in enumerate(xyz0):
            f.write(f"{i + 1} {float(p[0])!r} {float(p[1])!r} {float(p[2])!r} {int(p[0] == 0.0)}\n")
    with open(ele, "w") as f:
        f.write(f"{len(tets0)} 4 0\n")
        for t, q in enumerate(tets0):
            f.write(f"{t + 1} {q[0] + 1} {q[1] + 1} {q[2] + 1} {q[3] + 1}\n")
    xyz, tets, mark = read_tetgen(node, ele)
    assert np.array_equal(xyz, xyz0) and np.array_equal(tets, tets0)
    assert np.array_equal(mark, (xyz0[:, 0] == 0.0).astype(np.int32))
    xr, tr, vp, _ = (a.cpu().numpy() for a in ctx.reorder(_t(xyz, dev), _t(tets, dev)))

    def kappa(edges):  # a conductivity field of the edge midpoints, the same physics in any numbering
        mid = 0.5 * (xr[edges[:, 0]] + xr[edges[:, 1]])
        return 1.0 + 0.5 * np.sin(3.0 * mid[:, 0]) * np.cos(2.0 * mid[:, 1])

    Tg, fg, rms, _ = _gpu_solve(ctx, dev, xr, tr, kappa)
    To, fo = _oracle_solve(xr, tr, kappa)
    assert np.abs(Tg - To).max() <= 1e-9
    assert abs(fg["k_eff"] - fo["k_eff"]) <= 1e-10 * fo["k_eff"]
    # the unnumbered mesh: same physics (kappa from the midpoints of its own edges)
    def kappa0(edges):
        mid = 0.5 * (xyz[edges[:, 0]] + xyz[edges[:, 1]])
        return 1.0 + 0.5 * np.sin(3.0 * mid[:, 0]) * np.cos(2.0 * mid[:, 1])
    T0, f0, _, _ = _gpu_solve(ctx, dev, xyz, tets, kappa0)
    assert abs(f0["k_eff"] - fg["k_eff"]) <= 1e-10 * fg["k_eff"]
    assert np.abs(T0[vp] - Tg).max() <= 1e-9


def test_rms_error_matches_oracle(ctx, dev):
    xyz, tets = W.delaunay_cube(900, 60, 13)
    rng = np.random.Generator(np.random.PCG64(4))
    field = (0.7, -1.0, 0.25, 2.0)
    m = ctx.mesh(_t(xyz, dev), _t(tets, dev))
    try:
        Tv = rng.random(len(xyz))
        w = O.lumped_vertex_volumes(xyz, tets)
        exact_v = field[0] + xyz @ np.array(field[1:])
        rv = m.rms_error(_t(Tv, dev), field)
        assert abs(rv - O.rms_error(Tv, exact_v, w)) <= 1e-12 * rv
        Tt = rng.random(len(tets))
        rt = m.rms_error(_t(Tt, dev), field)
        assert abs(rt - D.rms_error_tets(xyz, tets, Tt, field)) <= 1e-12 * rt
        # the exact linear field at the vertices
        assert m.rms_error(_t(exact_v, dev), field) <= 1e-15
    finally:
        m.close()


def test_linear_solution_verification(ctx, dev):
    """The pristine-cube verification (Section 3.1): vertex unknowns on a jittered Kuhn mesh are
    exact for the linear solution (RMS at rounding level); tet unknowns on a Delaunay mesh carry
    the limiter's error, equal to the oracle's saddle-system value to within the solve's accuracy."""
    import scipy.sparse.linalg as spla
    n = 10
    xk, tk = W.kuhn_cube(n)
    xk = W.jitter_interior(xk, n, 0.2, 8)
    ones = lambda e: np.ones(len(e))  # noqa: E731
    _, f, rms_v, _ = _gpu_solve(ctx, dev, xk, tk, ones)
    assert rms_v < 1e-12 and abs(f["k_eff"] - 1.0) < 1e-11
    xyz, tets = W.delaunay_cube(1500, 90, 17)
    bt, bv, side = W.x_faces(xyz)
    m = ctx.mesh(_t(xyz, dev), _t(tets, dev))
    try:
        d = m.dual(_t(bt, dev), _t(bv, dev), _t(side, dev))
        try:
            T, st, rc = d.solve(tol=1e-12, check=False)
            assert rc == 0, st
            rms_t = m.rms_error(T)
        finally:
            d.close()
    finally:
        m.close()
    K, rhs, s = D.mixed_system(xyz, tets, bt, bv, side)
    To = spla.spsolve(K.tocsc(), rhs)[len(s["W"]):]
    ro = D.rms_error_tets(xyz, tets, To)
    print("rms vertex", rms_v, "tets", rms_t, "oracle tets", ro, flush=True)
    assert abs(rms_t - ro) <= 1e-6 * ro + 1e-12


def test_error_paths_of_the_mesh_calls(ctx, dev):
    """Bad arguments and calls on the wrong kind of mesh return status codes, and the context keeps
    working after each."""
    import ctypes
    import paper_2104_05999_amd as dec
    from paper_2104_05999_amd import _lib
    L = _lib.load()
    xyz, tets = W.kuhn_cube(3)
    x, t = _t(xyz, dev), _t(tets, dev)
    out_x = torch.empty_like(x)
    out_t = torch.empty_like(t)
    vp = lambda a: ctypes.c_void_p(a.data_ptr())  # noqa: E731
    EINVAL, ESTATE = -1, -8
    assert L.dec_reorder(ctx.handle, 0, 0, vp(x), len(tets), vp(t), vp(out_x), vp(out_t), None, None) == EINVAL
    assert L.dec_reorder(ctx.handle, 5, len(xyz), vp(x), len(tets), vp(t), vp(out_x), vp(out_t), None,
                         None) == EINVAL
    assert L.dec_reorder(ctx.handle, 0, len(xyz), vp(x), len(tets), vp(t), vp(x), vp(out_t), None, None) == EINVAL
    assert L.dec_reorder(None, 0, len(xyz), vp(x), len(tets), vp(t), vp(out_x), vp(out_t), None, None) == EINVAL
    bad = x.clone()
    bad[3, 1] = float("nan")
    with pytest.raises(dec.DecError):
        ctx.reorder(bad, t)
    m = ctx.mesh(x, t)
    try:
        f = (ctypes.c_double * 4)(1.0, -1.0, 0.0, 0.0)
        r = ctypes.c_double()
        T = torch.zeros(m.V, dtype=torch.float64, device=dev)
        assert L.dec_rms_error(m.handle, 2, vp(T), f, ctypes.byref(r)) == EINVAL
        assert L.dec_rms_error(m.handle, 0, None, f, ctypes.byref(r)) == EINVAL
        bt, bv, side = W.x_sides(3)
        d = m.dual(_t(bt, dev), _t(bv, dev), _t(side, dev))
        try:
            Td = torch.zeros(d.V, dtype=torch.float64, device=dev)
            assert L.dec_rms_error(d.handle, 1, vp(Td), f, ctypes.byref(r)) == ESTATE
            assert L.dec_dual_flux(d.handle, vp(Td), 1.0, 0.0, 1.0, None, None, None, None) == EINVAL
            assert L.dec_dual_faces(m.handle, None, None, None, None) == ESTATE  # not a tet system
            assert L.dec_dual_info(m.handle, None, None, None, None) == ESTATE
            assert b"dec_dual_build" in L.dec_last_error(ctx.handle)
            assert L.dec_dual_flux(d.handle, None, 1.0, 1.0, 1.0, None, None, None, None) == EINVAL
            assert b"NULL" in L.dec_last_error(ctx.handle)
            assert L.dec_dual_build(None, None, 0, None, None, None, None, 0.0, None, None) == EINVAL
            assert L.dec_dual_build(m.handle, None, -1, None, vp(_t(bt, dev)), vp(_t(bv, dev)), None, 0.0,
                                    ctypes.byref(ctypes.c_void_p()), None) == EINVAL
        finally:
            d.close()
        # still working
        assert abs(m.rms_error(_t(1.0 - xyz[:, 0], dev))) < 1e-15
    finally:
        m.close()
