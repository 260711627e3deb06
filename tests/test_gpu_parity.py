"""Parity of the HIP path (through the C ABI) with the FP64 oracle on seeded inputs.

Integer and index results (edges, CSR pattern, cut masks, pinned counts)
must match bit for bit; floating-point results within the stated
tolerances: *1 and the assembled values to 1e-13 relative (an h-scaled
absolute floor for entries that are zero), SpMV to 1e-14 relative in FP64,
solutions to 1e-10 relative against the oracle solved to 1e-14 (the GPU
solve runs to 1e-12), k_eff to 1e-9 relative.
"""
import numpy as np
import pytest
import torch

import oracle as O
import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx(dev):
    import paper_2104_05999_amd as dec
    c = dec.Context(dev)
    yield c
    c.close()


def _t(a, dev):
    return torch.as_tensor(np.ascontiguousarray(a), device=dev)


def _shuffled_mesh(n, seed):
    """Kuhn mesh with tets and each tet's vertex order shuffled (topology must not care)."""
    xyz, tets = W.kuhn_cube(n)
    rng = np.random.Generator(np.random.PCG64(seed))
    tets = tets[rng.permutation(len(tets))]
    tets = np.take_along_axis(tets, np.argsort(rng.random(tets.shape), axis=1), axis=1).astype(np.int32)
    return xyz, tets


def _system(n, sigma=1.0, n_cracks=20, kseed=1, cseed=2, rmin=0.02, rmax=0.08, xyz=None, tets=None):
    if xyz is None:
        xyz, tets = W.kuhn_cube(n)
    V = len(xyz)
    E = O.edges_of(tets, V)
    kap = W.lognormal_kappa(len(E), sigma, kseed) if sigma > 0 else np.ones(len(E))
    cr = W.penny_cracks(n_cracks, cseed, rmin, rmax)
    cut = O.crack_cut(xyz, E, cr)
    star = O.hodge1(xyz, tets, E, kappa=kap, cut=cut)
    L, _ = O.assemble(V, E, star)
    bt, bv, side = W.x_sides(n)
    A, b, pinned = O.apply_bc(L, bt, bv, E, star)
    return dict(xyz=xyz, tets=tets, V=V, E=E, kap=kap, cr=cr, cut=cut, star=star, L=L, A=A, b=b, pinned=pinned,
                bt=bt, bv=bv, side=side)


def _gpu(ctx, s, dev):
    m = ctx.mesh(_t(s["xyz"], dev), _t(s["tets"], dev))
    cut, star = m.hodge1(_t(s["kap"], dev), _t(s["cr"], dev))
    m.assemble()
    npin, b = m.apply_bc(_t(s["bt"], dev), _t(s["bv"], dev))
    return m, cut, star, npin, b


# ---------------------------------------------------------------- topology
@pytest.mark.parametrize("n", [1, 2, 3, 5, 16])
def test_topology_bit_exact(ctx, dev, n):
    xyz, tets = W.kuhn_cube(n)
    m = ctx.mesh(_t(xyz, dev), _t(tets, dev))
    E = O.edges_of(tets, len(xyz))
    F, count = O.faces_of(tets)
    assert (m.E, m.F, m.F_boundary, m.nnz) == (len(E), len(F), int((count == 1).sum()), len(xyz) + 2 * len(E))
    assert np.array_equal(m.edges().cpu().numpy(), E)
    L, _ = O.assemble(len(xyz), E, np.ones(len(E)))
    rp, col, _, _ = m.csr(values=False)
    assert np.array_equal(rp.cpu().numpy(), L.indptr)
    assert np.array_equal(col.cpu().numpy(), L.indices)


def _double_cone(k, seed):
    """Centre, two apexes and a ring of k vertices: the centre lies in 2k tets and the
    centre-apex edges in k each (2k = 16 and 32 fill exactly the one and two tets per lane that a
    16-lane group holds in registers; 40 and 80 go past them); tets in seeded random order."""
    th = 2 * np.pi * np.arange(k) / k
    xyz = np.concatenate([[[0.0, 0.0, 0.0], [0.0, 0.0, 1.0], [0.0, 0.0, -1.0]],
                          np.stack([np.cos(th), np.sin(th), np.zeros(k)], axis=1)])
    ring = 3 + np.arange(k)
    nxt = 3 + (np.arange(k) + 1) % k
    tets = np.concatenate([np.stack([np.zeros(k, int), np.full(k, 1), ring, nxt], axis=1),
                           np.stack([np.zeros(k, int), np.full(k, 2), ring, nxt], axis=1)])
    rng = np.random.Generator(np.random.PCG64(seed))
    tets = tets[rng.permutation(len(tets))]
    tets = np.take_along_axis(tets, rng.permuted(np.tile(np.arange(4), (len(tets), 1)), axis=1), axis=1)
    return xyz, tets.astype(np.int32)


@pytest.mark.parametrize("k", [8, 12, 16, 20, 40])
def test_topology_high_degree_vertices(ctx, dev, k):
    xyz, tets = _double_cone(k, k)
    m = ctx.mesh(_t(xyz, dev), _t(tets, dev))
    E = O.edges_of(tets, len(xyz))
    F, count = O.faces_of(tets)
    assert (m.E, m.F, m.F_boundary) == (len(E), len(F), int((count == 1).sum()))
    assert np.array_equal(m.edges().cpu().numpy(), E)
    L, _ = O.assemble(len(xyz), E, np.ones(len(E)))
    rp, col, _, _ = m.csr(values=False)
    assert np.array_equal(rp.cpu().numpy(), L.indptr) and np.array_equal(col.cpu().numpy(), L.indices)
    _, star = m.hodge1()
    ref = O.hodge1(xyz, tets, E)
    assert np.allclose(star.cpu().numpy(), ref, rtol=1e-13, atol=1e-15)
    m.close()


def test_topology_independent_of_tet_order(ctx, dev):
    xyz, tets = _shuffled_mesh(4, 3)
    m = ctx.mesh(_t(xyz, dev), _t(tets, dev))
    assert np.array_equal(m.edges().cpu().numpy(), O.edges_of(tets, len(xyz)))


@pytest.mark.parametrize("case", ["range", "repeat", "flat", "shared_face", "nan"])
def test_invalid_mesh_rejected(ctx, dev, case):
    import paper_2104_05999_amd as dec
    xyz, tets = W.kuhn_cube(2)
    if case == "range":
        tets = tets.copy()
        tets[3, 2] = len(xyz) + 5
    elif case == "repeat":
        tets = tets.copy()
        tets[5, 1] = tets[5, 0]
    elif case == "flat":
        xyz = xyz.copy()
        xyz[:, 2] = 0.0
    elif case == "nan":
        xyz = xyz.copy()
        xyz[7, 1] = np.nan
    else:
        tets = np.concatenate([tets, tets[:1]])
    with pytest.raises(dec.DecError) as ei:
        ctx.mesh(_t(xyz, dev), _t(tets, dev))
    assert ei.value.code == -6
    assert O.check_mesh(xyz, tets) is not None


# ---------------------------------------------------------------- Hodge star and cracks
@pytest.mark.parametrize("n,shuffle", [(3, False), (16, False), (24, False), (6, True)])
def test_hodge1_and_cut(ctx, dev, n, shuffle):
    xyz, tets = _shuffled_mesh(n, 5) if shuffle else W.kuhn_cube(n)
    s = _system(n, n_cracks=30, rmin=0.05, rmax=0.2, xyz=xyz, tets=tets)
    m, cut, star, _, _ = _gpu(ctx, s, dev)
    assert np.array_equal(cut.cpu().numpy().astype(bool), s["cut"])
    g = star.cpu().numpy()
    h = 1.0 / n
    assert np.all((g == 0) == (s["star"] == 0))
    assert np.allclose(g, s["star"], rtol=1e-13, atol=1e-15 * h)


def test_hodge1_jittered_geometry(ctx, dev):
    n = 6
    xyz, tets = W.kuhn_cube(n)
    xyz = W.jitter_interior(xyz, n, 0.2, 7)
    E = O.edges_of(tets, len(xyz))
    want = O.hodge1(xyz, tets, E)
    m = ctx.mesh(_t(xyz, dev), _t(tets, dev))
    _, star = m.hodge1()
    assert np.allclose(star.cpu().numpy(), want, rtol=1e-12, atol=1e-15)


def test_cut_mask_many_discs_over_lds_chunks(ctx, dev):
    n = 10
    xyz, tets = W.kuhn_cube(n)
    E = O.edges_of(tets, len(xyz))
    cr = W.penny_cracks(700, 9, 0.01, 0.06)  # more discs than one LDS chunk holds
    m = ctx.mesh(_t(xyz, dev), _t(tets, dev))
    cut, _ = m.hodge1(None, _t(cr, dev))
    assert np.array_equal(cut.cpu().numpy().astype(bool), O.crack_cut(xyz, E, cr))


def _odd_discs():
    """Degenerate discs: zero radius, negative radius, a disc larger than the domain, a zero
    normal, NaN and infinite centres."""
    nan, inf = float("nan"), float("inf")
    return np.array([
        [0.5, 0.5, 0.5, 0.0, 0.0, 1.0, 0.0],
        [0.31, 0.42, 0.53, 0.0, 1.0, 0.0, -0.2],
        [0.5, 0.5, 0.37, 0.3, 0.4, 0.866, 10.0],
        [0.2, 0.2, 0.2, 0.0, 0.0, 0.0, 0.3],
        [nan, 0.5, 0.5, 1.0, 0.0, 0.0, 0.3],
        [0.5, 0.5, 0.5, nan, 0.0, 1.0, 0.3],
        [inf, 0.5, 0.5, 1.0, 0.0, 0.0, 0.3],
        [0.5, 0.5, 0.5, 1.0, 0.0, 0.0, nan],
    ])


@pytest.mark.parametrize("many", [False, True])
def test_cut_mask_degenerate_discs(ctx, dev, many):
    """Both cut paths (at most 64 discs: every disc against every edge; more: spatial bins)
    agree with the oracle predicate on degenerate discs."""
    n = 7
    xyz, tets = W.kuhn_cube(n)
    E = O.edges_of(tets, len(xyz))
    cr = _odd_discs()
    if many:
        cr = np.concatenate([W.penny_cracks(80, 11, 0.02, 0.1), cr])
    m = ctx.mesh(_t(xyz, dev), _t(tets, dev))
    try:
        cut, star = m.hodge1(None, _t(cr, dev))
        want = O.crack_cut(xyz, E, cr)
        assert want.any()
        assert np.array_equal(cut.cpu().numpy().astype(bool), want)
        assert np.all(np.isfinite(star.cpu().numpy()))
    finally:
        m.close()


# ---------------------------------------------------------------- assembly and boundary data
@pytest.mark.parametrize("n", [4, 16])
def test_assembly_and_bc(ctx, dev, n):
    s = _system(n, n_cracks=25, rmin=0.05, rmax=0.25)
    m = ctx.mesh(_t(s["xyz"], dev), _t(s["tets"], dev))
    m.hodge1(_t(s["kap"], dev), _t(s["cr"], dev))
    m.assemble()
    _, _, v64, v32 = m.csr()
    assert np.allclose(v64.cpu().numpy(), s["L"].data, rtol=1e-13, atol=1e-15 / n)
    assert np.array_equal(v32.cpu().numpy(), v64.cpu().numpy().astype(np.float32))
    npin, b = m.apply_bc(_t(s["bt"], dev), _t(s["bv"], dev))
    assert npin == int(s["pinned"].sum())
    _, _, a64, _ = m.csr()
    assert np.allclose(a64.cpu().numpy(), s["A"].data, rtol=1e-13, atol=1e-15 / n)
    assert np.allclose(b.cpu().numpy(), s["b"], rtol=1e-13, atol=1e-15 / n)


def test_isolated_vertices_pinned(ctx, dev):
    n = 6
    xyz, tets = W.kuhn_cube(n)
    E = O.edges_of(tets, len(xyz))
    i, j, k = W.lattice_index(n)
    # a small box of discs around two interior vertices cuts every edge at them
    cr = []
    for v in (3 + 7 * (3 + 7 * 3), 2 + 7 * (4 + 7 * 2)):
        c = xyz[v]
        for ax in range(3):
            for sgn in (-1, 1):
                nrm = np.zeros(3)
                nrm[ax] = 1.0
                cr.append([*(c + sgn * 0.4 / n * nrm), *nrm, 0.3])
    cr = np.array(cr)
    cut = O.crack_cut(xyz, E, cr)
    star = O.hodge1(xyz, tets, E, cut=cut)
    bt, bv, _ = W.x_sides(n)
    _, _, pinned = O.apply_bc(O.assemble(len(xyz), E, star)[0], bt, bv, E, star)
    assert pinned.sum() >= 2
    m = ctx.mesh(_t(xyz, dev), _t(tets, dev))
    m.hodge1(None, _t(cr, dev))
    m.assemble()
    npin, _ = m.apply_bc(_t(bt, dev), _t(bv, dev))
    assert npin == int(pinned.sum())
    T, st, _ = m.solve(tol=1e-12)
    assert np.all(T.cpu().numpy()[pinned] == 0.0)


def test_boundary_data_applied_again_to_one_assembly(ctx, dev):
    """dec_apply_bc twice on one assembly: the second system is the oracle's for the second data
    (the first call's elimination is undone), and applying the first data again gives the first
    solution bit for bit."""
    n = 8
    s = _system(n, n_cracks=10)
    i, j, k = W.lattice_index(n)
    bt2 = ((j == 0) | (j == n)).astype(np.int8)
    bv2 = np.where(j == 0, 2.0, -1.0) * bt2 + 0.1 * k / n * bt2
    A2, b2, _ = O.apply_bc(s["L"], bt2, bv2, s["E"], s["star"])
    ref2 = O.pcg(A2, b2, precond="jacobi", tol=1e-14, stagnation=50)
    m, _, _, _, b1 = _gpu(ctx, s, dev)
    try:
        T1, _, rc1 = m.solve(tol=1e-12)
        T1 = T1.clone()
        _, b = m.apply_bc(_t(bt2, dev), _t(bv2, dev))
        assert np.abs(b.cpu().numpy() - b2).max() <= 1e-13 * np.abs(b2).max()
        T2, st, rc2 = m.solve(tol=1e-12)
        assert rc1 == 0 and rc2 == 0, st
        x = T2.cpu().numpy()
        assert np.linalg.norm(x - ref2.x) <= 1e-10 * np.linalg.norm(ref2.x)
        m.apply_bc(_t(s["bt"], dev), _t(s["bv"], dev))
        T3, _, _ = m.solve(tol=1e-12)
        assert torch.equal(T3, T1)
    finally:
        m.close()


def test_neumann_load(ctx, dev):
    n = 5
    xyz, tets = W.kuhn_cube(n)
    V = len(xyz)
    E = O.edges_of(tets, V)
    i, j, _ = W.lattice_index(n)
    bt = np.where(i == n, 1, np.where((i == 0) | (j == 0), 2, 0)).astype(np.int8)
    f0 = np.where(i == 0, -2.5, np.where(j == 0, 0.7, 0.0))
    g = O.neumann_load(xyz, tets, O.boundary_faces(tets), bt, f0)
    star = O.hodge1(xyz, tets, E)
    A, b, _ = O.apply_bc(O.assemble(V, E, star)[0], bt, np.zeros(V), E, star, neumann=g)
    m = ctx.mesh(_t(xyz, dev), _t(tets, dev))
    m.hodge1()
    m.assemble()
    _, bg = m.apply_bc(_t(bt, dev), _t(np.zeros(V), dev), _t(f0, dev))
    assert np.allclose(bg.cpu().numpy(), b, rtol=1e-13, atol=1e-16)
    # with a Neumann load k_eff is the flux density through the Dirichlet side (x = 1 only here)
    ref = O.pcg(A, b, precond="jacobi", tol=1e-14, stagnation=50)
    side = np.where(i == n, 2, 0).astype(np.int8)
    of = O.flux_effective_conductivity(ref.x, E, star, side, neumann=True)
    T, _, _ = m.solve(tol=1e-14)
    f = m.flux(T, _t(side, dev))
    assert abs(f["k_eff"] - of["k_eff"]) <= 1e-9 * abs(of["k_eff"]) and f["k_eff"] == f["q_out"]
    assert abs(f["energy"] - of["energy"]) <= 1e-9 * abs(of["energy"])


# ---------------------------------------------------------------- SpMV
@pytest.mark.parametrize("n", [3, 16, 33])
def test_spmv(ctx, dev, n):
    import paper_2104_05999_amd as dec
    s = _system(n)
    m, _, _, _, _ = _gpu(ctx, s, dev)
    x = np.random.Generator(np.random.PCG64(n)).normal(size=s["V"])
    want = s["A"] @ x
    for fmt in (dec.DEC_FMT_SELL, dec.DEC_FMT_CSR):
        y = m.spmv(_t(x, dev), fmt=fmt).cpu().numpy()
        assert np.allclose(y, want, rtol=1e-14, atol=1e-14 * np.abs(want).max())
        y32 = m.spmv(_t(x.astype(np.float32), dev), precision=dec.DEC_PREC_MIXED, fmt=fmt).cpu().numpy()
        w32 = s["A"].astype(np.float32) @ x.astype(np.float32)
        assert np.allclose(y32, w32, rtol=1e-5, atol=1e-5 * np.abs(w32).max())


# ---------------------------------------------------------------- solves
def test_homogeneous_16_linear_and_keff(ctx, dev):
    n = 16
    xyz, tets = W.kuhn_cube(n)
    bt, bv, side = W.x_sides(n)
    m = ctx.mesh(_t(xyz, dev), _t(tets, dev))
    m.hodge1()
    m.assemble()
    m.apply_bc(_t(bt, dev), _t(bv, dev))
    T, st, rc = m.solve(tol=1e-10)
    i, _, _ = W.lattice_index(n)
    assert rc == 0 and st["rel_residual"] <= 1e-10
    assert np.abs(T.cpu().numpy() - (1 - i / n)).max() < 1e-8
    f = m.flux(T, _t(side, dev))
    assert abs(f["k_eff"] - 1.0) < 1e-9 and abs(f["q_in"] - 1.0) < 1e-8 and abs(f["q_out"] - 1.0) < 1e-8


def _reference(s):
    return O.pcg(s["A"], s["b"], precond="jacobi", tol=1e-14, stagnation=50)


@pytest.mark.parametrize("precision,precond", [(0, 0), (0, 1), (1, 0), (1, 1)])
def test_solve_against_oracle(ctx, dev, precision, precond):
    n = 20
    s = _system(n, n_cracks=40, rmin=0.03, rmax=0.12)
    ref = _reference(s)
    m, _, _, _, _ = _gpu(ctx, s, dev)
    T, st, rc = m.solve(tol=1e-12, precision=precision, precond=precond)
    assert rc == 0, st
    x = T.cpu().numpy()
    err = np.linalg.norm(x - ref.x) / np.linalg.norm(ref.x)
    assert err <= 1e-10, (err, st)
    assert st["rel_residual"] <= 1e-12
    r = np.linalg.norm(s["b"] - s["A"] @ x) / np.linalg.norm(s["b"])
    assert r <= 1.5e-12
    f = m.flux(T, _t(s["side"], dev), want_edge_flux=True)
    of = O.flux_effective_conductivity(ref.x, s["E"], s["star"], s["side"])
    for key in ("k_eff", "q_in", "q_out", "energy"):
        assert abs(f[key] - of[key]) <= 1e-9 * abs(of["energy"]), key
    ef = f["edge_flux"].cpu().numpy()
    assert np.allclose(ef, of["edge_flux"], rtol=1e-8, atol=1e-9 * np.abs(of["edge_flux"]).max())


@pytest.mark.parametrize("split", ["1", "0"])
@pytest.mark.parametrize("precond", [0, 1])
def test_fp32_vector_kernels_one_or_two_rows_per_lane(ctx, dev, split, precond):
    """The FP32 update and closing kernels take two rows per lane (float2) where the vectors sit
    on 8-byte boundaries, with the last row of an odd V on its own, and one row per lane
    otherwise (DEC_VEC_PAIRS=0 forces that path): both mixed-precision solves meet the oracle's
    x* to 1e-10 in the 2-norm on a system with an odd number of rows (21^3), with Jacobi on A,
    in split form and with FSAI, and agree with each other to that accuracy."""
    import os
    s = _system(20, n_cracks=40, rmin=0.03, rmax=0.12)
    assert s["V"] % 2 == 1
    xs = _reference(s).x
    out = {}
    os.environ["DEC_JACOBI_SPLIT"] = split
    try:
        for pairs in ("1", "0"):
            os.environ["DEC_VEC_PAIRS"] = pairs
            try:
                m, _, _, _, _ = _gpu(ctx, s, dev)
                T, st, rc = m.solve(tol=1e-12, precision=1, precond=precond)
                m.close()
            finally:
                del os.environ["DEC_VEC_PAIRS"]
            assert rc == 0, (pairs, st)
            out[pairs] = T.cpu().numpy()
    finally:
        del os.environ["DEC_JACOBI_SPLIT"]
    rel = lambda a, b: np.linalg.norm(a - b) / np.linalg.norm(b)  # noqa: E731
    assert rel(out["1"], xs) <= 1e-10 and rel(out["0"], xs) <= 1e-10, (rel(out["1"], xs), rel(out["0"], xs))
    assert rel(out["1"], out["0"]) <= 2e-10

def test_fsai_factor_matches_oracle(ctx, dev):
    n = 7
    s = _system(n, n_cracks=15, rmin=0.05, rmax=0.2)
    m, _, _, _, _ = _gpu(ctx, s, dev)
    ptr, col, val = m.fsai()
    G = O.fsai_factor(s["A"])
    assert np.array_equal(ptr.cpu().numpy(), G.indptr)
    assert np.array_equal(col.cpu().numpy(), G.indices)
    assert np.allclose(val.cpu().numpy(), G.data, rtol=1e-12, atol=1e-14 * np.abs(G.data).max())


@pytest.mark.parametrize("precision,precond", [(0, 0), (0, 1), (1, 0), (1, 1)])
def test_solver_is_deterministic(ctx, dev, precision, precond):
    """Fixed-order folds: repeated solves, graph replay or plain launches, and sampled timing
    all give the same bits."""
    s = _system(12, n_cracks=20)
    m, _, _, _, _ = _gpu(ctx, s, dev)
    kw = dict(tol=1e-11, precision=precision, precond=precond)
    a, sa, _ = m.solve(**kw)
    b, sb, _ = m.solve(**kw)
    c, sc, _ = m.solve(use_graph=0, **kw)
    d, sd, _ = m.solve(profile=3, **kw)
    assert torch.equal(a, b) and torch.equal(a, c) and torch.equal(a, d)
    assert sa["iterations"] == sb["iterations"] == sc["iterations"] == sd["iterations"]


def test_warm_start_and_limits(ctx, dev):
    s = _system(12, n_cracks=10)
    m, _, _, _, _ = _gpu(ctx, s, dev)
    T, st, rc = m.solve(tol=1e-10)
    T2, st2, rc2 = m.solve(T=T.clone(), tol=1e-10, warm_start=1)
    assert rc2 == 0 and st2["iterations"] <= 1
    _, st3, rc3 = m.solve(tol=1e-12, max_iters=3, check=False)
    assert rc3 == -4 and st3["iterations"] == 3


def test_profiled_solve_counts_spmv(ctx, dev):
    s = _system(10, n_cracks=5)
    m, _, _, _, _ = _gpu(ctx, s, dev)
    T, st, rc = m.solve(tol=1e-10, profile=1)
    assert rc == 0 and st["spmv_launches"] == st["iterations"] and st["spmv_ms"] > 0
    T4, st4, rc4 = m.solve(tol=1e-10, profile=4)  # SpMV k of each 32-iteration batch timed when k % 4 == 3
    n = st4["iterations"]
    assert rc4 == 0 and n == st["iterations"] and torch.equal(T4, T)
    if st4["restarts"] == 0:  # one run of batches from iteration 0
        assert st4["spmv_launches"] == 8 * (n // 32) + (n % 32) // 4
    assert 0 <= st4["spmv_launches"] <= n
    T0, st0, _ = m.solve(tol=1e-10)
    assert torch.equal(T0, T) and st0["spmv_launches"] == 0


def test_pruned_pattern_products_are_bit_identical(ctx, dev):
    import paper_2104_05999_amd as dec
    n = 9
    s = _system(n, n_cracks=20, rmin=0.05, rmax=0.2)
    m, _, _, _, _ = _gpu(ctx, s, dev)
    x = torch.as_tensor(np.random.Generator(np.random.PCG64(4)).normal(size=s["V"]), device=dev)
    y_pruned = m.spmv(x)
    y_csr = m.spmv(x, fmt=dec.DEC_FMT_CSR)
    T_pruned, st_p, _ = m.solve(tol=1e-11)
    m.assemble(full_pattern=True)
    m.apply_bc(_t(s["bt"], dev), _t(s["bv"], dev))
    y_full = m.spmv(x)
    T_full, st_f, _ = m.solve(tol=1e-11)
    assert torch.equal(y_pruned, y_full) and torch.equal(y_full, y_csr)
    assert torch.equal(T_pruned, T_full)
    assert st_p["spmv_nnz"] < st_f["spmv_nnz"] == m.nnz


@pytest.mark.parametrize("precision,norm", [(0, 0), (1, 0), (0, 1)])
def test_split_jacobi_matches_jacobi(ctx, dev, precision, norm):
    """Jacobi in split form (CG on D^-1/2 A D^-1/2, the solver's default) takes the iterates of
    Jacobi-preconditioned CG on A up to rounding: the same solution to the tolerance's accuracy,
    the same iteration count within a few, in FP64, with FP32 inner solves, and with the A-norm
    test.  Both against the oracle's x*: relative 2-norm error <= 1e-10 with the residual test
    (tol 1e-12), relative A-norm error <= 10 tol with the A-norm test."""
    import os
    s = _system(12, n_cracks=30)
    xs = _reference(s).x
    out = {}
    for split in ("1", "0"):
        os.environ["DEC_JACOBI_SPLIT"] = split
        try:
            m, _, _, _, _ = _gpu(ctx, s, dev)
            T, st, rc = m.solve(tol=1e-12, precision=precision, norm=norm)
            assert rc == 0, (split, st)
            m.close()
        finally:
            del os.environ["DEC_JACOBI_SPLIT"]
        out[split] = (T.cpu().numpy(), st)
    (Ts, ss), (Tp, sp) = out["1"], out["0"]
    A = s["A"]
    if norm == 0:
        rel = lambda a, b: np.linalg.norm(a - b) / np.linalg.norm(b)  # noqa: E731
        assert rel(Ts, xs) <= 1e-10 and rel(Tp, xs) <= 1e-10, (rel(Ts, xs), rel(Tp, xs))
        assert rel(Ts, Tp) <= 2e-10
    else:
        rel = lambda a, b: np.sqrt((a - b) @ (A @ (a - b)) / (b @ (A @ b)))  # noqa: E731
        assert rel(Ts, xs) <= 1e-11 and rel(Tp, xs) <= 1e-11, (rel(Ts, xs), rel(Tp, xs))
        assert rel(Ts, Tp) <= 2e-11
    assert abs(ss["iterations"] - sp["iterations"]) <= max(3, sp["iterations"] // 50), (ss, sp)


def test_column_offsets_and_their_fallback(ctx, dev):
    """The sliced-ELL copy reads one-byte indices into a table of column offsets when the stored
    entries take at most 256 distinct offsets (the 41^3-vertex lattice: seven), 16-bit offsets
    from the row when every column lies within 2^15 of it (also the lattice with its vertex
    numbers shuffled within windows of 1024, whose offsets are too many for a table), and int32
    columns otherwise (the lattice with its vertices scrambled).  Each format, forced through the
    environment (a missing one falls back to the next wider), gives the CSR product and the
    same temperatures bit for bit, and the solve's byte count states which columns it read; the
    two numberings give the same temperatures."""
    import os
    import paper_2104_05999_amd as dec
    n = 40
    xyz, tets = W.kuhn_cube(n)
    rng = np.random.Generator(np.random.PCG64(11))
    perm = rng.permutation(len(xyz))            # new number of old vertex i: perm[i]
    xyz_s = np.empty_like(xyz)
    xyz_s[perm] = xyz
    tets_s = perm[tets].astype(np.int32)
    bt, bv, _ = W.x_sides(n)
    bt_s, bv_s = np.empty_like(bt), np.empty_like(bv)
    bt_s[perm], bv_s[perm] = bt, bv
    win = np.arange(len(xyz)) // 1024 * 1024     # shuffled within windows of 1024 ids
    perm_w = win + np.concatenate([rng.permutation(min(1024, len(xyz) - w)) for w in range(0, len(xyz), 1024)])
    xyz_w = np.empty_like(xyz)
    xyz_w[perm_w] = xyz
    tets_w = perm_w[tets].astype(np.int32)
    bt_w, bv_w = np.empty_like(bt), np.empty_like(bv)
    bt_w[perm_w], bv_w[perm_w] = bt, bv
    # forced format -> bytes per column actually read, per mesh
    cases = {"lattice": ((xyz, tets, bt, bv), {8: 1, 16: 2, 32: 4}),
             "windows": ((xyz_w, tets_w, bt_w, bv_w), {8: 2, 16: 2, 32: 4}),
             "scrambled": ((xyz_s, tets_s, bt_s, bv_s), {8: 4, 16: 4, 32: 4})}
    out = {}
    for name, ((x3, tt, b_t, b_v), want) in cases.items():
        x = torch.as_tensor(rng.normal(size=len(x3)), device=dev)
        got = {}
        for cols, col_bytes in want.items():
            os.environ["DEC_SELL_COLS"] = str(cols)
            try:
                m = ctx.mesh(_t(x3, dev), _t(tt, dev))
                m.hodge1()
                m.assemble()
                m.apply_bc(_t(b_t, dev), _t(b_v, dev))
                T, st, rc = m.solve(tol=1e-12)
                assert rc == 0, (name, cols, st)
                V, nz = len(x3), st["spmv_nnz"]
                assert st["spmv_bytes"] == nz * (8 + col_bytes) + 4 * (V + 1) + 16 * V, (name, cols)
                assert torch.equal(m.spmv(x), m.spmv(x, fmt=dec.DEC_FMT_CSR)), (name, cols)
                got[cols] = T
                m.close()
            finally:
                del os.environ["DEC_SELL_COLS"]
        assert torch.equal(got[8], got[16]) and torch.equal(got[16], got[32]), name
        out[name] = got[32].cpu().numpy()
    Tl, Ts = out["lattice"], out["scrambled"][perm]
    assert np.abs(Tl - Ts).max() <= 1e-10 * np.abs(Tl).max()


def test_error_paths(ctx, dev):
    import paper_2104_05999_amd as dec
    n = 3
    xyz, tets = W.kuhn_cube(n)
    m = ctx.mesh(_t(xyz, dev), _t(tets, dev))
    try:
        bt, bv, _ = W.x_sides(n)
        with pytest.raises(dec.DecError) as ei:      # assembly before *1
            m.assemble()
        assert ei.value.code == -8
        m.hodge1()
        with pytest.raises(dec.DecError) as ei:      # solve before boundary data
            m.assemble()
            m.solve()
        assert ei.value.code == -8
        bad = bt.copy()
        bad[0] = 7
        with pytest.raises(dec.DecError) as ei:
            m.apply_bc(_t(bad, dev), _t(bv, dev))
        assert ei.value.code == -1
        m.apply_bc(_t(bt, dev), _t(bv, dev))
        for kw in ({"tol": 0.0}, {"inner_tol": 2.0}, {"precision": 5}, {"precond": 9}, {"max_iters": 0}):
            with pytest.raises(dec.DecError) as ei:
                m.solve(**kw)
            assert ei.value.code == -1
        with pytest.raises((ValueError, TypeError)):  # a crack record is 7 doubles
            m.hodge1(None, torch.zeros(5, dtype=torch.float64, device=dev).reshape(1, 5))
    finally:
        m.close()


def test_context_outlives_its_meshes(dev):
    """A context that still owns a mesh refuses to go; closing it from Python closes the mesh first."""
    import paper_2104_05999_amd as dec
    c = dec.Context(dev)
    xyz, tets = W.kuhn_cube(2)
    m = c.mesh(_t(xyz, dev), _t(tets, dev))
    assert c.lib.dec_destroy(c.handle) == -8   # DEC_ESTATE
    c.close()
    assert m.handle is None and c.handle is None


def test_nonfinite_conductivity_breaks_down(ctx, dev):
    n = 4
    xyz, tets = W.kuhn_cube(n)
    bt, bv, _ = W.x_sides(n)
    edges = O.edges_of(tets, len(xyz))
    interior = np.flatnonzero((bt[edges[:, 0]] == 0) & (bt[edges[:, 1]] == 0))
    kap = np.ones(len(edges))
    kap[interior[len(interior) // 2]] = np.nan   # an edge between two unknowns
    m = ctx.mesh(_t(xyz, dev), _t(tets, dev))
    try:
        m.hodge1(_t(kap, dev))
        m.assemble()
        m.apply_bc(_t(bt, dev), _t(bv, dev))
        _, st, rc = m.solve(check=False)
        assert rc == -5  # DEC_EBREAKDOWN, reported rather than a silent NaN solution
    finally:
        m.close()


@pytest.mark.parametrize("order", [0, 1])
@pytest.mark.parametrize("cols", [8, 16, 32])
@pytest.mark.parametrize("unroll,nt", [(2, 0), (2, 1), (3, 0), (3, 1), (4, 0), (4, 1)])
def test_every_sell_variant_gives_the_same_bits(ctx, dev, unroll, nt, cols, order):
    """The autotuner's variants (pairs in flight, non-temporal loads, a row's loads interleaved or
    columns first) sum every row in the same order and fold the partials in the same order, and
    the one-byte offset indices and 16-bit offsets name the same columns as the int32 columns:
    pinned through the environment, each gives the tuned solve's bits, on a vertex system and on
    a tet system, in FP64 and with FP32 inner solves (most vertex rows store 7 entries: with 2, 3
    and 4 pairs in flight such a row needs more pairs than one group holds, as many, and fewer)."""
    import os
    import paper_2104_05999_amd as dec
    s = _system(12, n_cracks=20)
    m, _, _, _, _ = _gpu(ctx, s, dev)
    ref = [m.solve(tol=1e-11, precision=p)[0] for p in (0, 1)]
    xyz, tets = W.kuhn_cube(7)
    bt, bv, side = W.x_sides(7)
    t = lambda a: torch.as_tensor(np.ascontiguousarray(a), device=dev)  # noqa: E731
    kap = t(W.lognormal_kappa(W.kuhn_counts(7)["F"], 1.0, 3))
    mt = ctx.mesh(t(xyz), t(tets))
    d = mt.dual(t(bt), t(bv), t(side), kap, t(W.penny_cracks(5, 9, 0.1, 0.3)))
    mt.close()
    ref_d = d.solve(tol=1e-11)[0]
    d.close()
    os.environ["DEC_SELL_UNROLL"], os.environ["DEC_SELL_NT"] = str(unroll), str(nt)
    os.environ["DEC_SELL_COLS"], os.environ["DEC_SELL_ORDER"] = str(cols), str(order)
    try:
        m2, _, _, _, _ = _gpu(ctx, s, dev)
        for p, r in zip((0, 1), ref):
            T, st, rc = m2.solve(tol=1e-11, precision=p)
            assert rc == 0 and torch.equal(T, r), p
            # the stats report the variant the solve ran (this lattice holds every encoding)
            assert (st["spmv_unroll"], st["spmv_nontemporal"], st["spmv_col_bytes"], st["spmv_order"]) == (
                unroll, nt, cols // 8, order), p
        mt = ctx.mesh(t(xyz), t(tets))
        d = mt.dual(t(bt), t(bv), t(side), kap, t(W.penny_cracks(5, 9, 0.1, 0.3)))
        mt.close()
        assert torch.equal(d.solve(tol=1e-11)[0], ref_d)
        d.close()
    finally:
        del os.environ["DEC_SELL_UNROLL"], os.environ["DEC_SELL_NT"], os.environ["DEC_SELL_COLS"]
        del os.environ["DEC_SELL_ORDER"]


@pytest.mark.parametrize("band", ["7,3", "5,5", "1,1", "13,64", "40,16"])
def test_banded_slice_order(ctx, dev, band):
    """The banded slice order (planes of `plane` slices walked band by band, for matrices whose
    far offsets outrun the L2) is a permutation of each XCD's slices: forced onto small systems
    through the environment, every row of the product is the plain order's bit for bit (y starts
    as NaN, so a slice left out shows), and the p.Ap partials cover each row once, so the solves
    agree with the plain order's to rounding (their sums are grouped differently) with the same
    iteration counts to within a few; on a vertex system in FP64 and mixed precision and on a
    tet system."""
    import os
    n = 40  # 68,921 rows: 1,077 slices, about 135 per XCD
    xyz_v, tets_v = W.kuhn_cube(n)
    bt_v, bv_v, _ = W.x_sides(n)
    s = dict(xyz=xyz_v, tets=tets_v, V=len(xyz_v), kap=W.lognormal_kappa(W.kuhn_counts(n)["E"], 1.0, 1),
             cr=W.penny_cracks(20, 2, 0.02, 0.08), bt=bt_v, bv=bv_v)
    xyz, tets = W.kuhn_cube(16)  # 24,576 tets: 384 slices
    bt, bv, side = W.x_sides(16)
    t = lambda a: torch.as_tensor(np.ascontiguousarray(a), device=dev)  # noqa: E731
    kap = t(W.lognormal_kappa(W.kuhn_counts(16)["F"], 1.0, 3))
    cr = t(W.penny_cracks(5, 9, 0.1, 0.3))

    def run():
        m, _, _, _, _ = _gpu(ctx, s, dev)
        x = torch.as_tensor(np.random.default_rng(4).standard_normal(s["V"]), device=dev)
        y = torch.full_like(x, float("nan"))
        m.spmv(x, y)
        sols = [m.solve(tol=1e-11, precision=p) for p in (0, 1)]
        m.close()
        mt = ctx.mesh(t(xyz), t(tets))
        d = mt.dual(t(bt), t(bv), t(side), kap, cr)
        mt.close()
        sd = d.solve(tol=1e-11)
        d.close()
        return y, sols, sd

    os.environ["DEC_SELL_BAND"] = "0"
    try:
        y0, sols0, sd0 = run()
        os.environ["DEC_SELL_BAND"] = band
        y1, sols1, sd1 = run()
    finally:
        del os.environ["DEC_SELL_BAND"]
    assert not torch.isnan(y0).any() and torch.equal(y0, y1)
    for (T0, st0, rc0), (T1, st1, rc1) in zip(sols0 + [sd0], sols1 + [sd1]):
        assert rc0 == 0 and rc1 == 0
        assert float(torch.linalg.norm(T1 - T0)) <= 1e-9 * float(torch.linalg.norm(T0))
        assert abs(st1["iterations"] - st0["iterations"]) <= max(3, st0["iterations"] // 50)
