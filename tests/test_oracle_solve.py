"""Pins of the oracle's operator, boundary data, solvers and effective conductivity (CPU)."""
import numpy as np
import pytest
import scipy.sparse as sp

import oracle as O
import workloads as W


def _problem(n, sigma=0.0, n_cracks=0, kseed=1, cseed=2, xyz=None):
    xyz0, tets = W.kuhn_cube(n)
    xyz = xyz0 if xyz is None else xyz
    V = len(xyz)
    E = O.edges_of(tets, V)
    kap = W.lognormal_kappa(len(E), sigma, kseed) if sigma > 0 else None
    cut = O.crack_cut(xyz, E, W.penny_cracks(n_cracks, cseed)) if n_cracks else None
    s = O.hodge1(xyz, tets, E, kappa=kap, cut=cut)
    L, eid = O.assemble(V, E, s)
    bt, bv, side = W.x_sides(n)
    A, b, pinned = O.apply_bc(L, bt, bv, E, s)
    return dict(xyz=xyz, tets=tets, E=E, s=s, L=L, A=A, b=b, pinned=pinned, bt=bt, bv=bv, side=side)


def _fem_stiffness(xyz, tets):
    """Brute-force P1 finite-element stiffness: K_T[a,b] = vol(T) grad(lambda_a) . grad(lambda_b)."""
    V = len(xyz)
    K = np.zeros((V, V))
    for t in tets:
        p = xyz[t]
        M = np.column_stack([np.ones(4), p])  # lambda = M^-1 applied to (1, x, y, z)
        C = np.linalg.inv(M)                    # row r+1 of C holds d(lambda)/dx_r
        G = C[1:, :].T                          # [4 vertices, 3] gradients
        vol = abs(np.linalg.det(np.column_stack([p[1] - p[0], p[2] - p[0], p[3] - p[0]]))) / 6
        K[np.ix_(t, t)] += vol * G @ G.T
    return K


def test_regular_tet_equals_fem():
    xyz = np.array([[1, 1, 1], [1, -1, -1], [-1, 1, -1], [-1, -1, 1]], dtype=float)
    tets = np.array([[0, 1, 2, 3]])
    E = O.edges_of(tets, 4)
    L, _ = O.assemble(4, E, O.hodge1(xyz, tets, E))
    assert np.allclose(L.toarray(), _fem_stiffness(xyz, tets), rtol=0, atol=1e-14)


@pytest.mark.parametrize("n", [2, 3, 4, 5, 6])
def test_kuhn_rows_off_domain_edges_equal_fem(n):
    xyz, tets = W.kuhn_cube(n)
    E = O.edges_of(tets, len(xyz))
    L, _ = O.assemble(len(xyz), E, O.hodge1(xyz, tets, E))
    K = _fem_stiffness(xyz, tets)
    i, j, k = W.lattice_index(n)
    on_bdry = (i % n == 0).astype(int) + (j % n == 0) + (k % n == 0)
    rows = on_bdry <= 1  # not on one of the cube's 12 edges or 8 corners
    D = L.toarray()
    assert np.abs(D[rows] - K[rows]).max() <= 1.5e-15
    # on the cube's edges the two operators differ (DEC crease weight h/4)
    assert np.abs(D[~rows] - K[~rows]).max() > 1e-3


def test_symmetric_and_zero_row_sums():
    p = _problem(6, sigma=1.0, n_cracks=15)
    L = p["L"]
    assert (abs(L - L.T)).max() == 0
    rs = np.abs(np.asarray(L.sum(axis=1)).ravel())
    assert np.all(rs <= 16 * np.finfo(float).eps * L.diagonal())
    # static pattern: full edge graph plus the diagonal
    assert L.nnz == len(p["xyz"]) + 2 * len(p["E"])


def test_linear_exactness_jittered():
    n = 5
    xyz, tets = W.kuhn_cube(n)
    xyz = W.jitter_interior(xyz, n, 0.2, 7)
    V = len(xyz)
    E = O.edges_of(tets, V)
    L, _ = O.assemble(V, E, O.hodge1(xyz, tets, E))
    i, j, k = W.lattice_index(n)
    interior = (i > 0) & (i < n) & (j > 0) & (j < n) & (k > 0) & (k < n)
    rng = np.random.Generator(np.random.PCG64(8))
    for _ in range(3):
        g = rng.normal(size=3)
        u = xyz @ g + rng.normal()
        assert np.abs((L @ u)[interior]).max() < 1e-13


@pytest.mark.parametrize("n", [2, 4, 8, 16])
def test_homogeneous_linear_solution_and_keff(n):
    p = _problem(n)
    res = O.pcg(p["A"], p["b"], precond="jacobi", tol=1e-12)
    i, _, _ = W.lattice_index(n)
    assert res.converged
    assert np.abs(res.x - (1 - i / n)).max() < 1e-10
    f = O.flux_effective_conductivity(res.x, p["E"], p["s"], p["side"])
    assert abs(f["k_eff"] - 1.0) < 1e-10
    assert abs(f["q_in"] - 1.0) < 1e-10 and abs(f["q_out"] - 1.0) < 1e-10
    w = O.lumped_vertex_volumes(p["xyz"], p["tets"])
    assert abs(w.sum() - 1.0) < 1e-13
    assert O.rms_error(res.x, 1 - i / n, w) < 1e-10


def test_pcg_matches_dense_solve():
    p = _problem(5, sigma=1.0, n_cracks=20)
    x = np.linalg.solve(p["A"].toarray(), p["b"])
    for pre in (None, "jacobi"):
        res = O.pcg(p["A"], p["b"], precond=pre, tol=1e-13)
        assert np.linalg.norm(res.x - x) <= 1e-11 * np.linalg.norm(x)
    # the recursion is the textbook one: on a 1D Laplacian CG ends in at most m steps
    m = 30
    A = sp.diags([-np.ones(m - 1), 2 * np.ones(m), -np.ones(m - 1)], [-1, 0, 1]).tocsr()
    b = np.arange(1.0, m + 1)
    res = O.pcg(A, b, tol=1e-13)
    assert res.iterations <= m
    assert np.allclose(res.x, np.linalg.solve(A.toarray(), b), rtol=1e-11)


def test_dirichlet_elimination_is_exact():
    p = _problem(4, sigma=1.0, n_cracks=10)
    x = np.linalg.solve(p["A"].toarray(), p["b"])
    d = p["bt"] == 1
    free = ~d & ~p["pinned"]
    assert np.allclose(x[d], p["bv"][d], rtol=0, atol=0)
    # the original operator is balanced at every free vertex
    assert np.abs((p["L"] @ x)[free]).max() < 1e-12
    # symmetric elimination keeps A symmetric with the fixed pattern
    assert (abs(p["A"] - p["A"].T)).max() == 0 and p["A"].nnz == p["L"].nnz


def test_keff_scales_with_kappa_and_energy_identity():
    p = _problem(6, sigma=1.0, n_cracks=12)
    res = O.pcg(p["A"], p["b"], precond="jacobi", tol=1e-13)
    f = O.flux_effective_conductivity(res.x, p["E"], p["s"], p["side"])
    assert abs(f["q_in"] - f["energy"]) <= 1e-10 * f["energy"]
    assert abs(f["q_out"] - f["energy"]) <= 1e-10 * f["energy"]
    # Dirichlet principle: the exact solution minimises energy; u = 1 - x is admissible
    i, _, _ = W.lattice_index(6)
    u = 1 - i / 6
    du = u[p["E"][:, 1]] - u[p["E"][:, 0]]
    assert f["energy"] <= (p["s"] * du * du).sum()
    c = 3.5
    L2, _ = O.assemble(len(p["xyz"]), p["E"], c * p["s"])
    A2, b2, _ = O.apply_bc(L2, p["bt"], p["bv"], p["E"], c * p["s"])
    res2 = O.pcg(A2, b2, precond="jacobi", tol=1e-13)
    f2 = O.flux_effective_conductivity(res2.x, p["E"], c * p["s"], p["side"])
    assert abs(f2["k_eff"] - c * f["k_eff"]) <= 1e-10 * c * f["k_eff"]
    assert np.abs(res2.x - res.x).max() < 1e-10


def test_rayleigh_monotone_under_growing_cracks():
    n = 8
    xyz, tets = W.kuhn_cube(n)
    V = len(xyz)
    E = O.edges_of(tets, V)
    kap = W.lognormal_kappa(len(E), 1.0, 1)
    discs = W.penny_cracks(30, 4)
    bt, bv, side = W.x_sides(n)
    prev = np.inf
    for s in range(0, 60, 6):
        cut = O.crack_cut(xyz, E, W.grown_radii(discs, s, 1.05))
        st = O.hodge1(xyz, tets, E, kappa=kap, cut=cut)
        L, _ = O.assemble(V, E, st)
        A, b, _ = O.apply_bc(L, bt, bv, E, st)
        res = O.pcg(A, b, precond="jacobi", tol=1e-13)
        k = O.flux_effective_conductivity(res.x, E, st, side)["k_eff"]
        assert k <= prev * (1 + 1e-10)
        prev = k


def test_full_plane_crack_stops_the_flow():
    n = 4
    xyz, tets = W.kuhn_cube(n)
    V = len(xyz)
    E = O.edges_of(tets, V)
    cut = O.crack_cut(xyz, E, np.array([[0.501, 0.5, 0.5, 1.0, 0.0, 0.0, 2.0]]))
    s = O.hodge1(xyz, tets, E, cut=cut)
    bt, bv, side = W.x_sides(n)
    A, b, pinned = O.apply_bc(O.assemble(V, E, s)[0], bt, bv, E, s)
    assert not pinned.any()
    res = O.pcg(A, b, precond="jacobi", tol=1e-13)
    f = O.flux_effective_conductivity(res.x, E, s, side)
    assert f["k_eff"] < 1e-20
    i, _, _ = W.lattice_index(n)
    assert np.allclose(res.x, (i <= 2).astype(float), atol=1e-12)


def test_isolated_vertex_is_pinned():
    n = 4
    xyz, tets = W.kuhn_cube(n)
    V = len(xyz)
    E = O.edges_of(tets, V)
    v = 2 + 5 * (2 + 5 * 2)  # the centre vertex
    cut = (E[:, 0] == v) | (E[:, 1] == v)
    s = O.hodge1(xyz, tets, E, cut=cut)
    bt, bv, side = W.x_sides(n)
    A, b, pinned = O.apply_bc(O.assemble(V, E, s)[0], bt, bv, E, s)
    assert pinned.sum() == 1 and pinned[v]
    res = O.pcg(A, b, precond="jacobi", tol=1e-12)
    assert res.x[v] == 0.0 and res.converged


def test_fsai_properties():
    # with the full lower pattern, FSAI is the exact inverse Cholesky factor: G A G^T = I
    rng = np.random.Generator(np.random.PCG64(9))
    B = rng.normal(size=(7, 7))
    A = sp.csr_matrix(B @ B.T + 7 * np.eye(7))
    G = O.fsai_factor(A, [np.arange(i + 1) for i in range(7)])
    assert np.allclose((G @ A @ G.T).toarray(), np.eye(7), atol=1e-12)
    p = _problem(6, sigma=1.0, n_cracks=15)
    G = O.fsai_factor(p["A"])
    Gd = G.toarray()
    assert np.all(np.triu(Gd, 1) == 0)
    assert np.allclose((G @ p["A"] @ G.T).diagonal(), 1.0, rtol=1e-12)
    pat = O.fsai_pattern(p["A"])
    assert all(np.array_equal(G.indices[G.indptr[i]:G.indptr[i + 1]], pat[i]) for i in range(len(pat)))
    res_j = O.pcg(p["A"], p["b"], precond="jacobi", tol=1e-12)
    res_f = O.pcg(p["A"], p["b"], precond=O.krylov.fsai_apply(G), tol=1e-12)
    assert res_f.converged and res_f.iterations < res_j.iterations
    assert np.linalg.norm(res_f.x - res_j.x) <= 1e-10 * np.linalg.norm(res_j.x)


@pytest.mark.parametrize("precond", ["jacobi", "fsai"])
def test_iterative_refinement_reaches_fp64_accuracy(precond):
    p = _problem(8, sigma=1.0, n_cracks=25)
    ref = O.pcg(p["A"], p["b"], precond="jacobi", tol=1e-14, stagnation=50)
    x, outer, inner, rel = O.iterative_refinement(p["A"], p["b"], tol=1e-10, precond=precond)
    assert rel <= 1e-10 and outer >= 2 and len(inner) == outer
    # the error is bounded by ||A^-1|| ||b - A x|| (A SPD, smallest eigenvalue by dense solve)
    lam_min = np.linalg.eigvalsh(p["A"].toarray())[0]
    r = np.linalg.norm(p["b"] - p["A"] @ x)
    assert np.linalg.norm(x - ref.x) <= 1.01 * r / lam_min + 1e-13 * np.linalg.norm(ref.x)


def test_neumann_inflow_linear_solution():
    n = 4
    xyz, tets = W.kuhn_cube(n)
    V = len(xyz)
    E = O.edges_of(tets, V)
    s = O.hodge1(xyz, tets, E)
    i, _, _ = W.lattice_index(n)
    bt = np.where(i == n, 1, np.where(i == 0, 2, 0)).astype(np.int8)
    bv = np.zeros(V)
    q = 2.5
    f0 = np.where(i == 0, -q, 0.0)  # outward normal flux -q on x = 0: heat flows in
    g = O.neumann_load(xyz, tets, O.boundary_faces(tets), bt, f0)
    assert abs(g.sum() + q) < 1e-13  # total inflow q over the unit face
    A, b, _ = O.apply_bc(O.assemble(V, E, s)[0], bt, bv, E, s, neumann=g)
    res = O.pcg(A, b, precond="jacobi", tol=1e-13)
    assert np.abs(res.x - q * (1 - i / n)).max() < 1e-10
    # k_eff with a Neumann load is the flux density through the Dirichlet side (x = 1, the only
    # one) over the gradient: q through the unit face over dT = q, i.e. 1
    side = np.where(i == n, 2, 0).astype(np.int8)
    f = O.flux_effective_conductivity(res.x, E, s, side, dT=q, neumann=True)
    assert abs(f["q_out"] - q) < 1e-9 and abs(f["k_eff"] - 1.0) < 1e-9


def test_keff_with_a_neumann_load_is_the_prescribed_flux_through_the_dirichlet_side():
    """Lognormal conductivity, T = 1 / 0 on x = 0 / 1, outward flux densities prescribed on y = 0
    and z = 1.  L has zero row sums, so the balances of all vertices add up to zero: the flux
    leaving through the two Dirichlet sides, Q_out - Q_in, equals the prescribed inflow
    -sum(g).  k_eff is Q_in length / (area dT) (the energy form, which also holds the work of the
    prescribed fluxes, differs), and Q_out without a marked inflow face."""
    n = 6
    xyz, tets = W.kuhn_cube(n)
    V = len(xyz)
    E = O.edges_of(tets, V)
    s = O.hodge1(xyz, tets, E, kappa=W.lognormal_kappa(len(E), 1.0, 9))
    i, j, k = W.lattice_index(n)
    bt0, bv, side = W.x_sides(n)
    bt = np.where(bt0 == 1, 1, np.where((j == 0) | (k == n), 2, 0)).astype(np.int8)
    f0 = np.where(bt == 2, np.where(j == 0, -0.8, 0.3), 0.0)
    g = O.neumann_load(xyz, tets, O.boundary_faces(tets), bt, f0)
    A, b, pinned = O.apply_bc(O.assemble(V, E, s)[0], bt, bv, E, s, neumann=g)
    assert not pinned.any()
    x = O.pcg(A, b, precond="jacobi", tol=1e-14, stagnation=50).x
    f = O.flux_effective_conductivity(x, E, s, side, neumann=True)
    assert abs((f["q_out"] - f["q_in"]) + g.sum()) < 1e-10
    assert f["k_eff"] == f["q_in"] and abs(f["energy"] - f["q_in"]) > 1e-3
    f2 = O.flux_effective_conductivity(x, E, s, np.where(side == 2, 2, 0), neumann=True)
    assert f2["k_eff"] == f2["q_out"] == f["q_out"]
    assert np.isnan(O.flux_effective_conductivity(x, E, s, np.zeros(V, np.int8), neumann=True)["k_eff"])


def test_neumann_faces_next_to_dirichlet():
    # Neumann on x = 0 and Dirichlet on y = 0: faces of x = 0 that touch y = 0 still carry flux
    n = 3
    xyz, tets = W.kuhn_cube(n)
    i, j, _ = W.lattice_index(n)
    bt = np.where(j == 0, 1, np.where(i == 0, 2, 0)).astype(np.int8)
    f0 = np.where(bt == 2, 1.0, 0.0)
    g = O.neumann_load(xyz, tets, O.boundary_faces(tets), bt, f0)
    # the whole x = 0 face is Neumann; its Dirichlet row j = 0 keeps no load
    h2 = 1.0 / n ** 2
    assert abs(g.sum() - (1.0 - (n + 1 - 1) * h2 / 2 - 0 * h2)) < 1e-13
    assert np.all(g[bt != 2] == 0.0)
