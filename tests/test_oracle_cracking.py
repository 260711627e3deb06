"""Pins of the oracle cracking processes (Section 3: deterministic and stochastic cracking;
Section 2.5: a crack is a dual face of zero conductivity).  CPU only."""
import numpy as np

import oracle as O
import workloads as W
from oracle import cracking as C


def _system(n, kappa=None):
    xyz, tets = W.kuhn_cube(n)
    bt, bv, side = W.x_sides(n)
    E = len(O.edges_of(tets, len(xyz)))
    return C.CrackingSystem(xyz, tets, np.ones(E) if kappa is None else kappa, bt, bv, side)


def _axis(s):
    d = s.xyz[s.edges[:, 1]] - s.xyz[s.edges[:, 0]]
    return [(np.abs(d[:, a]) > 0) & (np.abs(d[:, (a + 1) % 3]) == 0) & (np.abs(d[:, (a + 2) % 3]) == 0)
            for a in range(3)]


def test_flux_density_of_the_linear_solution():
    """T = 1 - x on a homogeneous cube: the flux density is kappa = 1 through every face of an
    x edge and 0 through the faces of y and z edges; the diagonals have no face."""
    s = _system(4)
    T, f = s.solve()
    assert abs(f["k_eff"] - 1.0) < 1e-12
    dens = C.flux_density(T, s.edges, s.star1, s.area)
    fx = C.faces(s.area)
    x, y, z = _axis(s)
    assert np.array_equal(fx, x | y | z)  # Kuhn diagonals have zero dual area
    assert np.allclose(dens[x], 1.0, rtol=1e-12)
    assert np.nanmax(dens[y | z]) < 1e-12
    e, d = C.max_flux_edge(T, s.edges, s.star1, s.area)
    assert e == int(np.flatnonzero(x)[np.argmax(dens[x] == dens[x].max())]) and abs(d - dens[x].max()) == 0
    # scaling the conductivity scales the density
    s2 = _system(4, kappa=np.full(len(s.edges), 3.0))
    T2, _ = s2.solve()
    assert np.allclose(C.flux_density(T2, s2.edges, s2.star1, s2.area)[x], 3.0, rtol=1e-12)


def test_max_flux_edge_ties_and_eligibility():
    s = _system(2)
    T = np.linspace(0.0, 1.0, s.V) ** 2
    dens = C.flux_density(T, s.edges, s.star1, s.area)
    e, d = C.max_flux_edge(T, s.edges, s.star1, s.area)
    ok = C.faces(s.area)
    assert d == np.nanmax(dens[ok]) and e == int(np.flatnonzero(ok & (dens == d))[0])
    elig = ok.copy()
    elig[e] = False
    e2, d2 = C.max_flux_edge(T, s.edges, s.star1, s.area, eligible=elig)
    assert e2 != e and d2 <= d
    assert C.max_flux_edge(T, s.edges, s.star1, s.area, eligible=np.zeros(len(ok), bool))[0] == -1


def test_deterministic_process_cuts_one_cross_section():
    """Homogeneous 3^3 cube: the largest-flux rule cracks exactly one full cross-section of
    (n+1)^2 x-edge faces, after which no conductive path joins the two Dirichlet faces."""
    n = 3
    s = _system(n)
    path, k_end = C.cracking_process(s, 500)
    assert len(path) == (n + 1) ** 2 and k_end <= C.ZERO_REL
    ks = [k for _, k in path] + [k_end]
    assert all(a >= b - 1e-13 for a, b in zip(ks, ks[1:]))  # Rayleigh: cracking never raises k_eff
    x, _, _ = _axis(s)
    cracked = np.array([e for e, _ in path])
    assert x[cracked].all()
    lo_x = s.xyz[s.edges[cracked, 0], 0]
    assert np.unique(np.round(lo_x, 12)).size == 1  # one plane
    # the graph of uncracked faces no longer joins the face x = 0 to the face x = 1
    cut_off = O.isolated_components(s.V, s.edges, s.star1, s.xyz[:, 0] == 0.0)
    assert cut_off[s.xyz[:, 0] == 1.0].all()


def test_stochastic_path_follows_its_order_and_stops_at_separation():
    n = 3
    s = _system(n)
    x, y, z = _axis(s)
    plane = np.flatnonzero(x & (np.round(s.xyz[s.edges[:, 0], 0], 12) == np.round(1.0 / n, 12)))
    assert len(plane) == (n + 1) ** 2
    rng = np.random.Generator(np.random.PCG64(5))
    others = np.flatnonzero(C.faces(s.area) & ~np.isin(np.arange(len(s.edges)), plane))
    order = np.concatenate([rng.permutation(others)[:10], rng.permutation(plane)])
    path, k_end = C.cracking_process(s, len(order) + 5, order=order)
    assert [e for e, _ in path] == list(order)  # stops exactly when the plane is complete
    assert k_end <= C.ZERO_REL and path[-1][1] > 0.05
    ks = [k for _, k in path]
    assert all(a >= b - 1e-13 for a, b in zip(ks, ks[1:]))
