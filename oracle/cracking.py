"""Oracle cracking processes (test infrastructure only).

Section 2.5 models a crack as a dual face whose conductivity drops to zero;
Section 3 grows a crack population one face per step, re-solving the
steady state after each crack, until the domain stops conducting:

* deterministic: the face carrying the largest heat-flux density in the
  previous solution is cracked;
* stochastic (Monte Carlo): faces are cracked in a random order; each order
  is one path.

With the temperature on the vertices (the reading taken for the whole
path), the faces are the dual 2-cells *e of the primal edges.  The heat
through *e is *1_e (T_lo - T_hi), so its flux density is
    |*1_e (T_hi - T_lo)| / |*e| = kappa_e |T_hi - T_lo| / |e|.
Only dual cells of nonzero area are faces (an edge with |*e| = 0 carries no
heat whatever its conductivity).  A cracked face has kappa_e = 0.  The
damage parameter is D_n = cracked faces / faces.  Ties in the flux density
go to the smallest edge id.  Random orders are inputs (drawn by the caller).
The domain counts as non-conductive once k_eff <= 1e-12 of its uncracked
value (rounding keeps a separated domain's energy near, not at, zero).
"""
import numpy as np
import scipy.sparse.linalg as spla

from .flux import flux_effective_conductivity
from .geometry import dual_areas, edge_lengths
from .laplacian import apply_bc, assemble
from .topology import edges_of


def faces(area):
    """Mask of the edges whose dual cell is a face (nonzero area)."""
    return np.asarray(area) != 0.0


def flux_density(T, edges, star1, area):
    """|*1_e (T_hi - T_lo)| / |*e| per edge; NaN where |*e| = 0."""
    T = np.asarray(T, dtype=np.float64)
    edges = np.asarray(edges, dtype=np.int64)
    star1 = np.asarray(star1, dtype=np.float64)
    area = np.asarray(area, dtype=np.float64)
    d = T[edges[:, 1]] - T[edges[:, 0]]
    with np.errstate(divide="ignore", invalid="ignore"):
        return np.where(area != 0.0, np.abs(star1 * d) / np.abs(area), np.nan)


def max_flux_edge(T, edges, star1, area, eligible=None):
    """(edge, density) of the largest flux density over the eligible edges (default: faces
    not yet cracked, *1_e != 0); ties to the smallest edge id; (-1, nan) when none."""
    dens = flux_density(T, edges, star1, area)
    if eligible is None:
        eligible = faces(area) & (np.asarray(star1) != 0.0)
    ok = np.asarray(eligible, dtype=bool) & ~np.isnan(dens)
    if not ok.any():
        return -1, float("nan")
    idx = np.flatnonzero(ok)
    best = dens[idx].max()
    e = int(idx[dens[idx] == best][0])
    return e, float(best)


class CrackingSystem:
    """One mesh with fixed Dirichlet data whose conductivities are cracked face by face."""

    def __init__(self, xyz, tets, kappa, bc_type, bc_value, side):
        self.xyz = np.asarray(xyz, dtype=np.float64)
        self.tets = np.asarray(tets)
        self.V = len(self.xyz)
        self.edges = edges_of(self.tets, self.V)
        self.area = dual_areas(self.xyz, self.tets, self.edges)
        self.length = edge_lengths(self.xyz, self.edges)
        self.kappa = np.array(kappa, dtype=np.float64)
        self.bc_type, self.bc_value, self.side = bc_type, bc_value, side

    @property
    def star1(self):
        return self.kappa * (self.area / self.length)

    def n_faces(self):
        return int(faces(self.area).sum())

    def solve(self):
        """Direct sparse solve of the eliminated system; returns (T, flux dict)."""
        star = self.star1
        L, _ = assemble(self.V, self.edges, star)
        A, b, _ = apply_bc(L, self.bc_type, self.bc_value, self.edges, star)
        T = spla.spsolve(A.tocsc(), b)
        return T, flux_effective_conductivity(T, self.edges, star, self.side)

    def crack(self, e):
        self.kappa[e] = 0.0


ZERO_REL = 1e-12


def cracking_process(system, steps, order=None):
    """Run `steps` crack steps (fewer when the domain stops conducting or no face is left).

    order=None: deterministic (largest flux density); else the stochastic path that
    cracks order[0], order[1], ...  Returns a list of (edge cracked, k_eff before it),
    and the k_eff after the last crack.
    """
    path = []
    T, f = system.solve()
    k0 = f["k_eff"]
    for k in range(steps):
        if f["k_eff"] <= ZERO_REL * k0:
            break
        if order is None:
            e, _ = max_flux_edge(T, system.edges, system.star1, system.area)
        else:
            if k >= len(order):
                break
            e = int(order[k])
        if e < 0:
            break
        path.append((e, f["k_eff"]))
        system.crack(e)
        T, f = system.solve()
    return path, f["k_eff"]
