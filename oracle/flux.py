"""Oracle flux and effective conductivity (test infrastructure).

Section 2.5: in the unit-cube conduction test with T fixed on two opposite
faces and the other four insulated, the effective conductivity equals the
flux density through either Dirichlet face.  With vertex unknowns the heat
leaving vertex v through its dual cell is (L_full T)_v, L_full the operator
before any boundary elimination, so
    Q_in  =  sum over inflow-face vertices of (L_full T)_v,
    Q_out = -sum over outflow-face vertices of (L_full T)_v,
and, when no Neumann flux is prescribed, the dissipated energy
E = sum_e *1_e (T_hi - T_lo)^2 equals Q_in dT at the exact discrete
solution.  The reported conductivity is the flux density through a Dirichlet
side over the gradient, k_eff = Q length / (area dT), with Q = Q_in (or
Q_out when no inflow face is marked: the paper allows either side); without
a Neumann load it is taken in the energy form k_eff = E length / (area dT^2),
the same number at the exact solution and second order in the solution's
error (with a Neumann load the energy also holds the work of the prescribed
fluxes).
"""
import numpy as np


def flux_effective_conductivity(T, edges, star1, side, length=1.0, area=1.0, dT=1.0, neumann=False):
    """Return dict(k_eff, q_in, q_out, energy, edge_flux) with edge_flux_e = *1_e (T_lo - T_hi);
    ``neumann``: the system carries a Neumann load (k_eff from Q_in, else from E)."""
    T = np.asarray(T, dtype=np.float64)
    edges = np.asarray(edges, dtype=np.int64)
    star1 = np.asarray(star1, dtype=np.float64)
    lo, hi = edges[:, 0], edges[:, 1]
    flow = star1 * (T[lo] - T[hi])  # heat carried from lo to hi
    V = len(T)
    out_of = np.bincount(lo, weights=flow, minlength=V) - np.bincount(hi, weights=flow, minlength=V)
    side = np.asarray(side)
    q_in = float(out_of[side == 1].sum())
    q_out = float(-out_of[side == 2].sum())
    dTe = T[hi] - T[lo]
    energy = float((star1 * dTe * dTe).sum())
    return {
        "k_eff": energy * length / (area * dT * dT) if not neumann else
                 (q_in if (side == 1).any() else q_out if (side == 2).any() else np.nan) * length / (area * dT),
        "q_in": q_in,
        "q_out": q_out,
        "energy": energy,
        "edge_flux": flow,
    }
