"""Full-size checks of the tet-unknown path (Section 2.3, eq. 11-13) on the 128^3 workload and in
the configuration `bench.py --dual` times: face conductivity lognormal (sigma 1, seed 1), 200 discs
(seed 2), T = 1 / 0 on x = 0 / 1, block Jacobi, A-norm test at 1e-10.

The oracle cannot assemble a system of 12.6M tets, so: counts against the Kuhn closed forms (every
face inside a cube limited, every cube one block of six); the face numbering checked over all
faces (owner order, neighbour consistency on a sample); weights and cut flags of 20,000 seeded
faces recomputed by the oracle from their tets alone; and properties that hold at any size for the
solution: the discrete maximum principle (all weights are >= 0, so 0 <= T <= 1 up to rounding),
Q_in and Q_out against the energy E within the bound the A-norm test implies (Cauchy-Schwarz:
|Q - E| <= sqrt(sum of the side's W_f) e + e^2 with e = 10 tol ||T||_A), and bit-identical
repeated solves.
"""
import numpy as np
import pytest
import torch

import workloads as W
from oracle import dual as D

pytestmark = pytest.mark.gpu
N = 128
TOL = 1e-10


@pytest.fixture(scope="module")
def tets128(dev):
    import paper_2104_05999_amd as dec
    ctx = dec.Context(dev)
    xyz, tets = W.kuhn_cube(N)
    F = W.kuhn_counts(N)["F"]
    kappa = W.lognormal_kappa(F, 1.0, 1)
    cracks = W.penny_cracks(200, 2)
    bt, bv, side = W.x_sides(N)
    t = lambda a: torch.as_tensor(np.ascontiguousarray(a), device=dev)  # noqa: E731
    m = ctx.mesh(t(xyz), t(tets))
    d = m.dual(t(bt), t(bv), t(side), t(kappa), t(cracks))
    m.close()
    T, st, rc = d.solve(tol=TOL, check=False)
    ft, fl, w, cut = (a.cpu().numpy() for a in d.faces())
    yield dict(ctx=ctx, d=d, T=T, st=st, rc=rc, xyz=xyz, tets=tets, kappa=kappa, cracks=cracks, bt=bt, bv=bv,
               side=side, ft=ft, fl=fl, w=w, cut=cut)
    d.close()
    ctx.close()


def test_counts(tets128):
    d = tets128["d"]
    c = W.kuhn_counts(N)
    assert d.V == c["T"] and d.F == c["F"] and d.F_boundary == 12 * N * N
    assert d.info() == {"faces": c["F"], "limited": 6 * N ** 3, "blocks": N ** 3, "max_block": 6}


def test_face_numbering(tets128):
    ft, fl, tets = tets128["ft"], tets128["fl"], tets128["tets"]
    t1, t2, k1, k2 = ft[:, 0].astype(np.int64), ft[:, 1].astype(np.int64), fl[:, 0], fl[:, 1]
    key = t1 * 4 + k1
    assert (np.diff(key) > 0).all()                      # owner order, each (tet, local face) once
    inner = t2 >= 0
    assert (t1[inner] < t2[inner]).all() and ((k2 >= 0) == inner).all()
    assert int((~inner).sum()) == 12 * N * N
    rng = np.random.Generator(np.random.PCG64(3))
    for f in rng.choice(np.flatnonzero(inner), 2000, replace=False):
        a = set(tets[t1[f]]) - {tets[t1[f], k1[f]]}
        b = set(tets[t2[f]]) - {tets[t2[f], k2[f]]}
        assert a == b and len(a) == 3


def test_sampled_weights_and_cuts(tets128):
    """The oracle's face geometry, cut predicate and boundary rule on 20,000 seeded faces, from
    their own tets (remapped into a small tet array)."""
    ft, fl, w, cut, tets, xyz = (tets128[k] for k in ("ft", "fl", "w", "cut", "tets", "xyz"))
    rng = np.random.Generator(np.random.PCG64(5))
    cut_ids = np.flatnonzero(cut)
    sample = np.unique(np.concatenate([rng.choice(len(w), 20000, replace=False), cut_ids[:2000]]))
    t1, t2 = ft[sample, 0].astype(np.int64), ft[sample, 1].astype(np.int64)
    k1, k2 = fl[sample, 0], fl[sample, 1]
    used = np.unique(np.concatenate([t1, t2[t2 >= 0]]))
    sub = tets[used]
    r1 = np.searchsorted(used, t1)
    r2 = np.where(t2 >= 0, np.searchsorted(used, np.maximum(t2, 0)), -1)
    loc = np.array([[j for j in range(4) if j != k] for k in range(4)])
    verts = sub[r1[:, None], loc[k1]]
    faces = (r1, k1, r2, k2, verts)
    geo = D.face_geometry(xyz, sub, faces)
    ocut = D.face_cut(xyz, sub, faces, geo, tets128["cracks"])
    assert np.array_equal(cut[sample].astype(bool), ocut) and ocut.sum() >= 100
    dirichlet = D.face_bc(faces, tets128["bt"], tets128["bv"], tets128["side"])[0]
    kap = np.where(ocut, 0.0, tets128["kappa"][sample])
    wo = np.where((r2 >= 0) | dirichlet, kap * geo["gw"], 0.0)
    assert np.array_equal(w[sample] == 0.0, wo == 0.0)
    assert np.abs(w[sample] - wo).max() <= 1e-14 * np.abs(wo).max()


def test_solution_properties(tets128):
    d, T, st, rc = tets128["d"], tets128["T"], tets128["st"], tets128["rc"]
    assert rc == 0, st
    assert 0.0 < st["rel_residual"] <= TOL
    Th = T.cpu().numpy()
    assert Th.min() >= -1e-12 and Th.max() <= 1.0 + 1e-12
    f = d.flux(T)
    ft, w, bt, bv, side, tets = (tets128[k] for k in ("ft", "w", "bt", "bv", "side", "tets"))
    t1, t2 = ft[:, 0], ft[:, 1]
    inner = t2 >= 0
    # ||T||_A^2 over the eliminated operator: the face energy of T with zero Dirichlet values
    dd = Th[t1[inner]] - Th[t2[inner]]
    bnd = ~inner & (w != 0.0)
    norm_a = np.sqrt((w[inner] * dd * dd).sum() + (w[bnd] * Th[t1[bnd]] ** 2).sum())
    e = 10.0 * TOL * norm_a
    loc = np.array([[j for j in range(4) if j != k] for k in range(4)])
    verts = tets[t1[~inner][:, None], loc[tets128["fl"][~inner, 0]]]
    sides = side[verts]
    for key, sd in (("q_in", 1), ("q_out", 2)):
        on = (sides == sd).all(axis=1) & (bt[verts] == 1).all(axis=1)
        bound = np.sqrt(w[~inner][on].sum()) * e + e * e
        assert abs(f[key] - f["energy"]) <= bound, (key, f, bound)
    assert 0.0 < f["k_eff"] < tets128["kappa"].max()


def test_repeated_solves_are_identical(tets128):
    d = tets128["d"]
    T2, st2, rc2 = d.solve(tol=TOL, check=False)
    assert rc2 == 0 and st2["iterations"] == tets128["st"]["iterations"]
    assert torch.equal(T2, tets128["T"])
