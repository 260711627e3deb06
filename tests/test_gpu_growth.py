"""Crack growth: 1000 penny discs grown by 2% per step, each step warm-started from the last.

64^3 replica: against stored oracle values (tests/golden/growth64.*, written
by tests/golden/make_golden_growth.py from the oracle only) -- cut and
pinned counts and the first/last cut sets bit-exact, the solution on a seeded
sample S of 65,536 vertices to ||x_S - x*_S||_2 <= 1e-10 ||x*_S||_2 (GPU to
1e-14), k_eff to 1e-9 of the uncracked value.

256^3 (16,974,593 vertices): counts against the closed forms, the cut
flags of 20,000 seeded lattice edges against the oracle predicate, the
solver's product (the sliced-ELL copy in the encoding the autotuner picked,
one-byte offset indices on this lattice) equal to the CSR product bit for bit
and, on 256 seeded interior rows, to the oracle's row of A (its *1 from the
row's own tets, kappa and grown discs) to 1e-13; the solutions balance those
oracle rows (right-hand side 0) to within tol ||b||_2, which bounds every
entry of the residual; and properties that hold at any size: the FP64
residual, Rayleigh monotonicity of k_eff as cracks grow, Q_in = Q_out = E,
mixed precision agreeing with FP64.
"""
import json
import os

import numpy as np
import pytest
import torch

import oracle as O
import workloads as W

pytestmark = pytest.mark.gpu
HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def ctx(dev):
    import paper_2104_05999_amd as dec
    c = dec.Context(dev)
    yield c
    c.close()


def _mesh(ctx, dev, n):
    xyz, tets = W.kuhn_cube(n, device=dev)
    m = ctx.mesh(xyz, tets)
    c = W.kuhn_counts(n)
    kappa = torch.as_tensor(W.lognormal_kappa(c["E"], 1.0, 1), device=dev)
    bt, bv, side = W.x_sides(n)
    t = lambda a: torch.as_tensor(a, device=dev)  # noqa: E731
    return m, kappa, t(bt), t(bv), t(side)


def _step(m, kappa, discs, s, dev, bt, bv, want_rhs=False):
    cut, _ = m.hodge1(kappa, torch.as_tensor(W.grown_radii(discs, s), device=dev), want_star=False)
    m.assemble()
    npin, b = m.apply_bc(bt, bv, want_rhs=want_rhs)
    return (cut, npin, b) if want_rhs else (cut, npin)


def test_growth64_against_oracle(ctx, dev):
    meta = json.load(open(os.path.join(HERE, "golden", "growth64.json")))
    arr = np.load(os.path.join(HERE, "golden", "growth64.npz"))
    n = meta["n"]
    m, kappa, bt, bv, side = _mesh(ctx, dev, n)
    discs = W.penny_cracks(1000, 4)
    vs = torch.as_tensor(arr["vertex_sample"], device=dev)
    k0 = meta["steps"]["0"]["k_eff"]
    T = torch.zeros(m.V, dtype=torch.float64, device=dev)
    steps = sorted(int(s) for s in meta["steps"])
    for s in steps:
        ref = meta["steps"][str(s)]
        cut, npin = _step(m, kappa, discs, s, dev, bt, bv)
        assert int(cut.sum()) == ref["n_cut"] and npin == ref["n_pinned"], s
        if f"cut_edges_{s}" in arr.files:
            assert np.array_equal(torch.nonzero(cut).flatten().cpu().numpy(), arr[f"cut_edges_{s}"])
        T, st, rc = m.solve(T=T, tol=1e-14, warm_start=1, check=False)
        assert rc == 0, (s, st)
        xs = arr[f"x_sample_{s}"]
        err = np.linalg.norm(T[vs].cpu().numpy() - xs) / np.linalg.norm(xs)
        print(f"step {s}: sample error {err:.3e} (oracle 1e-10 solve {ref['loose_sample_error_vs_ref']:.3e})",
              flush=True)
        assert err <= 1e-10, (s, err)
        f = m.flux(T, side)
        assert abs(f["k_eff"] - ref["k_eff"]) <= 1e-9 * k0, s
        assert abs(f["q_in"] - ref["q_in"]) <= 1e-9 * k0 and abs(f["q_out"] - ref["q_out"]) <= 1e-9 * k0
    # the last step again in mixed precision, cold
    Tm, st, rc = m.solve(tol=1e-14, precision=1, check=False)
    assert rc == 0
    xs = arr[f"x_sample_{steps[-1]}"]
    err = np.linalg.norm(Tm[vs].cpu().numpy() - xs) / np.linalg.norm(xs)
    print(f"step {steps[-1]} mixed: sample error {err:.3e}", flush=True)
    assert err <= 1e-10, err
    m.close()


def _kuhn_edge_sample(n, count, seed):
    """Seeded lattice edges (lo, hi) of the Kuhn split: v -> v + d for the seven directions it uses."""
    rng = np.random.Generator(np.random.PCG64(seed))
    dirs = np.array([[1, 0, 0], [0, 1, 0], [0, 0, 1], [1, 1, 0], [1, 0, 1], [0, 1, 1], [1, 1, 1]])
    ijk = rng.integers(0, n, size=(count, 3))
    d = dirs[rng.integers(0, 7, size=count)]
    m = n + 1
    lo = ijk[:, 2] + m * (ijk[:, 1] + m * ijk[:, 0])
    hj = ijk + d
    hi = hj[:, 2] + m * (hj[:, 1] + m * hj[:, 0])
    return np.stack([lo, hi], axis=1)


def _oracle_rows(xyz, tets, n, rows, edge_keys, kappa, discs):
    """Rows `rows` of the eliminated operator A from the oracle, for interior vertices whose
    neighbours are all free (lattice index 2..n-2 along x): {row: (cols, vals)}.  A vertex's
    tets are those of the 8 cubes around it that hold it; every edge at the vertex has all its
    tets there, so its *1 is complete."""
    m = n + 1
    out = {}
    for v in rows:
        a, b, c = v // (m * m), (v // m) % m, v % m
        cubes = [(k + n * (j + n * i)) for i in (a - 1, a) for j in (b - 1, b) for k in (c - 1, c)]
        cand = tets[np.concatenate([np.arange(6 * q, 6 * q + 6) for q in cubes])]
        pt = cand[(cand == v).any(axis=1)].astype(np.int64)
        E = O.edges_of(pt, len(xyz))
        at = (E == v).any(axis=1)
        ids = np.searchsorted(edge_keys, E[:, 0] * len(xyz) + E[:, 1])
        cut = O.crack_cut(xyz, E, discs)
        star = O.hodge1(xyz, pt, E, kappa=kappa[ids], cut=cut)
        other = np.where(E[at, 0] == v, E[at, 1], E[at, 0])
        cols = np.concatenate([[v], other])
        vals = np.concatenate([[star[at].sum()], -star[at]])
        out[v] = (cols, vals)
    return out


def test_growth256_properties(ctx, dev):
    import paper_2104_05999_amd as dec
    n = 256
    m, kappa, bt, bv, side = _mesh(ctx, dev, n)
    c = W.kuhn_counts(n)
    assert (m.V, m.T, m.E, m.F, m.nnz) == (c["V"], c["T"], c["E"], c["F"], c["nnz"])
    discs = W.penny_cracks(1000, 4)
    xyz, tets_h = W.kuhn_cube(n)
    sample = _kuhn_edge_sample(n, 20000, 99)
    edges = m.edges().cpu().numpy().astype(np.int64)
    keys = edges[:, 0] * m.V + edges[:, 1]
    ids = np.searchsorted(keys, sample[:, 0] * m.V + sample[:, 1])
    assert np.array_equal(keys[ids], sample[:, 0] * m.V + sample[:, 1])
    T = torch.zeros(m.V, dtype=torch.float64, device=dev)
    prev, k0 = np.inf, None
    for s in (0, 10, 20, 30, 40, 50):
        cut, npin, b = _step(m, kappa, discs, s, dev, bt, bv, want_rhs=True)
        want = O.crack_cut(xyz, sample, W.grown_radii(discs, s))
        assert np.array_equal(cut.cpu().numpy()[ids].astype(bool), want), s
        ref = None
        if s in (0, 50):
            x = torch.as_tensor(np.random.default_rng(7 + s).standard_normal(m.V), device=dev)
            y = m.spmv(x)
            assert torch.equal(y, m.spmv(x, fmt=dec.DEC_FMT_CSR)), s  # sliced ELL = CSR, bit for bit
            rng = np.random.default_rng(11 + s)
            ijk = rng.integers(2, n - 1, size=(256, 3))
            rows = np.unique(ijk[:, 2] + (n + 1) * (ijk[:, 1] + (n + 1) * ijk[:, 0]))
            ref = _oracle_rows(xyz, tets_h, n, rows, keys, kappa.cpu().numpy(), W.grown_radii(discs, s))
            xh, yh, bh = x.cpu().numpy(), y.cpu().numpy(), b.cpu().numpy()
            pinned = 0
            for v, (cols, vals) in ref.items():
                if yh[v] == xh[v] and bh[v] == 0.0:
                    # a vertex of a part the cracks cut off from every Dirichlet vertex: pinned, an
                    # identity row (pinning is a global property; its sets are checked against the
                    # oracle on the 64^3 replica)
                    pinned += 1
                    continue
                want_y = float(np.dot(vals, xh[cols]))
                scale = float(np.dot(np.abs(vals), np.abs(xh[cols])))
                assert abs(yh[v] - want_y) <= 1e-13 * scale, (s, v, yh[v], want_y)
            print(f"step {s}: {len(ref) - pinned} sampled rows against the oracle, {pinned} pinned", flush=True)
            assert pinned <= len(ref) // 4, pinned
        T, st, rc = m.solve(T=T, tol=1e-10, warm_start=1)
        assert rc == 0 and st["rel_residual"] <= 1e-10
        if ref is not None:
            # the solution balances the oracle's equations on the sampled rows (right-hand side 0
            # there): each row's residual is below the global bound tol ||b||_2
            bn = float(torch.linalg.norm(b))
            Th = T.cpu().numpy()
            worst = max(abs(float(np.dot(vals, Th[cols]))) for cols, vals in ref.values())
            print(f"step {s}: largest sampled row residual of the oracle's operator {worst:.3e} "
                  f"(tol ||b|| = {1e-10 * bn:.3e})", flush=True)
            assert worst <= 1e-10 * bn, (s, worst, bn)
        f = m.flux(T, side)
        assert f["k_eff"] <= prev * (1 + 1e-9), (s, f["k_eff"], prev)
        prev = f["k_eff"]
        k0 = f["k_eff"] if k0 is None else k0
        # the boundary fluxes are first-order in the residual; bound them on the uncracked flux scale
        assert abs(f["q_in"] - f["energy"]) <= 1e-6 * k0, s
        assert abs(f["q_out"] - f["energy"]) <= 1e-6 * k0, s
    Tm, stm, rc = m.solve(tol=1e-10, precision=1)  # cold, mixed precision
    fm = m.flux(Tm, side)
    assert rc == 0 and abs(fm["k_eff"] - prev) <= 1e-9 * max(prev, 1e-12) + 1e-12
    m.close()
