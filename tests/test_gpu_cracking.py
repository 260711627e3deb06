"""Cracking processes (Section 3) on the GPU against the oracle.

The largest-flux-density face must be a valid arg max of the oracle's flux
densities (several faces may tie up to rounding; ties go to the smallest edge
id on both sides, so away from ties the edges agree exactly).  Along a path,
both sides crack the same face, and k_eff after every crack agrees to 1e-9 of
the uncracked value.
"""
import numpy as np
import pytest
import torch

import oracle as O
import workloads as W
from oracle import cracking as C

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx(dev):
    import paper_2104_05999_amd as dec
    c = dec.Context(dev)
    yield c
    c.close()


def _setup(ctx, dev, n, sigma, seed):
    xyz, tets = W.kuhn_cube(n)
    bt, bv, side = W.x_sides(n)
    E = W.kuhn_counts(n)["E"]
    kappa = W.lognormal_kappa(E, sigma, seed) if sigma > 0 else np.ones(E)
    t = lambda a: torch.as_tensor(np.ascontiguousarray(a), device=dev)  # noqa: E731
    m = ctx.mesh(t(xyz), t(tets))
    sysm = C.CrackingSystem(xyz, tets, kappa, bt, bv, side)
    return m, sysm, t(kappa), t(bt), t(bv), t(side)


def _gpu_solve(m, kappa, bt, bv, side, T=None):
    m.hodge1(kappa, want_cut=False, want_star=False)
    m.assemble()
    m.apply_bc(bt, bv, want_rhs=False)
    T, st, rc = m.solve(T=T, tol=1e-13, warm_start=T is not None, check=False)
    assert rc == 0, st
    return T, m.flux(T, side)


def _valid_argmax(e, dens, eligible, rel=1e-9):
    ok = eligible & ~np.isnan(dens)
    return bool(ok[e]) and dens[e] >= dens[ok].max() * (1.0 - rel)


def test_max_flux_edge_matches_oracle(ctx, dev):
    m, s, kappa, bt, bv, side = _setup(ctx, dev, 6, 1.0, 3)
    try:
        T, _ = _gpu_solve(m, kappa, bt, bv, side)
        Th = T.cpu().numpy()
        dens = C.flux_density(Th, s.edges, s.star1, s.area)
        faces = C.faces(s.area) & (s.star1 != 0)
        e, d = m.max_flux_edge(T)
        eo, do = C.max_flux_edge(Th, s.edges, s.star1, s.area)
        assert e == eo and abs(d - do) <= 1e-13 * do
        # an explicit candidate set, and a temperature field with no ties at all
        rng = np.random.Generator(np.random.PCG64(8))
        elig = faces & (rng.random(len(faces)) < 0.3)
        e2, _ = m.max_flux_edge(T, torch.as_tensor(elig.astype(np.uint8), device=dev))
        assert e2 == C.max_flux_edge(Th, s.edges, s.star1, s.area, eligible=elig)[0]
        Tr = rng.random(s.V)
        e3, d3 = m.max_flux_edge(torch.as_tensor(Tr, device=dev))
        e3o, d3o = C.max_flux_edge(Tr, s.edges, s.star1, s.area)
        assert e3 == e3o and abs(d3 - d3o) <= 1e-13 * d3o
        assert _valid_argmax(e, dens, faces)
        assert m.max_flux_edge(T, torch.zeros(m.E, dtype=torch.uint8, device=dev))[0] == -1
    finally:
        m.close()


@pytest.mark.parametrize("n,sigma", [(3, 0.0), (5, 1.0)])
def test_deterministic_process_against_oracle(ctx, dev, n, sigma):
    m, s, kappa, bt, bv, side = _setup(ctx, dev, n, sigma, 5)
    try:
        T, f = _gpu_solve(m, kappa, bt, bv, side)
        To, fo = s.solve()
        k0 = fo["k_eff"]
        steps = 0
        while fo["k_eff"] > C.ZERO_REL * k0 and steps < 60:
            assert abs(f["k_eff"] - fo["k_eff"]) <= 1e-9 * k0, steps
            e, _ = m.max_flux_edge(T)
            dens = C.flux_density(To, s.edges, s.star1, s.area)
            assert _valid_argmax(e, dens, C.faces(s.area) & (s.star1 != 0)), steps
            kappa[e] = 0.0
            s.crack(e)
            T, f = _gpu_solve(m, kappa, bt, bv, side, T)
            To, fo = s.solve()
            steps += 1
        assert abs(f["k_eff"] - fo["k_eff"]) <= 1e-9 * k0
        if sigma == 0.0:  # homogeneous: at least one full cross-section, then no conduction
            assert steps >= (n + 1) ** 2 and f["k_eff"] <= 1e-9 * k0
    finally:
        m.close()


def test_stochastic_path_against_oracle(ctx, dev):
    n = 4
    m, s, kappa, bt, bv, side = _setup(ctx, dev, n, 0.5, 6)
    try:
        rng = np.random.Generator(np.random.PCG64(21))
        order = rng.permutation(np.flatnonzero(C.faces(s.area)))[:40]
        T, f = _gpu_solve(m, kappa, bt, bv, side)
        _, fo = s.solve()
        k0 = fo["k_eff"]
        ks = [f["k_eff"]]
        for e in order:
            kappa[int(e)] = 0.0
            s.crack(int(e))
            T, f = _gpu_solve(m, kappa, bt, bv, side, T)
            _, fo = s.solve()
            assert abs(f["k_eff"] - fo["k_eff"]) <= 1e-9 * k0
            ks.append(f["k_eff"])
        assert all(a >= b - 1e-12 * k0 for a, b in zip(ks, ks[1:]))
    finally:
        m.close()


def test_paths_from_parallel_threads_match_sequential(dev):
    """Cracking paths driven from several host threads, each with its own context and stream (as
    the benchmark runs its Monte Carlo paths), give the same k_eff after every crack, bit for bit,
    as the same paths run one after another."""
    import threading

    import paper_2104_05999_amd as dec
    n, paths, steps = 4, 4, 25
    xyz, tets = W.kuhn_cube(n)
    bt, bv, side = W.x_sides(n)
    E = W.kuhn_counts(n)["E"]
    rng = np.random.Generator(np.random.PCG64(12))
    orders = [rng.permutation(E)[:steps] for _ in range(paths)]

    def run(ctx, order):
        t = lambda a: torch.as_tensor(np.ascontiguousarray(a), device=dev)  # noqa: E731
        with torch.cuda.stream(ctx.stream):
            m = ctx.mesh(t(xyz), t(tets))
            kappa = torch.ones(m.E, dtype=torch.float64, device=dev)
            T, ks = None, []
            for e in order:
                kappa[int(e)] = 0.0
                m.hodge1(kappa, want_cut=False, want_star=False)
                m.assemble()
                m.apply_bc(t(bt), t(bv), want_rhs=False)
                T, st, rc = m.solve(T=T, tol=1e-10, warm_start=T is not None, check=False)
                ks.append(m.flux(T, t(side))["k_eff"] if rc == 0 else rc)
            m.close()
            torch.cuda.current_stream().synchronize()
        return ks

    c0 = dec.Context(dev, stream=torch.cuda.Stream(dev))
    seq = [run(c0, o) for o in orders]
    c0.close()
    ctxs = [dec.Context(dev, stream=torch.cuda.Stream(dev)) for _ in range(2)]
    par = [None] * paths

    def worker(tid):
        for i in range(tid, paths, 2):
            par[i] = run(ctxs[tid], orders[i])

    th = [threading.Thread(target=worker, args=(k,)) for k in range(2)]
    for x in th:
        x.start()
    for x in th:
        x.join()
    for c in ctxs:
        c.close()
    assert par == seq


def test_monte_carlo_paths_served_with_warm_starts(ctx, dev):
    """Monte Carlo paths as served requests (bench.served_paths: one request per step, warm-started
    from the path's last temperature, the topology copied from one prepared mesh), mixed precision
    at 1e-10: after every crack k_eff equals that of the same path solved step by step with
    dec_solve (FP64, warm-started) to 1e-9 of the uncracked value, and path 0 equals the oracle's
    step by step (direct solves)."""
    import bench
    n, paths, steps = 4, 4, 60
    rng = np.random.Generator(np.random.PCG64(31))
    xyz, tets = W.kuhn_cube(n)
    bt, bv, side = W.x_sides(n)
    E = W.kuhn_counts(n)["E"]
    s0 = C.CrackingSystem(xyz, tets, np.ones(E), bt, bv, side)
    faces = np.flatnonzero(C.faces(s0.area))
    orders = [rng.permutation(faces)[:steps] for _ in range(paths)]
    served = bench.served_paths(ctx, dev, n, orders, precision=1, max_steps=steps)
    assert served["status"] == 0 and served["steps"] == [steps] * paths
    t = lambda a: torch.as_tensor(np.ascontiguousarray(a), device=dev)  # noqa: E731
    for i, order in enumerate(orders):
        m = ctx.mesh(t(xyz), t(tets))
        kappa = torch.ones(E, dtype=torch.float64, device=dev)
        T, f = _gpu_solve(m, kappa, t(bt), t(bv), t(side))
        ks = [f["k_eff"]]
        for e in order:
            kappa[int(e)] = 0.0
            T, f = _gpu_solve(m, kappa, t(bt), t(bv), t(side), T)
            ks.append(f["k_eff"])
        m.close()
        k0 = ks[0]
        assert len(served["ks"][i]) == len(ks)
        assert max(abs(a - b) for a, b in zip(served["ks"][i], ks)) <= 1e-9 * k0, i
    s = C.CrackingSystem(xyz, tets, np.ones(E), bt, bv, side)
    _, fo = s.solve()
    ko = [fo["k_eff"]]
    for e in orders[0]:
        s.crack(int(e))
        ko.append(s.solve()[1]["k_eff"])
    assert max(abs(a - b) for a, b in zip(served["ks"][0], ko)) <= 1e-9 * ko[0]
