"""dec_solve_noalloc, the solve that allocates nothing, against dec_solve through the C ABI.

Two calls in a row on one context, the second on a smaller system, each
checked against dec_solve on the same system: ||x - x_ref||_2 <= 1e-10
||x_ref||_2 with both solved to 1e-14, and bit for bit where dec_solve takes
the same recurrence (Jacobi on A below 65,536 rows).  Then the refusals: a
system beyond the scratch's row maximum, options the call does not run, a
mesh without boundary data.
"""
import numpy as np
import pytest
import torch

import workloads as W

pytestmark = pytest.mark.gpu


def _system(ctx, dev, n, n_cracks, seed):
    xyz, tets = W.kuhn_cube(n, device=dev)
    m = ctx.mesh(xyz, tets)
    kappa = torch.as_tensor(W.lognormal_kappa(m.E, 1.0, seed), device=dev)
    cracks = torch.as_tensor(W.penny_cracks(n_cracks, seed + 1), device=dev)
    m.hodge1(kappa, cracks, want_cut=False, want_star=False)
    m.assemble()
    bt, bv, _ = W.x_sides(n)
    m.apply_bc(torch.as_tensor(bt, device=dev), torch.as_tensor(bv, device=dev), want_rhs=False)
    return m


def test_noalloc_matches_dec_solve_twice(dev):
    import paper_2104_05999_amd as dec

    ctx = dec.Context(dev)
    for n, cracks, seed in ((40, 60, 11), (20, 20, 13)):  # the second system is smaller
        print(f"[noalloc] n={n} V={(n + 1) ** 3}", flush=True)
        m = _system(ctx, dev, n, cracks, seed)
        ref, sref, rc = m.solve(tol=1e-14, check=False)
        assert rc == 0, sref
        T, st, rc = m.solve_noalloc(tol=1e-14, check=False)
        assert rc == 0, st
        assert st["rel_residual"] <= 1e-14
        err = float(torch.linalg.norm(T - ref) / torch.linalg.norm(ref))
        assert err <= 1e-10, (n, err)
        if m.V < 65536:  # dec_solve runs the same recurrence here: the same bits
            assert torch.equal(T, ref), n
            assert st["iterations"] == sref["iterations"]
        # warm start from the solution: nothing left to do
        T2, st2, rc = m.solve_noalloc(T=T.clone(), tol=1e-14, warm_start=1, check=False)
        assert rc == 0 and st2["iterations"] <= 2 and float(torch.linalg.norm(T2 - T)) <= 1e-12 * float(torch.linalg.norm(T))
        m.close()
    ctx.close()


def test_noalloc_refusals(dev):
    import paper_2104_05999_amd as dec

    ctx = dec.Context(dev)
    m = _system(ctx, dev, 6, 2, 3)
    for kw in ({"precision": dec.DEC_PREC_MIXED}, {"precond": dec.DEC_PRECOND_FSAI}, {"profile": 1},
               {"norm": dec.DEC_NORM_ENERGY}):
        _, _, rc = m.solve_noalloc(check=False, **kw)
        assert rc == -1, kw
    m.close()
    xyz, tets = W.kuhn_cube(6, device=dev)
    bare = ctx.mesh(xyz, tets)
    _, _, rc = bare.solve_noalloc(check=False)
    assert rc == -8  # DEC_ESTATE: no boundary data yet
    bare.close()
    n = 161  # (n + 1)^3 = 4,251,528 rows, beyond the maximum
    xyz, tets = W.kuhn_cube(n, device=dev)
    big = ctx.mesh(xyz, tets)
    assert big.V > dec._lib.DEC_NOALLOC_MAX_ROWS
    with pytest.raises(dec.DecError, match="exceed the scratch's maximum"):
        big.solve_noalloc()
    big.close()
    del xyz, tets
    ctx.close()
