"""Degenerate inputs of the vertex path (Section 2: the 0-form Laplacian with Dirichlet data), solved
by dec_solve and by the server, against the oracle.

- An empty mesh is refused (DEC_EINVAL) before anything runs on the device.
- One regular tetrahedron, two Dirichlet vertices and two free ones: the smallest system with
  unknowns; every circumcentric dual area is positive, so the 2 x 2 system is SPD.  The oracle's
  value is the dense solve of that system.
- Every vertex Dirichlet: no unknowns, so the solve must return the data itself, bit for bit, in
  zero iterations, and the flux must be the oracle's flux of that field.
- Zero data (b = 0): the solution is exactly zero, and the solve reports success.
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


def _oracle(xyz, tets, bt, bv):
    V = len(xyz)
    E = O.edges_of(tets, V)
    star = O.hodge1(xyz, tets, E)
    A, b, pinned = O.apply_bc(O.assemble(V, E, star)[0], bt, bv, E, star)
    return E, star, A, b, pinned


def _gpu_solve(ctx, dev, xyz, tets, bt, bv, **kw):
    m = ctx.mesh(_t(xyz, dev), _t(tets, dev))
    m.hodge1()
    m.assemble()
    m.apply_bc(_t(bt, dev), _t(bv, dev))
    return m, m.solve(**kw)


def _served(ctx, dev, xyz, tets, bt, bv, side, precision):
    import paper_2104_05999_amd as dec
    V = len(xyz)
    E = O.edges_of(tets, V)
    req = dict(xyz=_t(xyz, dev), tets=_t(tets, dev), kappa=_t(np.ones(len(E)), dev), bc_type=_t(bt, dev),
               bc_value=_t(bv, dev), side=_t(side, dev), T_out=torch.full((V,), 7.0, dtype=torch.float64,
                                                                          device=dev))
    srv = dec.Server(ctx, 1 << 30, tol=1e-12, precision=precision)
    srv.submit(req, user_tag=5)
    out = []
    for _ in range(100):
        srv.step()
        out += srv.poll()
        if out:
            break
    srv.close()
    assert len(out) == 1 and out[0]["user_tag"] == 5
    return req["T_out"].cpu().numpy(), out[0]


def test_empty_mesh_is_refused(ctx, dev):
    import paper_2104_05999_amd as dec
    with pytest.raises(dec.DecError) as ei:
        ctx.mesh(torch.empty((0, 3), dtype=torch.float64, device=dev),
                 torch.empty((0, 4), dtype=torch.int32, device=dev))
    assert ei.value.code == -1


REGULAR_TET = (np.array([[1.0, 1.0, 1.0], [1.0, -1.0, -1.0], [-1.0, -1.0, 1.0], [-1.0, 1.0, -1.0]]),
               np.array([[0, 1, 2, 3]], dtype=np.int32))


@pytest.mark.parametrize("precision,precond", [(0, 0), (0, 1), (1, 0)])
def test_one_regular_tet(ctx, dev, precision, precond):
    xyz, tets = REGULAR_TET
    assert np.linalg.det(xyz[1:] - xyz[0]) > 0
    bt = np.array([1, 1, 0, 0], np.int8)
    bv = np.array([1.0, 0.0, 0.0, 0.0])
    side = np.array([1, 2, 0, 0], np.int8)
    E, star, A, b, pinned = _oracle(xyz, tets, bt, bv)
    assert (star > 0).all() and not pinned.any()
    x_ref = np.linalg.solve(A.toarray(), b)
    assert np.allclose(x_ref[2:], 0.5)  # the free vertices are symmetric between the two values
    m, (T, st, rc) = _gpu_solve(ctx, dev, xyz, tets, bt, bv, tol=1e-12, precision=precision, precond=precond)
    assert rc == 0, st
    assert np.abs(T.cpu().numpy() - x_ref).max() <= 1e-12
    f = m.flux(T, _t(side, dev))
    of = O.flux_effective_conductivity(x_ref, E, star, side)
    for key in ("q_in", "q_out", "energy"):
        assert abs(f[key] - of[key]) <= 1e-12 * abs(of["energy"]), key
    m.close()
    Ts, res = _served(ctx, dev, xyz, tets, bt, bv, side, precision)
    assert res["status"] == 0 and np.abs(Ts - x_ref).max() <= 1e-12


@pytest.mark.parametrize("precision", [0, 1])
def test_every_vertex_dirichlet(ctx, dev, precision):
    n = 3
    xyz, tets = W.kuhn_cube(n)
    _, _, side = W.x_sides(n)
    bt = np.ones(len(xyz), np.int8)
    bv = 1.0 - xyz[:, 0] + 0.25 * xyz[:, 1] * xyz[:, 2]
    E, star, A, b, _ = _oracle(xyz, tets, bt, bv)
    assert np.array_equal(np.linalg.solve(A.toarray(), b), bv)
    m, (T, st, rc) = _gpu_solve(ctx, dev, xyz, tets, bt, bv, tol=1e-12, precision=precision)
    assert rc == 0 and st["iterations"] == 0, st
    assert np.array_equal(T.cpu().numpy(), bv)
    f = m.flux(T, _t(side, dev))
    of = O.flux_effective_conductivity(bv, E, star, side)
    for key in ("k_eff", "q_in", "q_out", "energy"):
        assert abs(f[key] - of[key]) <= 1e-12 * abs(of["energy"]), key
    m.close()
    Ts, res = _served(ctx, dev, xyz, tets, bt, bv, side, precision)
    assert res["status"] == 0 and res["inner_iterations"] == 0 and np.array_equal(Ts, bv)


@pytest.mark.parametrize("precision", [0, 1])
def test_zero_data_gives_zero(ctx, dev, precision):
    n = 4
    xyz, tets = W.kuhn_cube(n)
    bt, _, side = W.x_sides(n)
    bv = np.zeros(len(xyz))
    m, (T, st, rc) = _gpu_solve(ctx, dev, xyz, tets, bt, bv, tol=1e-10, precision=precision)
    assert rc == 0, st
    assert not T.cpu().numpy().any()
    m.close()
    Ts, res = _served(ctx, dev, xyz, tets, bt, bv, side, precision)
    assert res["status"] == 0 and not Ts.any()
