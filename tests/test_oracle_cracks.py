"""Pins of the oracle's crack predicate (CPU)."""
import numpy as np

import oracle as O
import workloads as W


def _one(p0, p1, disc):
    xyz = np.array([p0, p1], dtype=float)
    return bool(O.crack_cut(xyz, np.array([[0, 1]]), np.array([disc], dtype=float))[0])


def test_hand_cases():
    disc = [0.5, 0.5, 0.5, 1.0, 0.0, 0.0, 0.25]
    assert _one([0.25, 0.5, 0.5], [0.75, 0.5, 0.5], disc)          # through the centre
    assert not _one([0.25, 0.5, 0.8], [0.75, 0.5, 0.8], disc)      # misses: 0.3 > r
    assert _one([0.25, 0.5, 0.75], [0.75, 0.5, 0.75], disc)        # exactly on the rim: inclusive
    assert not _one([0.5, 0.3, 0.5], [0.5, 0.7, 0.5], disc)        # lies in the plane
    assert not _one([0.5, 0.5, 0.5], [0.75, 0.5, 0.5], disc)       # starts on the plane, goes +
    assert _one([0.25, 0.5, 0.5], [0.5, 0.5, 0.5], disc)           # ends on the plane from -
    assert not _one([0.6, 0.5, 0.5], [0.9, 0.5, 0.5], disc)        # both on one side
    flipped = [0.5, 0.5, 0.5, -1.0, 0.0, 0.0, 0.25]
    assert _one([0.25, 0.5, 0.5], [0.75, 0.5, 0.5], flipped)
    assert _one([0.5, 0.5, 0.5], [0.75, 0.5, 0.5], flipped)        # on plane counts as + side


def test_random_against_line_plane_solve():
    rng = np.random.Generator(np.random.PCG64(11))
    P = rng.uniform(0, 1, size=(4000, 2, 3))
    xyz = P.reshape(-1, 3)
    edges = np.arange(len(xyz)).reshape(-1, 2)
    discs = W.penny_cracks(5, 12, 0.1, 0.4)
    got = np.zeros(len(edges), dtype=bool)
    for d in discs:
        got_d = O.crack_cut(xyz, edges, d[None])
        c, n, r = d[:3], d[3:6], d[6]
        # independent formulation: solve (p0 + t (p1 - p0) - c) . n = 0 for t in [0, 1] and
        # measure the in-plane distance of the hit point by projection
        a = P[:, 0] - c
        b = P[:, 1] - P[:, 0]
        den = b @ n
        t = -(a @ n) / den
        hit = P[:, 0] + t[:, None] * b
        dist = np.linalg.norm(hit - c, axis=1)
        want = (t >= 0) & (t <= 1) & (dist <= r)
        clear = (np.abs(dist - r) > 1e-9) & (np.abs(a @ n) > 1e-9) & (np.abs((P[:, 1] - c) @ n) > 1e-9)
        assert np.array_equal(got_d[clear], want[clear])
        got |= got_d
    assert np.array_equal(got, O.crack_cut(xyz, edges, discs))
    assert got.sum() > 50


def test_slab_filter_changes_nothing():
    n = 6
    xyz, tets = W.kuhn_cube(n)
    E = O.edges_of(tets, len(xyz))
    discs = W.penny_cracks(40, 3, 0.05, 0.3)
    fast = O.crack_cut(xyz, E, discs)
    slow = np.zeros(len(E), dtype=bool)
    p0, p1 = xyz[E[:, 0]], xyz[E[:, 1]]
    for d in discs:
        slow |= O.cracks._cut_by_disc(p0, p1, d)
    assert np.array_equal(fast, slow)
    sub = np.arange(0, len(E), 3)
    assert np.array_equal(O.crack_cut(xyz, E, discs, edge_ids=sub), slow[sub])


def test_full_plane_cut_brute_force():
    n = 4
    xyz, tets = W.kuhn_cube(n)
    E = O.edges_of(tets, len(xyz))
    x0 = 0.5 + 1e-3
    disc = np.array([[x0, 0.5, 0.5, 1.0, 0.0, 0.0, 2.0]])
    cut = O.crack_cut(xyz, E, disc)
    want = (xyz[E[:, 0], 0] < x0) != (xyz[E[:, 1], 0] < x0)
    assert np.array_equal(cut, want)
    assert cut.sum() > 0
