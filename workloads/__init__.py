"""Seeded synthetic inputs for the DEC diffusion path.

This module only *draws* inputs: Kuhn-split cube meshes, per-edge
conductivities, penny-shaped crack discs, Dirichlet side masks and serving
arrival traces.  It holds none of the method's arithmetic (no topology, no
Hodge star, no assembly, no solve), so that both the FP64 oracle and the HIP
path can be fed from it without sharing any of the method's code.

Stand-ins: the paper's meshes come from TetGen (Section 2.2) and are not
available; Kuhn-split unit cubes with the same vertex numbering the paper's
pre-processing produces (z fastest, then y, then x; Section 2.2) stand in for
them.  Cracks in the paper are single faces switched to zero conductivity
(Section 2.5); here they are penny-shaped discs whose cut edges get zero
conductivity.
"""
from __future__ import annotations

import itertools
from dataclasses import dataclass

import numpy as np

__all__ = [
    "kuhn_counts",
    "kuhn_cube",
    "lattice_index",
    "jitter_interior",
    "x_sides",
    "delaunay_cube",
    "delaunay_lattice",
    "x_faces",
    "lognormal_kappa",
    "penny_cracks",
    "grown_radii",
    "ServeRequestSpec",
    "serving_trace",
]


def kuhn_counts(n: int) -> dict:
    """Cell counts of the Kuhn-split n^3 cube (closed forms, used as input sizes)."""
    V = (n + 1) ** 3
    T = 6 * n ** 3
    E = 3 * n * (n + 1) ** 2 + 3 * n * n * (n + 1) + n ** 3
    F = 6 * n ** 3 + 6 * n * n * (n + 1)
    return {"V": V, "T": T, "E": E, "F": F, "nnz": V + 2 * E}


def lattice_index(n: int):
    """(i, j, k) lattice coordinates of every vertex; vertex id = k + (n+1)(j + (n+1) i)."""
    m = n + 1
    v = np.arange(m ** 3, dtype=np.int64)
    return v // (m * m), (v // m) % m, v % m


# Kuhn split of one cube: for each permutation (a, b, c) of the axes, in
# lexicographic order, the path 000 -> e_a -> e_a + e_b -> 111.
_PERMS = list(itertools.permutations(range(3)))


def kuhn_cube(n: int, device=None):
    """Unit cube split into n^3 cells, each cut into 6 Kuhn tetrahedra.

    Returns ``(xyz, tets)``: ``xyz`` float64 [V, 3] with x = i/n (exact at the
    faces), ``tets`` int32 [T, 4].  Cube (i, j, k) has id k + n(j + n i) and
    owns tets 6*id .. 6*id+5.  With ``device`` set, the arrays are torch
    tensors built on that device (integer work on the device, coordinates on
    the host and copied), otherwise numpy arrays.
    """
    m = n + 1
    i, j, k = lattice_index(n)
    xyz = np.stack([i / n, j / n, k / n], axis=1).astype(np.float64)
    steps = np.array([m * m, m, 1], dtype=np.int64)  # vertex-id stride per axis
    offs = []
    for a, b, c in _PERMS:
        offs.append([0, steps[a], steps[a] + steps[b], steps[a] + steps[b] + steps[c]])
    offs = np.array(offs, dtype=np.int64)  # [6, 4]
    if device is None:
        ci = np.arange(n ** 3, dtype=np.int64)
        base = (ci // (n * n)) * m * m + ((ci // n) % n) * m + ci % n
        tets = (base[:, None, None] + offs[None, :, :]).reshape(-1, 4).astype(np.int32)
        return xyz, tets
    import torch

    ci = torch.arange(n ** 3, dtype=torch.int64, device=device)
    base = (ci // (n * n)) * m * m + ((ci // n) % n) * m + ci % n
    offs_t = torch.as_tensor(offs, device=device)
    tets = (base[:, None, None] + offs_t[None, :, :]).reshape(-1, 4).to(torch.int32)
    return torch.as_tensor(xyz, device=device), tets


def jitter_interior(xyz: np.ndarray, n: int, amplitude: float, seed: int) -> np.ndarray:
    """Move every vertex not on the cube's boundary by U[-a, a]·h per axis."""
    rng = np.random.Generator(np.random.PCG64(seed))
    i, j, k = lattice_index(n)
    interior = (i > 0) & (i < n) & (j > 0) & (j < n) & (k > 0) & (k < n)
    out = xyz.copy()
    d = rng.uniform(-amplitude, amplitude, size=xyz.shape) / n
    out[interior] += d[interior]
    return out


def x_sides(n: int):
    """Dirichlet data of the paper's conduction test (Section 2.5).

    T = 1 on the face x = 0 and T = 0 on x = 1, selected by lattice index.
    Returns ``bc_type`` int8 [V] (1 = Dirichlet), ``bc_value`` float64 [V] and
    ``side`` int8 [V] (1 = inflow face x = 0, 2 = outflow face x = 1).
    """
    i, _, _ = lattice_index(n)
    bc_type = ((i == 0) | (i == n)).astype(np.int8)
    bc_value = (i == 0).astype(np.float64)
    side = np.where(i == 0, 1, np.where(i == n, 2, 0)).astype(np.int8)
    return bc_type, bc_value, side


def delaunay_cube(n_interior: int, n_face: int, seed: int):
    """Delaunay tetrahedralisation of random points in the unit cube (stand-in
    for the paper's TetGen Delaunay meshes, Section 2.2).

    Points: the 8 corners, ``n_face`` uniform points on each of the 6 faces
    (coordinates exactly 0 or 1 on the face's axis) and ``n_interior`` uniform
    interior points, from PCG64(seed).  Tets from scipy's Qhull Delaunay;
    simplices of volume <= 1e-12 (flat ones Qhull can leave on coplanar hull
    points) are dropped, and every tet is ordered to positive volume.
    Returns ``xyz`` float64 [V,3] and ``tets`` int32 [T,4].
    """
    import scipy.spatial
    rng = np.random.Generator(np.random.PCG64(seed))
    pts = [np.array(list(itertools.product((0.0, 1.0), repeat=3)))]
    for ax in range(3):
        for side in (0.0, 1.0):
            p = rng.random((n_face, 3))
            p[:, ax] = side
            pts.append(p)
    pts.append(rng.random((n_interior, 3)))
    xyz = np.concatenate(pts)
    tets = scipy.spatial.Delaunay(xyz).simplices.astype(np.int64)
    p = xyz[tets]
    vol = np.einsum("ij,ij->i", np.cross(p[:, 1] - p[:, 0], p[:, 2] - p[:, 0]), p[:, 3] - p[:, 0]) / 6.0
    keep = np.abs(vol) > 1e-12
    tets, vol = tets[keep], vol[keep]
    tets[vol < 0] = tets[vol < 0][:, [0, 2, 1, 3]]
    return xyz, np.ascontiguousarray(tets, dtype=np.int32)


def delaunay_lattice(n: int, jitter: float, seed: int):
    """Delaunay tetrahedralisation of a jittered lattice of the unit cube (a quality mesh, the
    closer stand-in for the paper's TetGen meshes: few slivers, near-uniform sizes).

    Points: the (n+1)^3 lattice x = (i, j, k)/n with interior points moved as in
    ``jitter_interior(..., n, jitter, seed)`` (boundary points stay on the lattice, so the cube's
    faces are planes of points).  Tets from scipy's Qhull Delaunay; simplices of volume <= 1e-12
    (flat ones on coplanar hull points) dropped, every tet ordered to positive volume.
    Returns ``xyz`` float64 [V,3] and ``tets`` int32 [T,4].
    """
    import scipy.spatial
    xyz = jitter_interior(kuhn_cube(n)[0], n, jitter, seed)
    tets = scipy.spatial.Delaunay(xyz).simplices.astype(np.int64)
    p = xyz[tets]
    vol = np.einsum("ij,ij->i", np.cross(p[:, 1] - p[:, 0], p[:, 2] - p[:, 0]), p[:, 3] - p[:, 0]) / 6.0
    keep = np.abs(vol) > 1e-12
    tets, vol = tets[keep], vol[keep]
    tets[vol < 0] = tets[vol < 0][:, [0, 2, 1, 3]]
    return xyz, np.ascontiguousarray(tets, dtype=np.int32)


def x_faces(xyz: np.ndarray):
    """The conduction test's Dirichlet data on any mesh of the unit cube: T = 1 on
    x = 0 and T = 0 on x = 1 (vertices exactly on those planes); same outputs as
    ``x_sides``."""
    x = np.asarray(xyz)[:, 0]
    bc_type = ((x == 0.0) | (x == 1.0)).astype(np.int8)
    bc_value = (x == 0.0).astype(np.float64)
    side = np.where(x == 0.0, 1, np.where(x == 1.0, 2, 0)).astype(np.int8)
    return bc_type, bc_value, side


def lognormal_kappa(E: int, sigma: float, seed: int, mu: float = 0.0) -> np.ndarray:
    """kappa_e = exp(mu + sigma Z_e), Z_e ~ N(0,1) drawn in canonical edge order."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return np.exp(mu + sigma * rng.standard_normal(E))


def penny_cracks(N: int, seed: int, rmin: float = 0.02, rmax: float = 0.08) -> np.ndarray:
    """N discs as rows (cx, cy, cz, nx, ny, nz, r).

    Centres U[0,1]^3, then normals as normalised N(0, I3) draws, then radii
    U[rmin, rmax], drawn in that order from one PCG64 stream.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    c = rng.uniform(0.0, 1.0, size=(N, 3))
    nrm = rng.standard_normal((N, 3))
    nrm /= np.sqrt((nrm * nrm).sum(axis=1))[:, None]
    r = rng.uniform(rmin, rmax, size=N)
    return np.concatenate([c, nrm, r[:, None]], axis=1).astype(np.float64)


def grown_radii(cracks: np.ndarray, step: int, rate: float = 1.02) -> np.ndarray:
    """Discs of crack-growth step s: every radius multiplied by ``rate`` s times."""
    out = cracks.copy()
    for _ in range(step):
        out[:, 6] = out[:, 6] * rate
    return out


@dataclass
class ServeRequestSpec:
    """One request of a serving stream: mesh size, crack count, seeds, arrival time."""

    index: int
    n: int
    n_cracks: int
    kappa_seed: int
    crack_seed: int
    arrival_s: float


def serving_trace(count: int, seed: int, rate_per_s: float, nmin: int = 24, nmax: int = 96,
                  cmax: int = 400) -> list:
    """Poisson arrival trace: n ~ U{nmin..nmax}, cracks ~ U{0..cmax}, exponential gaps."""
    rng = np.random.Generator(np.random.PCG64(seed))
    ns = rng.integers(nmin, nmax + 1, size=count)
    cs = rng.integers(0, cmax + 1, size=count)
    gaps = rng.exponential(1.0 / rate_per_s, size=count) if rate_per_s > 0 else np.zeros(count)
    t = np.cumsum(gaps) - gaps[0]
    return [ServeRequestSpec(q, int(ns[q]), int(cs[q]), 1000 + 2 * q, 1001 + 2 * q, float(t[q]))
            for q in range(count)]
