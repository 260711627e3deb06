"""Oracle solvers: preconditioned CG, Jacobi and FSAI preconditioners, iterative refinement (test infrastructure).

The paper solves its (mixed) system with PETSc's FGMRES and a ParaSails
sparse-approximate-inverse preconditioner (Section 2.3).  The vertex system
here is symmetric positive definite, so the oracle uses the textbook
preconditioned conjugate-gradient recurrence (Hestenes-Stiefel; Saad,
Iterative Methods for Sparse Linear Systems, Algorithm 9.1), and as the
sparse-approximate-inverse preconditioner the factored form of Kolotilina
and Yeremin (FSAI): G lower triangular on a fixed pattern, M^-1 = G^T G.
"""
from dataclasses import dataclass, field

import numpy as np
import scipy.sparse as sp


@dataclass
class PCGResult:
    x: np.ndarray
    iterations: int
    converged: bool
    breakdown: bool
    rel_residual: float
    history: list = field(default_factory=list)


def _norm(v):
    return float(np.sqrt(np.dot(v, v)))


def pcg(A, b, x0=None, precond=None, tol=1e-10, max_iters=100000, stagnation=None, history=False):
    """Preconditioned CG on SPD A.

    precond: None (identity), "jacobi", or a callable r -> z.
    Stops when the recursive residual satisfies ||r|| <= tol ||b||, then
    recomputes b - A x and continues from it if it is still above tol.
    ``stagnation``: also stop once the best residual has not improved for
    that many iterations (used for the tight reference solve).
    """
    dt = A.dtype
    b = np.asarray(b, dtype=dt)
    if precond is None:
        M = lambda r: r.copy()  # noqa: E731
    elif precond == "jacobi":
        inv = (1.0 / A.diagonal()).astype(dt)
        M = lambda r: inv * r  # noqa: E731
    else:
        M = precond
    x = np.zeros_like(b) if x0 is None else np.array(x0, dtype=dt)
    bnorm = _norm(b)
    if bnorm == 0.0:
        return PCGResult(np.zeros_like(b), 0, True, False, 0.0)
    r = b - A @ x
    z = M(r)
    p = z.copy()
    rho = float(np.dot(r, z))
    it, restarts, best, since_best = 0, 0, np.inf, 0
    hist = []
    breakdown = False
    while True:
        rn = _norm(r)
        if history:
            hist.append(rn / bnorm)
        if rn <= tol * bnorm:
            rt = b - A @ x
            if _norm(rt) <= tol * bnorm or restarts >= 20:
                break
            restarts += 1
            r = rt
            z = M(r)
            p = z.copy()
            rho = float(np.dot(r, z))
            continue
        if it >= max_iters:
            break
        if stagnation is not None:
            if rn < best:
                best, since_best = rn, 0
            else:
                since_best += 1
                if since_best >= stagnation:
                    break
        q = A @ p
        pq = float(np.dot(p, q))
        if not np.isfinite(pq) or pq <= 0.0:
            breakdown = True
            break
        alpha = rho / pq
        x = x + dt.type(alpha) * p
        r = r - dt.type(alpha) * q
        z = M(r)
        rho_new = float(np.dot(r, z))
        beta = rho_new / rho
        rho = rho_new
        p = z + dt.type(beta) * p
        it += 1
    rel = _norm(b.astype(np.float64) - A.astype(np.float64) @ x.astype(np.float64)) / float(bnorm)
    return PCGResult(x, it, rel <= tol, breakdown, rel, hist)


def fsai_pattern(A):
    """Lower triangle (diagonal included) of A's stored pattern, explicit zeros included."""
    A = sp.csr_matrix(A)
    out = []
    for i in range(A.shape[0]):
        cols = A.indices[A.indptr[i]:A.indptr[i + 1]]
        out.append(np.sort(cols[cols <= i]))
    return out


def fsai_factor(A, pattern=None):
    """FSAI factor G (CSR, lower triangular) with G A G^T having unit diagonal.

    For each row i with pattern S_i (ascending, i last): solve the dense SPD
    system A[S_i, S_i] y = e_i and set row i of G to y / sqrt(y_i).
    """
    A = sp.csr_matrix(A, dtype=np.float64)
    if pattern is None:
        pattern = fsai_pattern(A)
    rows = [dict(zip(A.indices[A.indptr[i]:A.indptr[i + 1]], A.data[A.indptr[i]:A.indptr[i + 1]]))
            for i in range(A.shape[0])]
    indptr = [0]
    indices = []
    data = []
    for i, S in enumerate(pattern):
        m = len(S)
        sub = np.array([[rows[a].get(c, 0.0) for c in S] for a in S])
        e = np.zeros(m)
        e[-1] = 1.0
        y = np.linalg.solve(sub, e)
        g = y / np.sqrt(y[-1])
        indices.extend(int(c) for c in S)
        data.extend(g.tolist())
        indptr.append(len(indices))
    return sp.csr_matrix((np.array(data), np.array(indices), np.array(indptr)), shape=A.shape)


def fsai_apply(G, GT=None):
    """Preconditioner callable z = G^T (G r)."""
    GT = G.T.tocsr() if GT is None else GT
    return lambda r: GT @ (G @ r)


def iterative_refinement(A, b, tol=1e-10, inner_tol=1e-5, precond="jacobi", adaptive_final=True,
                         max_outer=50, inner_max_iters=100000):
    """FP64 iterative refinement around FP32 PCG inner solves.

    Loop: r = b - A x in FP64; stop when ||r|| <= tol ||b||; solve
    A32 c = r/||r|| in FP32 PCG to the inner tolerance; x += ||r|| c in FP64.
    With ``adaptive_final`` the inner tolerance is max(inner_tol,
    0.5 tol ||b|| / ||r||), i.e. the last correction only has to close the
    remaining gap.  ``precond``: "jacobi" or "fsai" (factor computed in FP64,
    applied in FP32).
    Returns (x, outer_iterations, inner_iterations_list, rel_residual).
    """
    A = sp.csr_matrix(A, dtype=np.float64)
    A32 = A.astype(np.float32)
    if precond == "fsai":
        G = fsai_factor(A).astype(np.float32)
        M = fsai_apply(G)
    else:
        M = "jacobi"
    b = np.asarray(b, dtype=np.float64)
    bnorm = _norm(b)
    x = np.zeros_like(b)
    inner = []
    outer = 0
    if bnorm == 0.0:
        return x, 0, inner, 0.0
    while outer < max_outer:
        r = b - A @ x
        rn = _norm(r)
        if rn <= tol * bnorm:
            break
        itol = inner_tol
        if adaptive_final:
            itol = max(inner_tol, 0.5 * tol * bnorm / rn)
        res = pcg(A32, (r / rn).astype(np.float32), precond=M, tol=itol, max_iters=inner_max_iters)
        inner.append(res.iterations)
        x = x + rn * res.x.astype(np.float64)
        outer += 1
    rel = _norm(b - A @ x) / bnorm
    return x, outer, inner, rel
