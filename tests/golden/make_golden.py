"""Write the stored expected values of the full-size parity tests (calls only the oracle).

Workload "kuhn128_lognormal1_cracks200": unit cube, 128^3 Kuhn cells, per-edge
kappa = exp(Z) (sigma 1, seed 1, canonical edge order), 200 penny cracks
(seed 2, radius U[0.02, 0.08]), T = 1 on x = 0 and T = 0 on x = 1.

Stored: mesh counts, the full set of cut edges and pinned vertices
(bit-exact targets), *1 on a seeded sample of edges, the reference
solution x* (oracle PCG to 1e-14 relative residual or stagnation) on a
seeded sample S of 65,536 vertices with its norms, k_eff / Q_in / Q_out /
energy at x*, and the error against x* of the oracle's own solves stopped at
1e-10 (Jacobi PCG in FP64, and FP64 iterative refinement around FP32 Jacobi
PCG, the mixed-precision method), over the whole vector and on S
(||x_S - x*_S||_2 / ||x*_S||_2, the measure the parity tests apply to the
GPU's solution).

    python tests/golden/make_golden.py [n]      (n = 128 by default; minutes of CPU)
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle as O  # noqa: E402
import workloads as W  # noqa: E402


def main(n=128):
    t0 = time.time()
    name = f"kuhn{n}_lognormal1_cracks200"
    xyz, tets = W.kuhn_cube(n)
    V = len(xyz)
    E = O.edges_of(tets, V)
    print(f"[{time.time()-t0:.0f}s] edges {len(E)}", flush=True)
    kappa = W.lognormal_kappa(len(E), 1.0, 1)
    cracks = W.penny_cracks(200, 2)
    cut = O.crack_cut(xyz, E, cracks)
    print(f"[{time.time()-t0:.0f}s] cut {int(cut.sum())}", flush=True)
    star = O.hodge1(xyz, tets, E, kappa=kappa, cut=cut)
    print(f"[{time.time()-t0:.0f}s] star1", flush=True)
    L, _ = O.assemble(V, E, star)
    bt, bv, side = W.x_sides(n)
    A, b, pinned = O.apply_bc(L, bt, bv, E, star)
    print(f"[{time.time()-t0:.0f}s] system, pinned {int(pinned.sum())}", flush=True)
    ref = O.pcg(A, b, precond="jacobi", tol=1e-14, stagnation=50)
    print(f"[{time.time()-t0:.0f}s] reference: {ref.iterations} its, rel res {ref.rel_residual:.2e}", flush=True)
    loose = O.pcg(A, b, precond="jacobi", tol=1e-10)
    err_loose = float(np.linalg.norm(loose.x - ref.x) / np.linalg.norm(ref.x))
    print(f"[{time.time()-t0:.0f}s] 1e-10 solve: {loose.iterations} its, error vs x* {err_loose:.2e}", flush=True)
    x_ir, ir_outer, ir_inner, ir_res = O.iterative_refinement(A, b, tol=1e-10, inner_tol=1e-5, precond="jacobi",
                                                              adaptive_final=True)
    print(f"[{time.time()-t0:.0f}s] mixed refinement: inner {ir_inner}, residual {ir_res:.2e}", flush=True)
    f = O.flux_effective_conductivity(ref.x, E, star, side)
    rng = np.random.Generator(np.random.PCG64(12345))
    e_sample = np.sort(rng.choice(len(E), size=4096, replace=False))
    v_sample = np.sort(rng.choice(V, size=min(V, 65536), replace=False))
    x_s = ref.x[v_sample]
    err_loose_s = float(np.linalg.norm(loose.x[v_sample] - x_s) / np.linalg.norm(x_s))
    np.savez_compressed(
        os.path.join(HERE, f"{name}.npz"),
        cut_edges=np.nonzero(cut)[0].astype(np.int64),
        pinned=np.nonzero(pinned)[0].astype(np.int64),
        edge_sample=e_sample,
        edge_sample_lohi=E[e_sample],
        star1_sample=star[e_sample],
        vertex_sample=v_sample,
        x_sample=x_s,
        b_sample=b[v_sample],
    )
    meta = {
        "workload": name,
        "n": n,
        "V": int(V),
        "T": int(len(tets)),
        "E": int(len(E)),
        "nnz": int(L.nnz),
        "n_cut": int(cut.sum()),
        "n_pinned": int(pinned.sum()),
        "x_norm": float(np.linalg.norm(ref.x)),
        "b_norm": float(np.linalg.norm(b)),
        "ref_iterations": int(ref.iterations),
        "ref_rel_residual": float(ref.rel_residual),
        "loose_iterations": int(loose.iterations),
        "loose_error_vs_ref": err_loose,
        "x_sample_norm": float(np.linalg.norm(x_s)),
        "loose_sample_error_vs_ref": err_loose_s,
        "ir_inner_iterations": [int(k) for k in ir_inner],
        "ir_rel_residual": float(ir_res),
        "ir_sample_error_vs_ref": float(np.linalg.norm(x_ir[v_sample] - x_s) / np.linalg.norm(x_s)),
        "k_eff": f["k_eff"],
        "q_in": f["q_in"],
        "q_out": f["q_out"],
        "energy": f["energy"],
        "seconds": time.time() - t0,
    }
    with open(os.path.join(HERE, f"{name}.json"), "w") as fh:
        json.dump(meta, fh, indent=1)
    print(json.dumps(meta, indent=1))


if __name__ == "__main__":
    main(int(sys.argv[1]) if len(sys.argv) > 1 else 128)
